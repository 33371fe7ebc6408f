// Internal declarations shared by the HIP kernels and the host side of
// libccpt.  Nothing here is part of the public ABI (include/ccpt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ccpt.h"

namespace ccpt {

// Device-side descriptor of one frame of a launch group (32 bytes).
struct FrameDesc {
  const void* data;   // frame pixels (device)
  const void* rspec;  // conj F[B] of its reference, N x (N/2+1), row-major:
                      // float2, or double2 in FP64 mode
  int pitch;          // elements between row starts
  int dtype;          // ccpt_dtype
  int out_idx;        // index into the caller's result array
  int ref_id;         // reference index
};

// Per-frame scratch passed between the kernels of one chunk.  It lives in a
// buffer of its own that starts in the initial state (below) and is returned
// to it by the Newton kernel, the last of a chunk, for every frame: no reset
// launch is needed per chunk.
struct FrameState {
  unsigned long long peak_key;    // integer-lag maximum: value key << 32 | ~flat index
  unsigned long long grid_key;    // upsampled-grid maximum, same encoding
  unsigned long long second_key;  // runner-up of the integer-lag correlation, same
                                  // encoding (0 until set; FP32 and split paths)
  unsigned amin, amax;            // order-preserving keys of min/max of A
  unsigned flags;                 // CCPT_ST_NONFINITE; CCPT_ST_NEAR_TIE (FP64 mode)
  unsigned xmax;                  // largest |Re|, |Im| of the cross-power spectrum
                                  // without its DC term, as float bits (the 256x256
                                  // one-kernel correlation; 0 elsewhere)
};

// FP64 mode: best correlation value of one row block of a frame and its
// row-major index (ties to the lower index); reduced per frame before the
// upsampled DFT, since an FP64 value and an index do not fit one 64-bit key.
struct PeakCand {
  double v;     // best value of the block
  double v2;    // its runner-up value (a value equal to v at another index counts)
  unsigned idx;
  unsigned pad;
};

// Relative gap under which the two largest integer-lag correlation values
// count as a near tie (CCPT_ST_NEAR_TIE): v1 - v2 <= kNearTieRel |v1|.
constexpr double kNearTieRel = 1e-5;

// Scalar parameters of a launch group (passed by value to every kernel).
struct GroupParams {
  const FrameDesc* desc;  // descriptors of this group, frame i at desc[first + i]
  int first;              // first descriptor of the current chunk
  int count;              // frames in the current chunk
  float2* T;              // workspace [count][N][N/2+1] (FFT intermediate)
  float2* X;              // workspace [count][N][N/2+1] (cross-power spectrum)
  unsigned* Xb;           // split-precision copy of X for the matrix cores, or null:
                          // [count][2 (hi, lo)][N/2][xb_pitch(N)] words, one word =
                          // bf16 re | bf16 im << 16, ky contiguous, DC zeroed
  float2* Zc;             // split precision on the one-kernel 256 x 256 path (Xb
                          // null): [count][N], Z[ky] = X[ky, 0] + i X[ky, N/2] with
                          // the DC term dropped; the matrix DFT splits X itself
  FrameState* st;         // [count]
  ccpt_result* out;       // caller's results
  const float2* tw;       // exp(-2 pi i m / N), m < N
  int mode;               // CCPT_MODE_*
  float eps;              // CC-SN offset
  int u;                  // upsampling factor
  int M;                  // grid points per axis
  int c;                  // grid centre index
  int newton_iters;
  double half_window;     // Newton results farther than this from p fall back
  float* ypart;           // FP32 split-K partials for small launches, or null:
                          // [count][Mp/32][slices][32][N rounded up to 32]
  // FP64 mode (all null otherwise): T and X in double2, the per-row-block
  // peak candidates [count][N / row_block64(N)], twiddles in FP64
  double* nparts;         // Newton partial model coefficients of small launches, or
                          // null: [count][kNewtonParts][kNewtonCoef] doubles
  double eps64;           // CC-SN offset (FP64 mode)
  double2* T64;
  double2* X64;
  PeakCand* cand;
  const double2* tw64;
  int pairs_ok;           // every frame is uint16 or float32 with an even pitch and
                          // pixel pairs aligned to their size (one load per pair)
  int trans;              // 1: the frames are wider than tall and are processed as
                          // their transposes (NY x NX above is the transposed
                          // shape); integer-peak and grid indices keep the frame's
                          // own row-major order and the Newton stage writes the
                          // result in the frame's own axes
  int fused_min;          // 256x256: launches of at least this many frames take the
                          // one-kernel correlation (launch plan)
};

// Frame shapes of the kernels: square N x N for N in CCPT_FOR_SIZES, and the
// rectangles of CCPT_FOR_RECT, always held tall (NY = 2^k NX rows of NX
// columns) so that the half-spectrum axis of the real transforms is the short
// one; a wide frame is read transposed.  The twiddle table of a shape holds
// exp(-2 pi i m / NY), m < NY (NX divides NY).
#define CCPT_FOR_SIZES(X)                                                                           \
  X(16) X(18) X(24) X(32) X(36) X(48) X(54) X(64) X(72) X(96) X(108) X(128) X(144) X(162) X(192) \
      X(216) X(256) X(288) X(324) X(384) X(432) X(486) X(512)
#define CCPT_FOR_RECT(X) X(256, 128) X(512, 256) X(1024, 128)

// Launches of fewer than kNewtonSplitMax frames build the first Newton model
// over kNewtonParts blocks per frame (ky ranges), for latency.
constexpr int kNewtonSplitMax = 64;
constexpr int kNewtonParts = 8;
constexpr int kNewtonCoef = 36;  // Taylor coefficients of the degree-7 model

// Small FP32 launches (fewer than kSplitMaxBlocks row tiles in all, the
// default of the launch plan) split the Stage A contraction over kSplitSlices
// ky slices for latency; the split happens where the launch set-up hands the
// kernels a partials buffer (GroupParams::ypart).
constexpr int kSplitMaxBlocks = 128;
constexpr int kSplitSlices = 8;

// Row length (in words) of the split-precision spectrum rows: N rounded up to 32.
__host__ __device__ constexpr int xb_pitch(int n) { return (n + 31) / 32 * 32; }

// Rows per block of the FP64 row passes: 8 rows when they fit, else the
// largest divisor of N whose rows hold at most 1024 complex values.
__host__ __device__ constexpr int row_block64(int N) {
  if (N % 8 == 0 && 8 * (N / 2 + 1) <= 2100) return 8;
  int best = 1;
  for (int r = 1; r <= N; ++r)
    if (N % r == 0 && r * (N / 2) <= 1024) best = r;
  return best;
}

// Bytes per pixel of a ccpt_dtype.
__host__ __device__ constexpr int dtype_bytes(int dtype) {
  return dtype == CCPT_U16 ? 2 : dtype == CCPT_F64 ? 8 : 4;
}

// Order-preserving map float -> uint32 (a < b  <=>  key(a) < key(b)).
__host__ __device__ inline unsigned f2key(float v) {
  unsigned b;
  __builtin_memcpy(&b, &v, 4);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__host__ __device__ inline unsigned long long peak_key(float v, unsigned flat) {
  return ((unsigned long long)f2key(v) << 32) | (unsigned long long)(0xFFFFFFFFu - flat);
}

// The float value of a peak key (inverse of f2key on its high half).
__host__ __device__ inline float key_value(unsigned long long k) {
  const unsigned h = (unsigned)(k >> 32);
  const unsigned b = (h & 0x80000000u) ? (h & 0x7FFFFFFFu) : ~h;
  float v;
  __builtin_memcpy(&v, &b, 4);
  return v;
}

__host__ __device__ inline bool near_tie(double v1, double v2) {
  return v1 - v2 <= kNearTieRel * (v1 < 0.0 ? -v1 : v1);
}

__host__ __device__ inline unsigned key_index(unsigned long long k) {
  return 0xFFFFFFFFu - (unsigned)(k & 0xFFFFFFFFull);
}

// Tall-image coordinates (y, x) of the integer peak from its frame row-major
// index q (trans: the index in a wide frame of NX rows of NY pixels); an
// index that was never set (cannot happen for a tracked frame) reads as 0.
template <int NY, int NX>
__device__ __forceinline__ void peak_yx(unsigned q, int trans, int& y, int& x) {
  if (q >= (unsigned)(NY * NX)) q = 0;
  if (NY != NX && trans) {
    y = (int)(q % NY);
    x = (int)(q / NY);
  } else {
    y = (int)(q / NX);
    x = (int)(q % NX);
  }
}

// Frame row-major index of point (my, mx) of the M x M grid of the tall image.
__device__ __forceinline__ unsigned grid_index(int my, int mx, int M, bool trans) {
  return trans ? (unsigned)(mx * M + my) : (unsigned)(my * M + mx);
}

// The transpose flag of a kernel for frames of NY x NX: always false for
// square frames, so their kernels carry no code for it.
template <int NY, int NX>
__device__ __forceinline__ bool transposed(int trans) {
  return NY != NX && trans != 0;
}

// Optional callback around each kernel launch (stage id, begin/end), used
// to bracket launches with timing events.
struct Marker {
  void (*fn)(void* user, int stage, int begin) = nullptr;
  void* user = nullptr;
  void operator()(int stage, int begin) const {
    if (fn) fn(user, stage, begin);
  }
};

// ---- launchers (defined in the .hip files) -------------------------------

// Puts count frame states in the initial state (keys 0, amin all ones, amax
// and flags 0).
int launch_init_state(FrameState* st, int count, hipStream_t s);

// Stages 1-3: forward 2-D r2c FFT with the prologue, cross-power spectrum,
// inverse 2-D c2r FFT and the integer-peak search, for frames of the kernel
// shape ny x nx (g.trans: wide frames read transposed).
int launch_xcorr(int ny, int nx, const GroupParams& g, hipStream_t s, const Marker& mark);

// Forward 2-D r2c FFT of n images (pitch in elements; trans: each image is
// nx rows of ny and is read transposed) into spec [n][ny][nx/2+1]; weight:
// 0 = identity, 1 = CC-SN reference (-1/(E+eps)), 2 = CC-SN frame
// ((I+eps)^2).  If conj_out, stores the conjugate.
int launch_spectrum(int ny, int nx, const void* data, int dtype, int pitch, long img_stride,
                    int trans, int n, int weight, float eps, int conj_out, float2* T, float2* spec,
                    const float2* tw, hipStream_t s);

// The correlation stage of 256 x 256 frames (FP32 and split precision) in
// one kernel with the half spectrum held in registers: the same outputs as
// the three passes of launch_xcorr (X, Xb, the frame states), no T.
int launch_xcorr256(const GroupParams& g, hipStream_t s);

// Whether a launch of `count` frames of ny x nx takes that one-kernel path
// (pairs_ok as in GroupParams; fused_min from the launch plan);
// launch_xcorr and the launch set-up agree through it.  The kernel gives one
// frame to one CU, which pays only once the launch has about as many frames
// as the chip has CUs; smaller launches (the per-frame path) take the three
// passes, which spread a frame over about fifty blocks.  kFusedMinFrames is
// the default threshold.
constexpr int kFusedMinFrames = 128;
inline bool xcorr_fused(int ny, int nx, bool pairs_ok, int count, int fused_min) {
  return ny == 256 && nx == 256 && pairs_ok && count >= fused_min;
}

// FP64 mode: the same two calls with every FFT in FP64 (g.T64, g.X64,
// g.cand; the integer peak is left as per-row-block candidates).
int launch_xcorr64(int N, const GroupParams& g, hipStream_t s, const Marker& mark);
int launch_spectrum64(int N, const void* data, int dtype, int pitch, long img_stride, int n,
                      int weight, double eps, int conj_out, double2* T, double2* spec,
                      const double2* tw, hipStream_t s);

// Stage 4: upsampled matrix DFT around the integer peak and its maximum.
struct UpdftTables {
  const void* ky;    // Stage A operand table (layout depends on precision)
  const void* wb;    // Stage B operand table
  int Mp;            // padded grid size (multiple of 32)
  int precision;
  const void* kfold; // split precision, NX >= 256: folded K' table for every peak row
};

// Minimum row length NX of the wide split-precision kernel (and its folded table).
constexpr int kWideMinN = 256;
// 32-row grid tiles per block of the wide kernel.
constexpr int kWideMT = 5;

// Rows per plane of the folded table: Mp padded to whole blocks of kWideMT
// tiles (zero rows), so every block of the wide kernel runs all its tiles.
__host__ __device__ constexpr int kfold_rows(int Mp) {
  return (Mp / 32 + kWideMT - 1) / kWideMT * kWideMT * 32;
}

// Builds the folded split table [NY][2][rows][xb_pitch(NY)] words on the
// device for frames of NY rows (rows = kfold_rows(Mp); rows m >= M are zero).
int launch_build_kfold(unsigned* out, int N, int u, int M, int c, int rows, int f16, hipStream_t s);
int launch_updft(int ny, int nx, const GroupParams& g, const UpdftTables& t, hipStream_t s);

// FP64 mode: reduces the peak candidates, then the upsampled DFT in FP64 on
// the vector units; K [Mp][N] and W [N/2+1][Mp] are complex FP64 tables.
int launch_updft64(int N, const GroupParams& g, const double2* K, const double2* W, int Mp,
                   hipStream_t s);

// Stage 5: FP64 Newton refinement and the result record (from g.X64 when
// set, else from g.X).
int launch_newton(int ny, int nx, const GroupParams& g, double step_limit, hipStream_t s);

// Inverse 2-D c2r of n half spectra [n][ny][nx/2+1] into n float images of
// ny rows of nx (the tall layout of a rectangle) scaled by `scale` (T is
// scratch of the same size as the spectra).
int launch_inverse(int ny, int nx, const float2* spec, int n, float scale, float2* T, float* img,
                   const float2* tw, hipStream_t s);

// Forward 2-D r2c spectra (with the frame prologue of `mode`) of the frames of
// a descriptor chunk into spec [count][ny][nx/2+1], held tall (trans: wide
// frames read transposed).
int launch_frame_spectra(int ny, int nx, int trans, const FrameDesc* desc, int first, int count,
                         int mode, float eps, float2* T, float2* spec, const float2* tw,
                         hipStream_t s);

// Adjoint pieces (grad.hip).
int launch_grad_psi(int N, const FrameDesc* desc, int first, int count, const ccpt_result* fwd,
                    const double* g_d, const double* g_peak, const float2* FA, float2* QA,
                    float2* QB, hipStream_t s);
int launch_grad_frames(int N, const FrameDesc* desc, int first, int count, const float* img,
                       const long* goff, float* g_frames, int mode, float eps, hipStream_t s);
int launch_ref_accum(int N, const FrameDesc* desc, int first, int count, const float2* QB,
                     float2* const* acc, hipStream_t s);
int launch_grad_ref_chain(const float* img, const float* E, int nn, int mode, float eps,
                          float* out, hipStream_t s);
int launch_fisher_deriv(int N, const float2* F, float2* Dy, float2* Dx, hipStream_t s);
int launch_fisher_reduce(const float* dy, const float* dx, const void* mu, int dtype, int pitch,
                         int n, double* part, int nblocks, double* out, hipStream_t s);

// Offline reference (reference.hip): for a chunk of frames whose spectra
// are in F ([count][N][N/2+1]), multiplies each by the phases of its
// displacement (results fwd[desc.out_idx]), adds them in frame order to acc
// and counts the frames that tracked into cnt.
int launch_align_accumulate(int N, const FrameDesc* desc, int first, int count,
                            const ccpt_result* fwd, float2* F, float2* acc, unsigned* cnt,
                            hipStream_t s);
// Real-time reference update of Eq. 9 by one frame (spectrum F, result res):
// S <- a0 v + b1 S with v the frame shifted back (conjugated when conj_s);
// spectra held tall, ny x (nx/2+1) (trans: a wide frame, whose shift axes
// swap in that layout).
int launch_rt_update(int ny, int nx, int trans, const ccpt_result* res, const float2* F, float2* S,
                     float a0, float b1, int conj_s, hipStream_t s);
// img *= scale / *cnt (zeros when *cnt == 0).
int launch_scale_by_count(float* img, int nn, float scale, const unsigned* cnt, hipStream_t s);

// Static device scratch of ccpt_track_batch_static (scratch.hip): its size,
// the once-per-device set-up (call with `device` current; 0 on success) and
// the device address kept by the set-up (null before it).
constexpr size_t kScratchBytes = (size_t)64 << 20;
int scratch_setup(int device);
void* scratch_ptr(int device);

// Fills bytes of device memory with zero using a kernel (graph-safe).
int launch_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace ccpt
