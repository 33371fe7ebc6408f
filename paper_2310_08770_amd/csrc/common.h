// Internal declarations shared by the HIP kernels and the host side of
// libccpt.  Nothing here is part of the public ABI (include/ccpt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ccpt.h"

namespace ccpt {

// Device-side descriptor of one frame of a launch group (32 bytes).
struct FrameDesc {
  const void* data;     // frame pixels (device)
  const float2* rspec;  // conj F[B] of its reference, N x (N/2+1), row-major
  int pitch;            // elements between row starts
  int dtype;            // CCPT_U16 / CCPT_F32
  int out_idx;          // index into the caller's result array
  int ref_id;           // reference index
};

// Per-frame scratch kept in the workspace between the kernels of one chunk.
struct FrameState {
  unsigned long long peak_key;  // integer-lag maximum: value key << 32 | ~flat index
  unsigned long long grid_key;  // upsampled-grid maximum, same encoding
  unsigned amin, amax;          // order-preserving keys of min/max of A
  unsigned flags;               // CCPT_ST_NONFINITE
  unsigned pad;
};

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
};

// Row length (in words) of the split-precision spectrum rows: N rounded up to 32.
__host__ __device__ constexpr int xb_pitch(int n) { return (n + 31) / 32 * 32; }

// Order-preserving map float -> uint32 (a < b  <=>  key(a) < key(b)).
__host__ __device__ inline unsigned f2key(float v) {
  unsigned b;
  __builtin_memcpy(&b, &v, 4);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__host__ __device__ inline unsigned long long peak_key(float v, unsigned flat) {
  return ((unsigned long long)f2key(v) << 32) | (unsigned long long)(0xFFFFFFFFu - flat);
}

__host__ __device__ inline unsigned key_index(unsigned long long k) {
  return 0xFFFFFFFFu - (unsigned)(k & 0xFFFFFFFFull);
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

// Stage 0-3: state reset, forward 2-D r2c FFT with the prologue, cross-power
// spectrum, inverse 2-D c2r FFT and the integer-peak search.
int launch_xcorr(int N, const GroupParams& g, hipStream_t s, const Marker& mark);

// Forward 2-D r2c FFT of n images (pitch in elements) into spec
// [n][N][N/2+1]; weight: 0 = identity, 1 = CC-SN reference (-1/(E+eps)),
// 2 = CC-SN frame ((I+eps)^2).  If conj_out, stores the conjugate.
int launch_spectrum(int N, const void* data, int dtype, int pitch, long img_stride, int n,
                    int weight, float eps, int conj_out, float2* T, float2* spec,
                    const float2* tw, hipStream_t s);

// Stage 4: upsampled matrix DFT around the integer peak and its maximum.
struct UpdftTables {
  const void* ky;    // Stage A operand table (layout depends on precision)
  const void* wb;    // Stage B operand table
  int Mp;            // padded grid size (multiple of 32)
  int precision;
};
int launch_updft(int N, const GroupParams& g, const UpdftTables& t, hipStream_t s);

// Stage 5: FP64 Newton refinement and the result record.
int launch_newton(int N, const GroupParams& g, double step_limit, hipStream_t s);

// Inverse 2-D c2r of n half spectra [n][N][N/2+1] into n N x N float images
// scaled by `scale` (T is scratch of the same size as the spectra).
int launch_inverse(int N, const float2* spec, int n, float scale, float2* T, float* img,
                   const float2* tw, hipStream_t s);

// Forward 2-D r2c spectra (with the frame prologue of `mode`) of the frames of
// a descriptor chunk into spec [count][N][N/2+1].
int launch_frame_spectra(int N, const FrameDesc* desc, int first, int count, int mode, float eps,
                         float2* T, float2* spec, const float2* tw, hipStream_t s);

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

// Fills bytes of device memory with zero using a kernel (graph-safe).
int launch_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace ccpt
