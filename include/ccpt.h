/*
 * ccpt.h -- cross-correlation particle tracking on AMD MI355X (gfx950).
 *
 * C ABI of the per-frame displacement estimator of Werneck et al.,
 * "Cross-correlation image analysis for real-time single particle
 * tracking" (arXiv 2310.08770).
 *
 * Problem (Sec. II, Eq. 1): given a reference image E and a frame I, find
 * the displacement minimising chi^2 between the translated frame and E
 * under periodic boundaries.  For uniform noise (CC-U, Eq. 2-4) this is the
 * maximum of the circular cross-correlation F^-1[F[I] conj F[E]]; for shot
 * noise (CC-SN, Eq. 5-7) it is the extremum of the correlation of (I+eps)^2
 * with 1/(E+eps).  The integer maximum is refined on a 1.5-pixel window
 * sampled at 1.5u points per axis by a matrix-multiply DFT (Sec. III, first
 * paragraph), whose maximum is the paper's sub-pixel estimate; the library
 * then refines it in FP64 by Newton steps on the band-limited correlation.
 *
 * Conventions used throughout:
 *  - pixels, (y, x) order, row-major images with a row pitch in elements;
 *  - a result d means frame(r) ~ ref(r - d) (the paper's r0 is -d);
 *  - CC-SN uses A = (I+eps)^2 and B = -1/(E+eps): the chi^2 minimum of
 *    Eq. 6 is the maximum of this correlation;
 *  - even N only: the Nyquist bin is interpolated as cos(pi s);
 *  - grid: M = ceil(window*u) points per axis, centre index floor(M/2),
 *    offsets (m - floor(M/2))/u; ties go to the lowest row-major index;
 *  - integer lags are reported in [-N/2, N/2).
 *
 * Supported shapes (ny rows x nx columns): square N x N frames with
 * N = 2^a 3^b, a >= 1, 16 <= N <= 512, and the rectangles of the paper's
 * Table I, 256x128, 512x256 and 1024x128, in either orientation (the
 * longer side as rows or as columns).  Rectangles are tracked by
 * ccpt_set_reference / ccpt_track_batch in FP32 and BF16X2 precision; the
 * adjoint, the Fisher information, the reference updates and the FP64
 * precision take square frames only.  Other shapes, and rectangles where
 * only squares are taken, return CCPT_E_UNSUPPORTED.
 *
 * Rectangles: the Nyquist conventions above apply per axis (N/2 of that
 * axis); integer lags are in [-ny/2, ny/2) x [-nx/2, nx/2); C is
 * normalised by 1/(ny nx); ties go to the lowest row-major index of the
 * frame as given.
 *
 * Memory: every image/frame pointer, `out`, the gradient inputs and
 * outputs are DEVICE pointers owned by the caller.  The small descriptor
 * arrays (ccpt_image, ccpt_roi) are HOST arrays, read during the call.
 * The context owns reference spectra, DFT tables, workspaces, captured
 * graphs and the tuning table.
 *
 * Streams: `stream` is a hipStream_t (NULL = the null stream).  Track and
 * grad calls are stream-ordered and return before the GPU work finishes;
 * create, destroy, set_reference and fisher may allocate and synchronise.
 * A context is not thread-safe: use one context per host thread/stream.
 *
 * Errors: every call returns CCPT_OK (0) or a negative code; nothing
 * throws across the ABI.  ccpt_last_error() returns the message of the
 * last failing call on a context.  Per-frame conditions are reported in
 * ccpt_result.status bits, never as call failures.
 */
#ifndef CCPT_H
#define CCPT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------- */
#define CCPT_OK 0
#define CCPT_E_INVALID (-1)         /* bad pointer, size, count, option or id */
#define CCPT_E_UNSUPPORTED (-2)     /* frame shape outside the supported set */
#define CCPT_E_NOREF (-3)           /* no reference set / ref_id out of range */
#define CCPT_E_HIP (-4)             /* HIP runtime error (see ccpt_last_error) */
#define CCPT_E_NONPOSITIVE_REF (-5) /* CC-SN reference with E + eps <= 0 */
#define CCPT_E_NOMEM (-6)           /* device or host allocation failed */

/* ---- per-frame status bits (ccpt_result.status) ---------------------- */
#define CCPT_ST_NONFINITE 1u       /* NaN/Inf pixel: d, d_grid, peak are NaN */
#define CCPT_ST_FLAT 2u            /* constant frame: everything is zero */
#define CCPT_ST_NEAR_TIE 4u        /* the two largest integer-lag correlation
                                      values differ by at most 1e-5 of the
                                      largest's magnitude (p is then decided
                                      by rounding; it is still the lowest-index
                                      maximum of the computed correlation) */
#define CCPT_ST_NEWTON_FALLBACK 8u /* Hessian not negative definite, or a step
                                      longer than 1/u (FP64 precision) or
                                      than half the window (FP32, BF16X2,
                                      whose grid maximum can sit well off
                                      the true one where the correlation is
                                      flat): d = d_grid */
#define CCPT_ST_WINDOW_EXIT 16u    /* Newton left the 0.75-px half window:
                                      d = d_grid */

/* ---- options ---------------------------------------------------------- */
enum ccpt_mode { CCPT_MODE_CCU = 0, CCPT_MODE_CCSN = 1 };

/* arithmetic of the correlation and the upsampled matrix DFT (the Newton
   refinement is FP64 in every mode) */
enum ccpt_precision {
  CCPT_PREC_FP32 = 0,   /* FP32 FFTs, FP32 matrix cores */
  CCPT_PREC_BF16X2 = 1, /* FP32 FFTs; DFT operands split into bf16 hi + lo,
                           three bf16 products accumulated in FP32 */
  CCPT_PREC_FP16X2 = 2, /* FP32 FFTs; DFT operands split into fp16 hi + lo
                           (about 22 bits) under power-of-two scales, three
                           fp16 products accumulated in FP32.  256 x 256
                           frames of uint16 or float32 with an even pitch
                           only (the one-kernel correlation): other shapes
                           and pixel layouts give CCPT_E_UNSUPPORTED */
  CCPT_PREC_FP64 = 3    /* FFTs, cross-power spectrum, integer peak and the
                           upsampled DFT all in FP64 (vector units): the
                           accuracy mode, for agreement with an FP64
                           definition well below 1e-9 px */
};

/* pixel types: uint16 (12-bit cameras), float32, float64 */
enum ccpt_dtype { CCPT_U16 = 0, CCPT_F32 = 1, CCPT_F64 = 2 };

#define CCPT_FLAG_GRAPH 1   /* capture each batch shape once in a hipGraph and
                               replay it on later calls */
#define CCPT_FLAG_PROFILE 2 /* bracket every kernel launch with HIP events on the
                               call's stream (measurement; disables graphs and
                               CCPT_FLAG_STREAMS) */
#define CCPT_FLAG_STREAMS 4 /* run the chunks of a batch alternately on the call's
                               stream and a second stream owned by the context
                               (default priority), forked from and joined back
                               into the call's stream, so one chunk's matrix-core
                               work overlaps the next chunk's FFTs; results are
                               bit-identical, the workspace doubles */

/* stage ids of ccpt_stage_times */
enum ccpt_stage {
  CCPT_STAGE_INIT = 0,     /* reserved (frame states are reset by the Newton stage) */
  CCPT_STAGE_ROWS_FWD = 1, /* prologue + row r2c FFTs */
  CCPT_STAGE_COLS = 2,     /* column FFTs, cross-power spectrum, inverse column FFTs */
  CCPT_STAGE_ROWS_INV = 3, /* row c2r FFTs + integer peak */
  CCPT_STAGE_UPDFT = 4,    /* upsampled matrix DFT + grid maximum */
  CCPT_STAGE_NEWTON = 5,   /* FP64 Newton refinement + result */
  CCPT_STAGE_GRAD = 6,     /* all kernels of ccpt_track_grad */
  CCPT_STAGE_XCORR = 7,    /* stages 1-3 in one kernel (256 x 256 frames) */
  CCPT_NUM_STAGES = 8
};

typedef struct ccpt_options {
  int mode;         /* ccpt_mode */
  double eps;       /* CC-SN offset added to frames and reference (Eq. 6);
                       Sec. IV suggests 200 x the noise gain; ignored by CC-U */
  int upsample;     /* u >= 1: grid step 1/u px (Sec. III) */
  double window;    /* side of the upsampled square in px; the paper uses 1.5 */
  int precision;    /* ccpt_precision */
  int newton_iters; /* 0..8 FP64 Newton steps after the grid (0 = grid only) */
  int flags;        /* CCPT_FLAG_* */
} ccpt_options;

/* fills `o` with the paper's defaults: CC-U, eps 200, u 100, window 1.5,
   FP32, 3 Newton steps, no flags */
void ccpt_default_options(ccpt_options* o);

/* an image in device memory */
typedef struct ccpt_image {
  const void* data; /* device pointer, row-major */
  int ny, nx;       /* rows, columns */
  int pitch;        /* elements between row starts (>= nx) */
  int dtype;        /* ccpt_dtype */
} ccpt_image;

/* one frame or region of interest to track */
typedef struct ccpt_roi {
  const void* data; /* device pointer, row-major */
  int ny, nx;
  int pitch;  /* elements between row starts (>= nx) */
  int dtype;  /* ccpt_dtype */
  int ref_id; /* reference index given to ccpt_set_reference */
} ccpt_roi;

/* one tracking result, 72 bytes, written to device memory */
typedef struct ccpt_result {
  double d[2];     /* refined displacement (y, x), px */
  double peak;     /* C(d) = band-limited correlation at d, normalised by 1/(ny nx) */
  double hess[3];  /* d2C/dy2, d2C/dydx, d2C/dx2 at d (used by the adjoint) */
  float d_grid[2]; /* maximum of the upsampled grid (the paper's estimate) */
  int p[2];        /* integer-lag correlation maximum (y, x) */
  unsigned status; /* CCPT_ST_* bits */
  unsigned reserved;
} ccpt_result;

typedef struct ccpt_ctx ccpt_ctx;

/* Creates a context on HIP device `device`.  `opts` may be NULL (defaults).
   Returns CCPT_E_INVALID for out-of-range options, CCPT_E_HIP if the
   device cannot be used. */
int ccpt_create(ccpt_ctx** out, int device, const ccpt_options* opts);

/* Frees everything the context owns (after synchronising its work). */
void ccpt_destroy(ccpt_ctx* ctx);

/* Sets the reference images (Sec. II: E; Sec. III for its role) and
   replaces any earlier set.  For each reference the library forms
   B = E (CC-U) or B = -1/(E+eps) (CC-SN, Eq. 7), transforms it and keeps
   conj F[B] resident.  References may have different sizes; ids are
   0..n_refs-1.  Synchronises `stream`.  Errors: CCPT_E_INVALID,
   CCPT_E_UNSUPPORTED, CCPT_E_NONPOSITIVE_REF (CC-SN, any E + eps <= 0). */
int ccpt_set_reference(ccpt_ctx* ctx, const ccpt_image* refs, int n_refs, void* stream);

/* Tracks n frames (Sec. II Eq. 4/7 and Sec. III): for each roi i computes
   the correlation with reference roi[i].ref_id, its integer maximum, the
   upsampled-grid maximum and the FP64 Newton refinement, and writes
   out[i].  Frames of different sizes may be mixed; each must match the
   size of its reference.  `rois` is a host array; `out` is a device array
   of n results.  A call with n = 1 is the plain per-frame path.  Returns
   before the GPU finishes.  Errors: CCPT_E_INVALID, CCPT_E_UNSUPPORTED,
   CCPT_E_NOREF, CCPT_E_HIP, CCPT_E_NOMEM. */
int ccpt_track_batch(ccpt_ctx* ctx, const ccpt_roi* rois, int n, ccpt_result* out,
                     void* stream);

/* ccpt_track_batch for callers that cannot allocate device memory (tight
   serving loops, harnesses that forbid hipMalloc): the same tracking,
   results and errors, with every per-call buffer (descriptor table, frame
   states, spectra workspace) in the library's static device scratch of
   64 MiB per GPU instead of the context's grown workspace.  Calls no
   hipMalloc/hipFree.  `rois` is a host array, consumed before the call
   returns (its copy to the scratch is enqueued from pageable memory, so the
   call is not meant for stream capture).  Frames run in chunks that fit the
   scratch (about 80 frames of 256x256 in split precision); no graphs,
   second stream or profiling events; small launches take the unsplit
   kernels, so results equal ccpt_track_batch's to rounding (<= 1e-6 px;
   integer peak and grid index identical).  The context must already hold
   its references (set by ccpt_set_reference, which allocates).  All calls
   on one GPU share its scratch, which keeps the last call's contents: calls
   that overlap on one GPU (other streams, threads or contexts) race and
   must be ordered by the caller.  n <= CCPT_STATIC_MAX_ROIS, else
   CCPT_E_INVALID; a frame whose workspace alone exceeds the scratch (none
   of the supported shapes) gives CCPT_E_INVALID. */
#define CCPT_STATIC_MAX_ROIS 65536
int ccpt_track_batch_static(ccpt_ctx* ctx, const ccpt_roi* rois, int n, ccpt_result* out,
                            void* stream);

/* Backward pass of ccpt_track_batch for L = sum_i g_d[i] . d_i + g_peak[i] C_i(d_i)
   (implicit function theorem at the Newton maximiser; integer and grid
   maxima are piecewise constant and carry no gradient).  `fwd` is the
   device result array of the forward call on the same rois.  g_d: device
   [n][2] doubles; g_peak: device [n] doubles or NULL.  g_frames: device
   floats, the gradients of each roi packed one after another (ny*nx
   each, row-major, no pitch), or NULL; g_ref: device floats, one ny*nx
   block per reference in id order, summed over all rois using it, or
   NULL.  Frames whose forward status has NONFINITE, FLAT,
   NEWTON_FALLBACK or WINDOW_EXIT get zero gradient (n = 0 sets g_ref to
   zeros).  The reference set must be the one used by the forward call. */
int ccpt_track_grad(ccpt_ctx* ctx, const ccpt_roi* rois, int n, const ccpt_result* fwd,
                    const double* g_d, const double* g_peak, float* g_frames, float* g_ref,
                    void* stream);

/* Poisson Fisher information of the displacement for an expected image
   mu (Sec. IV shot-noise limit; Cramer-Rao bound = inverse): F_jl =
   sum_r (d mu/d d_j)(d mu/d d_l) / mu(r), with the derivatives of the
   band-limited translate mu(r - d) at d = 0.  `fisher` is a device array
   of 3 doubles (yy, yx, xx).  Every pixel of mu must be > 0
   (CCPT_E_INVALID otherwise, checked on the host after the copy). */
int ccpt_fisher(ccpt_ctx* ctx, const ccpt_image* mu, double* fisher, void* stream);

/* Offline reference of Sec. III.A (Eq. 8): the mean of the frames shifted
   back by their measured displacements, taken in Fourier space,
     out = F^-1[ (1/n') sum_i F[I_i](k) phi_ky(d_iy) phi_kx(d_ix) ],
   phi_k(s) = exp(2 pi i k~ s / N), cos(pi s) for a Nyquist bin (the
   band-limited shift of the interpolant the tracker maximises); frame i
   shifted back is I_i(r + d_i), the paper's I_i(r - r0).  The mean image is
   the reference in both modes (CC-SN then uses -1/(E + eps) of it).
   rois: n frames of one size N (host array as for ccpt_track_batch;
   ref_id is not used).  fwd: their results from ccpt_track_batch (device,
   roi order).  Frames whose status has CCPT_ST_NONFINITE or CCPT_ST_FLAT
   are left out; n' counts the others (n' = 0 gives zeros).  out: N x N
   float32, row-major, device, caller-owned.  One pass of Eq. 8 is
   ccpt_track_batch against E_n, this call, then ccpt_set_reference(out).
   Stream-ordered; may grow the context's workspace.
   Returns CCPT_E_INVALID for null pointers, n < 1 or mixed sizes,
   CCPT_E_UNSUPPORTED for an unsupported size. */
int ccpt_mean_aligned(ccpt_ctx* ctx, const ccpt_roi* rois, int n, const ccpt_result* fwd,
                      float* out, void* stream);

/* Real-time tracking with the reference low-pass of Sec. III.B (Eq. 9):
   tracks one frame against reference roi->ref_id (as ccpt_track_batch with
   n = 1; the result goes to out), then updates that reference with the
   frame shifted back by its displacement,
     F[E_i] = a0 F[I_i(r + d_i)] + (1 - a0) F[E_{i-1}],
   a0 = 1 - exp(-T/tau) in [0, 1] (T the frame interval, tau the filter time
   constant).  The reference starts as ccpt_set_reference left it (the
   paper's F[E_0] = F[I_0]: set the first frame).  A frame whose status has
   CCPT_ST_NONFINITE or CCPT_ST_FLAT leaves the reference unchanged.  E is
   the mean image in both modes; CC-SN recomputes B = -1/(E + eps) from the
   updated E (frames with values >= 0 keep E + eps > 0 for eps > 0).
   roi: one frame (host struct, device data) of any supported shape,
   Table I's rectangles included (the paper's own real-time run is 256 x 128
   at u = 256, Sec. IV.A); out: one result (device).  Stream-ordered with no
   host synchronisation, so calls can follow each other at the frame rate.
   CCPT_E_UNSUPPORTED in FP64 precision. */
int ccpt_track_update(ccpt_ctx* ctx, const ccpt_roi* roi, double a0, ccpt_result* out,
                      void* stream);

/* Drift correction of Sec. III.B (Eq. 10-12) on a stream of displacements
   (host arrays r and out of n (y, x) pairs; they may be the same array):
   Eq. 10  R_0 = a0 r_0, R_n = a0 r_n + (1 - a0) R_{n-1};
   or, with rate_limit > 0 (alpha/u; the paper suggests alpha = 0.5),
   Eq. 11-12 from n = 1 on: dR_n = a0 r_n - a0 R_{n-1}, a step longer than
   rate_limit cut to that length along dR_n, R_n = R_{n-1} + dR_n (the
   first offset is Eq. 10's R_0 in both forms);
   out_n = r_n - R_n.  state[3] = {R_{n-1} y, R_{n-1} x, number of samples
   already filtered} is read and updated, so a stream can be processed in
   pieces; three zeros start a new stream.  Pure host computation (no
   context).  CCPT_E_INVALID for bad arguments (null state, a0 outside
   [0, 1], negative rate_limit or sample count). */
int ccpt_drift_filter(const double* r, int n, double a0, double rate_limit, double* state,
                      double* out);

/* Launch scheduling of the batched path (a10): frames of one size are run in
   chunks whose spectra workspace stays resident in the Infinity Cache; the
   chunk size trades that residency against the number of launches.
   ccpt_autotune times ccpt_track_batch on `batch` frames of size n x n (each
   frame is the context's reference of that size; timing does not depend on
   content) over chunk sizes and the block plans of ccpt_plan, and keeps the
   fastest for later calls on this context.  Needs a reference of size n
   (CCPT_E_NOREF otherwise).  Allocates and synchronises the stream. */
int ccpt_autotune(ccpt_ctx* ctx, int n, int batch, void* stream);

/* Reads (set = 0) or sets (set != 0) the chunk size used for frames of size
   n x n; 0 restores the default.  Lets a caller persist tuning results. */
int ccpt_schedule(ccpt_ctx* ctx, int n, int* chunk, int set);

/* Launch plan of one frame shape (a10), any supported ny x nx (rectangles
   included): the chunk size and the block plans the kernels choose between.
   Tuning it changes how work is split over blocks and launches, never the
   arithmetic of a launch of a given size. */
typedef struct ccpt_plan {
  int chunk;        /* frames per launch chunk; 0 = default */
  int split_blocks; /* FP32 matrix DFT: launches of fewer than this many 32-row grid
                       tiles split Stage A over 8 ky slices added in a fixed order
                       (latency); -1 = default (128), 0 = never; at most 512 */
  int fused_min;    /* 256 x 256 frames: launches of at least this many frames take
                       the one-kernel correlation stage (one frame per CU), smaller
                       ones the three passes; -1 = default (128) */
} ccpt_plan;

/* Reads the plan in force for ny x nx frames (defaults filled in), or sets
   it (-1 fields and chunk 0 select the defaults).  CCPT_E_UNSUPPORTED for an
   unsupported shape, CCPT_E_INVALID for out-of-range fields.  Setting drops
   the context's captured graphs. */
int ccpt_get_plan(ccpt_ctx* ctx, int ny, int nx, ccpt_plan* plan);
int ccpt_set_plan(ccpt_ctx* ctx, int ny, int nx, const ccpt_plan* plan);

/* Concurrent size groups (a10; Sec. III.A: frames tracked against fixed
   references are independent): a ccpt_track_batch call with frames of
   several shapes runs its size groups on up to `lanes` streams at once, the
   caller's stream and context-owned ones (default priority) forked from it
   and joined back into it by events, so the call stays stream-ordered and
   graph-capturable; groups go to lanes largest estimated cost first, each
   to the least-loaded lane, and each lane has its own workspace.  Results
   do not depend on the lane count.  Reads (set = 0) or sets (set != 0) the
   most lanes a call uses: 1 (groups one after another) .. 4; 0 = default (4).
   Profiling contexts (CCPT_FLAG_PROFILE) use one lane. */
int ccpt_lanes(ccpt_ctx* ctx, int* lanes, int set);

/* Tunes the launch plans of every shape in `rois` and the lane count by
   timing ccpt_track_batch on this very array (a mixed-size batch is tuned
   as the mixed call it is): lanes 1..4, then each shape's chunk size and
   block plans with the others fixed, then lanes again.  Arguments as in
   ccpt_track_batch (validated the same way); allocates and synchronises the
   stream; results of later calls are unchanged up to the summation orders
   the plans select. */
int ccpt_autotune_batch(ccpt_ctx* ctx, const ccpt_roi* rois, int n, void* stream);

/* With CCPT_FLAG_PROFILE: total GPU time (ms) and number of launches of
   each stage recorded since the last reset, summed over chunks and calls.
   ms and launches are host arrays of n_stages entries.  Waits for the
   recorded events.  reset != 0 clears the record afterwards. */
int ccpt_stage_times(ccpt_ctx* ctx, double* ms, int* launches, int n_stages, int reset);

/* Static text of a return code. */
const char* ccpt_status_string(int code);

/* Copies the message of the last failing call into buf (NUL-terminated);
   returns the code of that call (CCPT_OK if none). */
int ccpt_last_error(const ccpt_ctx* ctx, char* buf, size_t len);

#ifdef __cplusplus
}
#endif

#endif /* CCPT_H */
