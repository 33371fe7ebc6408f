// Reference images from aligned frames: the offline reference of Sec. III.A
// (Eq. 8), the mean of all frames shifted back by their measured
// displacements, and the real-time low-pass of Sec. III.B (Eq. 9), both
// taken in Fourier space.
//
// A frame I tracked at displacement d (frame(r) ~ ref(r - d)) shifted back
// is I(r + d), the paper's I(r - r0) with r0 = -d; its spectrum is
// F[I](k) phi_ky(d_y) phi_kx(d_x) with phi_k(s) = exp(2 pi i k~ s / N) and
// phi = cos(pi s) for a Nyquist bin (the band-limited shift, the same
// interpolant the tracker maximises).  Frames whose tracking was non-finite
// or flat are left out of the mean.
#include <hip/hip_runtime.h>

#include <math.h>

#include "common.h"
#include "fft.h"

namespace ccpt {

constexpr int kRefThreads = 256;
constexpr int kAlignRows = 8;  // spectrum rows per block of k_align_spectra

__device__ __forceinline__ bool tracked(const ccpt_result& r) {
  return !(r.status & (CCPT_ST_NONFINITE | CCPT_ST_FLAT));
}

// phi_k(d) of one axis as FP32 complex, computed in FP64.
__device__ __forceinline__ float2 shift_phase(int k, int N, double d) {
  if (2 * k == N) return make_float2((float)cospi(d), 0.f);
  const int kt = 2 * k < N ? k : k - N;
  double sn, cs;
  sincospi(2.0 * (double)kt * d / (double)N, &sn, &cs);
  return make_float2((float)cs, (float)sn);
}

// F[f] (row-major N x (N/2+1)) *= phi_ky(d_y) phi_kx(d_x) for frame f's
// displacement; frames that did not track are zeroed.
template <int N>
__global__ void __launch_bounds__(kRefThreads) k_align_spectra(const FrameDesc* __restrict__ desc,
                                                               int first,
                                                               const ccpt_result* __restrict__ fwd,
                                                               float2* __restrict__ F) {
  constexpr int H = N / 2 + 1;
  __shared__ float2 px[H];
  __shared__ float2 py[kAlignRows];
  const int f = blockIdx.y, y0 = blockIdx.x * kAlignRows, tid = threadIdx.x;
  const ccpt_result r = fwd[desc[first + f].out_idx];
  const bool ok = tracked(r);
  for (int k = tid; k < H; k += kRefThreads) px[k] = ok ? shift_phase(k, N, r.d[1]) : make_float2(0.f, 0.f);
  for (int k = tid; k < kAlignRows; k += kRefThreads)
    py[k] = (ok && y0 + k < N) ? shift_phase(y0 + k, N, r.d[0]) : make_float2(0.f, 0.f);
  __syncthreads();
  float2* Ff = F + (size_t)f * N * H;
  const int rows = min(kAlignRows, N - y0);
  for (int i = tid; i < rows * H; i += kRefThreads) {
    const int ry = i / H, kx = i - ry * H;
    const size_t e = (size_t)(y0 + ry) * H + kx;
    // (a frame that did not track may hold NaN: written as zeros, not scaled)
    Ff[e] = ok ? cmul(Ff[e], cmul(py[ry], px[kx])) : make_float2(0.f, 0.f);
  }
}

// acc[k] += sum over the chunk's frames of F[f][k], frames in order.
template <int N>
__global__ void k_sum_spectra(int count, const float2* __restrict__ F, float2* __restrict__ acc) {
  constexpr int H = N / 2 + 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * H) return;
  float2 sum = make_float2(0.f, 0.f);
  for (int f = 0; f < count; ++f) sum = cadd(sum, F[(size_t)f * N * H + e]);
  acc[e] = cadd(acc[e], sum);
}

__global__ void k_count_tracked(const FrameDesc* __restrict__ desc, int first, int count,
                                const ccpt_result* __restrict__ fwd, unsigned* __restrict__ cnt) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f < count && tracked(fwd[desc[first + f].out_idx])) atomicAdd(cnt, 1u);
}

// img *= scale / count (count >= 1; an empty mean is left as zeros)
__global__ void k_scale_by_count(float* __restrict__ img, int nn, float scale,
                                 const unsigned* __restrict__ cnt) {
  const unsigned c = *cnt;
  const float s = c ? scale / (float)c : 0.f;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += gridDim.x * blockDim.x)
    img[i] *= s;
}

// Real-time reference update (Sec. III.B, Eq. 9) by one frame with spectrum
// F (row-major NY x (NX/2+1), the tall layout) and result res: v = F
// phi_ky(d_y) phi_kx(d_x) (the frame shifted back; for a wide frame, held
// transposed, the spectrum's rows run along the frame's x) enters the
// resident spectrum S as
//   S <- a0 conj(v) + b1 S   (conj_s: S = conj F[E], the CC-U reference)
//   S <- a0 v + b1 S         (S = F[E], kept for CC-SN)
// and a frame that did not track leaves S unchanged.
template <int NY, int NX>
__global__ void __launch_bounds__(kRefThreads) k_rt_update(const ccpt_result* __restrict__ res,
                                                           const float2* __restrict__ F,
                                                           float2* __restrict__ S, float a0,
                                                           float b1, int conj_s, int trans) {
  constexpr int H = NX / 2 + 1;
  __shared__ float2 px[H];
  __shared__ float2 py[kAlignRows];
  const int y0 = blockIdx.x * kAlignRows, tid = threadIdx.x;
  const ccpt_result r = *res;
  if (!tracked(r)) return;
  const double dy = trans ? r.d[1] : r.d[0], dx = trans ? r.d[0] : r.d[1];
  for (int k = tid; k < H; k += kRefThreads) px[k] = shift_phase(k, NX, dx);
  for (int k = tid; k < kAlignRows; k += kRefThreads)
    py[k] = y0 + k < NY ? shift_phase(y0 + k, NY, dy) : make_float2(0.f, 0.f);
  __syncthreads();
  const int rows = min(kAlignRows, NY - y0);
  for (int i = tid; i < rows * H; i += kRefThreads) {
    const int ry = i / H, kx = i - ry * H;
    const size_t e = (size_t)(y0 + ry) * H + kx;
    float2 v = cmul(F[e], cmul(py[ry], px[kx]));
    if (conj_s) v = cconj(v);
    const float2 o = S[e];
    S[e] = make_float2(a0 * v.x + b1 * o.x, a0 * v.y + b1 * o.y);
  }
}

template <int NY, int NX>
static int rt_update_n(const ccpt_result* res, const float2* F, float2* S, float a0, float b1,
                       int conj_s, int trans, hipStream_t s) {
  hipLaunchKernelGGL((k_rt_update<NY, NX>), dim3((NY + kAlignRows - 1) / kAlignRows),
                     dim3(kRefThreads), 0, s, res, F, S, a0, b1, conj_s, trans);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N>
static int align_accumulate_n(const FrameDesc* desc, int first, int count, const ccpt_result* fwd,
                              float2* F, float2* acc, unsigned* cnt, hipStream_t s) {
  constexpr int H = N / 2 + 1;
  hipLaunchKernelGGL((k_align_spectra<N>), dim3((N + kAlignRows - 1) / kAlignRows, count),
                     dim3(kRefThreads), 0, s, desc, first, fwd, F);
  hipLaunchKernelGGL((k_sum_spectra<N>), dim3((N * H + 255) / 256), dim3(256), 0, s, count,
                     (const float2*)F, acc);
  hipLaunchKernelGGL(k_count_tracked, dim3((count + 255) / 256), dim3(256), 0, s, desc, first,
                     count, fwd, cnt);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_align_accumulate(int N, const FrameDesc* desc, int first, int count,
                            const ccpt_result* fwd, float2* F, float2* acc, unsigned* cnt,
                            hipStream_t s) {
  switch (N) {
#define CASE(n) \
  case n:       \
    return align_accumulate_n<n>(desc, first, count, fwd, F, acc, cnt, s);
    CCPT_FOR_SIZES(CASE)
#undef CASE
  }
  return -2;
}

int launch_rt_update(int ny, int nx, int trans, const ccpt_result* res, const float2* F, float2* S,
                     float a0, float b1, int conj_s, hipStream_t s) {
  if (ny == nx) {
    switch (ny) {
#define CASE(n) \
  case n:       \
    return rt_update_n<n, n>(res, F, S, a0, b1, conj_s, 0, s);
      CCPT_FOR_SIZES(CASE)
#undef CASE
    }
    return -2;
  }
#define CASE(a, b) \
  if (ny == a && nx == b) return rt_update_n<a, b>(res, F, S, a0, b1, conj_s, trans, s);
  CCPT_FOR_RECT(CASE)
#undef CASE
  return -2;
}

int launch_scale_by_count(float* img, int nn, float scale, const unsigned* cnt, hipStream_t s) {
  int blocks = (nn + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_scale_by_count, dim3(blocks), dim3(256), 0, s, img, nn, scale, cnt);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ccpt
