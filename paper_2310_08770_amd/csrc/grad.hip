// Adjoint of the refined displacement and the Fisher information.
//
// At the Newton maximiser d of the band-limited correlation C(s) the
// gradient of C vanishes, so for L = g_d . d + g_c C(d) the implicit function
// theorem gives, with lam = -H^-1 g_d (H the Hessian of C at d),
//
//   dL/dA(x) = sum_k conj(F[B](k)) Psi(k) exp(-2 pi i k.x / N)
//   dL/dB(x) = sum_k F[A](k)       Psi(k) exp(+2 pi i k.x / N)
//   Psi(k)   = (lam_y d/ds_y + lam_x d/ds_x + g_c) phi_k(s) / N^2  at s = d,
//
// phi_k(s) = phi_ky(s_y) phi_kx(s_x) as in the forward pass (cos(pi s) for a
// Nyquist bin).  Both sums are real inverse transforms of Hermitian half
// spectra: Q_A = conj(R Psi) with R = conj F[B] (the resident reference
// spectrum) and Q_B = F[A] Psi.  CC-SN chains through A = (I+eps)^2 and
// B = -1/(E+eps).  The reference gradient is summed over frames in the
// frequency domain (fixed order, no float atomics) and transformed once.
//
// Fisher information of the displacement for an expected image mu under
// Poisson noise: F_jl = sum_r (d_j mu)(d_l mu) / mu, where d_j mu is the
// derivative of the band-limited translate mu(r - d) at d = 0.
#include <hip/hip_runtime.h>

#include <math.h>

#include "common.h"
#include "fft.h"

namespace ccpt {

constexpr int kGThreads = 256;

__device__ __forceinline__ void phi2(int k, int n, double s, double2& p0, double2& p1) {
  const double pi = 3.14159265358979323846;
  if (2 * k == n) {
    double sn, cs;
    sincospi(s, &sn, &cs);
    p0 = make_double2(cs, 0.0);
    p1 = make_double2(-pi * sn, 0.0);
    return;
  }
  const int kt = 2 * k < n ? k : k - n;
  double sn, cs;
  sincospi(2.0 * (double)kt * s / (double)n, &sn, &cs);
  const double w = 2.0 * pi * (double)kt / (double)n;
  p0 = make_double2(cs, sn);
  p1 = make_double2(-w * sn, w * cs);
}

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ bool grad_usable(unsigned status) {
  return (status & (CCPT_ST_NONFINITE | CCPT_ST_FLAT | CCPT_ST_NEWTON_FALLBACK |
                    CCPT_ST_WINDOW_EXIT)) == 0;
}

// One block per (ky block, frame): builds Psi on the half spectrum and writes
// QA = conj(R Psi) (frame gradient) and QB = F[A] Psi (reference gradient).
template <int N>
__global__ void __launch_bounds__(kGThreads) k_grad_psi(const FrameDesc* __restrict__ desc, int first,
                                                        const ccpt_result* __restrict__ fwd,
                                                        const double* __restrict__ g_d,
                                                        const double* __restrict__ g_peak,
                                                        const float2* __restrict__ FA,
                                                        float2* __restrict__ QA,
                                                        float2* __restrict__ QB, int rows) {
  constexpr int H = N / 2 + 1;
  __shared__ double2 ey0[N], ey1[N];
  __shared__ double2 ex0[H], ex1[H];
  const int tid = threadIdx.x;
  const int f = blockIdx.y;
  const int y0 = blockIdx.x * rows;
  const FrameDesc d = desc[first + f];
  const ccpt_result r = fwd[d.out_idx];
  double lam_y = 0.0, lam_x = 0.0, gc = 0.0;
  const bool ok = grad_usable(r.status);
  if (ok) {
    const double gy = g_d[2 * d.out_idx], gx = g_d[2 * d.out_idx + 1];
    const double hyy = r.hess[0], hyx = r.hess[1], hxx = r.hess[2];
    const double det = hyy * hxx - hyx * hyx;
    // lam = -H^-1 g
    lam_y = -(hxx * gy - hyx * gx) / det;
    lam_x = -(hyy * gx - hyx * gy) / det;
    gc = g_peak ? g_peak[d.out_idx] : 0.0;
  }
  for (int k = tid; k < N; k += kGThreads) phi2(k, N, r.d[0], ey0[k], ey1[k]);
  for (int k = tid; k < H; k += kGThreads) phi2(k, N, r.d[1], ex0[k], ex1[k]);
  __syncthreads();
  const double inv = 1.0 / ((double)N * (double)N);
  const size_t base = (size_t)f * N * H;
  const float2* R = (const float2*)d.rspec;
  for (int i = tid; i < rows * H; i += kGThreads) {
    const int ky = y0 + i / H, kx = i % H;
    const size_t e = (size_t)ky * H + kx;
    float2 qa = make_float2(0.f, 0.f), qb = qa;
    if (ok) {
      const double2 py = ey0[ky], dpy = ey1[ky], px = ex0[kx], dpx = ex1[kx];
      double2 psi = zmul(py, px);
      const double2 a = zmul(dpy, px), b = zmul(py, dpx);
      psi = make_double2((gc * psi.x + lam_y * a.x + lam_x * b.x) * inv,
                         (gc * psi.y + lam_y * a.y + lam_x * b.y) * inv);
      const float2 rr = R[e];
      const double2 ra = zmul(make_double2(rr.x, rr.y), psi);
      qa = make_float2((float)ra.x, (float)-ra.y);
      const float2 fa = FA[base + e];
      const double2 rb = zmul(make_double2(fa.x, fa.y), psi);
      qb = make_float2((float)rb.x, (float)rb.y);
    }
    QA[base + e] = qa;
    if (QB) QB[base + e] = qb;
  }
}

// Frame gradient: c2r output (already scaled) times the CC-SN chain factor
// 2 (I + eps), scattered to the caller's packed gradient array.
template <int N>
__global__ void k_grad_frames(const FrameDesc* __restrict__ desc, int first,
                              const float* __restrict__ img, const long* __restrict__ goff,
                              float* __restrict__ g_frames, int mode, float eps) {
  const int f = blockIdx.y;
  const FrameDesc d = desc[first + f];
  float* out = g_frames + goff[d.out_idx];
  const float* src = img + (size_t)f * N * N;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N * N; i += gridDim.x * blockDim.x) {
    float v = src[i];
    if (mode == CCPT_MODE_CCSN) {
      const int y = i / N, x = i - y * N;
      const long idx = (long)y * d.pitch + x;
      const float px = d.dtype == CCPT_U16   ? (float)((const unsigned short*)d.data)[idx]
                       : d.dtype == CCPT_F64 ? (float)((const double*)d.data)[idx]
                                             : ((const float*)d.data)[idx];
      v *= 2.0f * (px + eps);
    }
    out[i] = v;
  }
}

// acc[ref][k] += sum over the chunk's frames of that reference of QB[f][k],
// frames taken in order (deterministic).
template <int N>
__global__ void k_ref_accum(const FrameDesc* __restrict__ desc, int first, int count,
                            const float2* __restrict__ QB, float2* const* __restrict__ acc) {
  constexpr int H = N / 2 + 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * H) return;
  int cur = -1;
  float2 sum = make_float2(0.f, 0.f);
  for (int f = 0; f < count; ++f) {
    const int ref = desc[first + f].ref_id;
    if (ref != cur) {
      if (cur >= 0) {
        float2* a = acc[cur];
        a[e] = cadd(a[e], sum);
      }
      cur = ref;
      sum = make_float2(0.f, 0.f);
    }
    sum = cadd(sum, QB[(size_t)f * N * H + e]);
  }
  if (cur >= 0) {
    float2* a = acc[cur];
    a[e] = cadd(a[e], sum);
  }
}

// Reference gradient image: chain factor of B = -1/(E+eps) is 1/(E+eps)^2.
__global__ void k_grad_ref_chain(const float* __restrict__ img, const float* __restrict__ E, int nn,
                                 int mode, float eps, float* __restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += gridDim.x * blockDim.x) {
    float v = img[i];
    if (mode == CCPT_MODE_CCSN) {
      const float e = E[i] + eps;
      v /= e * e;
    }
    out[i] = v;
  }
}

// Derivative spectra of the band-limited translate at d = 0:
// d mu / d d_j = -sum_k F(k) (i w_kj) e^{2 pi i k.r/N} / N^2, Nyquist term 0.
template <int N>
__global__ void k_fisher_deriv(const float2* __restrict__ F, float2* __restrict__ Dy,
                               float2* __restrict__ Dx) {
  constexpr int H = N / 2 + 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * H) return;
  const int ky = e / H, kx = e % H;
  const double pi = 3.14159265358979323846;
  const int kty = 2 * ky < N ? ky : ky - N;
  const double wy = (2 * ky == N) ? 0.0 : 2.0 * pi * kty / N;
  const double wx = (2 * kx == N) ? 0.0 : 2.0 * pi * kx / N;
  const double inv = 1.0 / ((double)N * (double)N);
  const float2 v = F[e];
  // -(i w) v = (w v.y, -w v.x)
  Dy[e] = make_float2((float)(wy * v.y * inv), (float)(-wy * v.x * inv));
  Dx[e] = make_float2((float)(wx * v.y * inv), (float)(-wx * v.x * inv));
}

// Per-block partial sums of (dy^2/mu, dy dx/mu, dx^2/mu) in FP64.
__global__ void k_fisher_partial(const float* __restrict__ dy, const float* __restrict__ dx,
                                 const void* __restrict__ mu, int dtype, int pitch, int n,
                                 double* __restrict__ part) {
  __shared__ double red[3][kGThreads / 64];
  double a = 0, b = 0, c = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n * n; i += gridDim.x * blockDim.x) {
    const int y = i / n, x = i - y * n;
    const long idx = (long)y * pitch + x;
    const double m = dtype == CCPT_U16   ? (double)((const unsigned short*)mu)[idx]
                     : dtype == CCPT_F64 ? ((const double*)mu)[idx]
                                         : (double)((const float*)mu)[idx];
    const double p = dy[i], q = dx[i];
    a += p * p / m;
    b += p * q / m;
    c += q * q / m;
  }
  double v[3] = {a, b, c};
  for (int t = 0; t < 3; ++t) {
    double s = v[t];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[t][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0;
    for (int w = 0; w < kGThreads / 64; ++w) s += red[threadIdx.x][w];
    part[blockIdx.x * 3 + threadIdx.x] = s;
  }
}

__global__ void k_fisher_final(const double* __restrict__ part, int nblocks, double* __restrict__ out) {
  if (threadIdx.x < 3) {
    double s = 0;
    for (int b = 0; b < nblocks; ++b) s += part[b * 3 + threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// ------------------------------------------------------------ launchers

template <int N>
static int grad_psi_n(const FrameDesc* desc, int first, int count, const ccpt_result* fwd,
                      const double* g_d, const double* g_peak, const float2* FA, float2* QA,
                      float2* QB, hipStream_t s) {
  const int rows = N >= 64 ? 8 : N;
  hipLaunchKernelGGL((k_grad_psi<N>), dim3(N / rows, count), dim3(kGThreads), 0, s, desc, first,
                     fwd, g_d, g_peak, FA, QA, QB, rows);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N>
static int grad_frames_n(const FrameDesc* desc, int first, int count, const float* img,
                         const long* goff, float* g_frames, int mode, float eps, hipStream_t s) {
  hipLaunchKernelGGL((k_grad_frames<N>), dim3((N * N + 255) / 256 < 64 ? (N * N + 255) / 256 : 64, count),
                     dim3(256), 0, s, desc, first, img, goff, g_frames, mode, eps);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N>
static int ref_accum_n(const FrameDesc* desc, int first, int count, const float2* QB,
                       float2* const* acc, hipStream_t s) {
  constexpr int H = N / 2 + 1;
  hipLaunchKernelGGL((k_ref_accum<N>), dim3((N * H + 255) / 256), dim3(256), 0, s, desc, first,
                     count, QB, acc);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N>
static int fisher_deriv_n(const float2* F, float2* Dy, float2* Dx, hipStream_t s) {
  constexpr int H = N / 2 + 1;
  hipLaunchKernelGGL((k_fisher_deriv<N>), dim3((N * H + 255) / 256), dim3(256), 0, s, F, Dy, Dx);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_grad_psi(int N, const FrameDesc* desc, int first, int count, const ccpt_result* fwd,
                    const double* g_d, const double* g_peak, const float2* FA, float2* QA,
                    float2* QB, hipStream_t s) {
  switch (N) {
#define CASE(n) \
  case n:       \
    return grad_psi_n<n>(desc, first, count, fwd, g_d, g_peak, FA, QA, QB, s);
    CCPT_FOR_SIZES(CASE)
#undef CASE
  }
  return -2;
}

int launch_grad_frames(int N, const FrameDesc* desc, int first, int count, const float* img,
                       const long* goff, float* g_frames, int mode, float eps, hipStream_t s) {
  switch (N) {
#define CASE(n) \
  case n:       \
    return grad_frames_n<n>(desc, first, count, img, goff, g_frames, mode, eps, s);
    CCPT_FOR_SIZES(CASE)
#undef CASE
  }
  return -2;
}

int launch_ref_accum(int N, const FrameDesc* desc, int first, int count, const float2* QB,
                     float2* const* acc, hipStream_t s) {
  switch (N) {
#define CASE(n) \
  case n:       \
    return ref_accum_n<n>(desc, first, count, QB, acc, s);
    CCPT_FOR_SIZES(CASE)
#undef CASE
  }
  return -2;
}

int launch_grad_ref_chain(const float* img, const float* E, int nn, int mode, float eps,
                          float* out, hipStream_t s) {
  int blocks = (nn + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_grad_ref_chain, dim3(blocks), dim3(256), 0, s, img, E, nn, mode, eps, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_fisher_deriv(int N, const float2* F, float2* Dy, float2* Dx, hipStream_t s) {
  switch (N) {
#define CASE(n) \
  case n:       \
    return fisher_deriv_n<n>(F, Dy, Dx, s);
    CCPT_FOR_SIZES(CASE)
#undef CASE
  }
  return -2;
}

int launch_fisher_reduce(const float* dy, const float* dx, const void* mu, int dtype, int pitch,
                         int n, double* part, int nblocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_fisher_partial, dim3(nblocks), dim3(kGThreads), 0, s, dy, dx, mu, dtype,
                     pitch, n, part);
  hipLaunchKernelGGL(k_fisher_final, dim3(1), dim3(64), 0, s, part, nblocks, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ccpt
