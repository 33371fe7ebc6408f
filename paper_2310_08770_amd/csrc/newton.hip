// FP64 refinement of the upsampled-grid maximum and the result record.
//
// The band-limited correlation (the function the paper's upsampled DFT
// samples, Sec. III) is evaluated directly from the FP32 cross-power
// spectrum in FP64 arithmetic, with its gradient and Hessian:
//
//   C(s) = 1/N^2 sum_kx w_kx Re[ phi_kx(s_x) V_kx(s_y) ],
//   V_kx(s_y) = sum_ky X[ky, kx] phi_ky(s_y),
//   phi_k(s) = exp(2 pi i k~ s / N),  phi_{N/2}(s) = cos(pi s),
//
// and Newton steps s <- s - H^-1 grad C start from the grid maximum.  The
// same safeguards as the reference definition apply: a Hessian that is not
// negative definite or a step beyond the step limit falls back to the grid
// estimate, and a result more than 0.75 px from the integer peak is
// flagged and replaced by the grid estimate (0.75 px for the paper's
// 1.5-px window).
#include <hip/hip_runtime.h>

#include <math.h>

#include "common.h"

namespace ccpt {

constexpr int kNThreads = 256;

struct CEval {
  double c, gy, gx, hyy, hxx, hxy;
};

__device__ __forceinline__ void phi3(int k, int n, double s, double2& p0, double2& p1, double2& p2) {
  if (2 * k == n) {
    double sn, cs;
    sincospi(s, &sn, &cs);
    const double pi = 3.14159265358979323846;
    p0 = make_double2(cs, 0.0);
    p1 = make_double2(-pi * sn, 0.0);
    p2 = make_double2(-pi * pi * cs, 0.0);
    return;
  }
  const int kt = 2 * k < n ? k : k - n;
  double sn, cs;
  sincospi(2.0 * (double)kt * s / (double)n, &sn, &cs);
  const double w = 2.0 * 3.14159265358979323846 * (double)kt / (double)n;
  p0 = make_double2(cs, sn);
  p1 = make_double2(-w * sn, w * cs);
  p2 = make_double2(-w * w * cs, -w * w * sn);
}

__device__ __forceinline__ double re_mul(double2 a, double2 b) { return a.x * b.x - a.y * b.y; }

template <int N>
__device__ CEval eval_c(const float2* __restrict__ Xf, double sy, double sx, double2 (*ey)[3],
                        double (*red)[kNThreads / 64]) {
  constexpr int H = N / 2 + 1;
  const int tid = threadIdx.x;
  for (int ky = tid; ky < N; ky += kNThreads) phi3(ky, N, sy, ey[ky][0], ey[ky][1], ey[ky][2]);
  __syncthreads();
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int kx = tid; kx < H; kx += kNThreads) {
    double2 v0 = make_double2(0, 0), v1 = v0, v2 = v0;
    const float2* col = Xf + kx;
#pragma unroll 4
    for (int ky = 0; ky < N; ++ky) {
      const float2 xf = col[(size_t)ky * H];
      const double xr = xf.x, xi = xf.y;
      const double2 a = ey[ky][0], b = ey[ky][1], c = ey[ky][2];
      v0.x += xr * a.x - xi * a.y;
      v0.y += xr * a.y + xi * a.x;
      v1.x += xr * b.x - xi * b.y;
      v1.y += xr * b.y + xi * b.x;
      v2.x += xr * c.x - xi * c.y;
      v2.y += xr * c.y + xi * c.x;
    }
    double2 e0, e1, e2;
    phi3(kx, N, sx, e0, e1, e2);
    const double wt = (kx == 0 || 2 * kx == N) ? 1.0 : 2.0;
    acc[0] += wt * re_mul(e0, v0);
    acc[1] += wt * re_mul(e0, v1);
    acc[2] += wt * re_mul(e1, v0);
    acc[3] += wt * re_mul(e0, v2);
    acc[4] += wt * re_mul(e2, v0);
    acc[5] += wt * re_mul(e1, v1);
  }
  // deterministic block reduction
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    double v = acc[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    acc[q] = v;
  }
  __syncthreads();
  if ((tid & 63) == 0)
    for (int q = 0; q < 6; ++q) red[q][tid >> 6] = acc[q];
  __syncthreads();
  double r[6];
  for (int q = 0; q < 6; ++q) {
    double v = 0;
    for (int w = 0; w < kNThreads / 64; ++w) v += red[q][w];
    r[q] = v / ((double)N * (double)N);
  }
  __syncthreads();
  return CEval{r[0], r[1], r[2], r[3], r[4], r[5]};
}

template <int N>
__global__ void __launch_bounds__(kNThreads) k_newton(GroupParams g, double step_limit) {
  constexpr int H = N / 2 + 1;
  __shared__ double2 ey[N][3];
  __shared__ double red[6][kNThreads / 64];
  const int f = blockIdx.x;
  const int tid = threadIdx.x;
  const FrameState st = g.st[f];
  const FrameDesc d = g.desc[g.first + f];
  ccpt_result* out = g.out + d.out_idx;
  ccpt_result r;
  r.reserved = 0;
  if (st.flags & CCPT_ST_NONFINITE) {
    if (tid == 0) {
      const double nan = __builtin_nan("");
      r.d[0] = r.d[1] = nan;
      r.peak = nan;
      r.hess[0] = r.hess[1] = r.hess[2] = nan;
      r.d_grid[0] = r.d_grid[1] = __builtin_nanf("");
      r.p[0] = r.p[1] = 0;
      r.status = CCPT_ST_NONFINITE;
      *out = r;
    }
    return;
  }
  if (st.amin == st.amax) {
    if (tid == 0) {
      r.d[0] = r.d[1] = 0.0;
      r.peak = 0.0;
      r.hess[0] = r.hess[1] = r.hess[2] = 0.0;
      r.d_grid[0] = r.d_grid[1] = 0.f;
      r.p[0] = r.p[1] = 0;
      r.status = CCPT_ST_FLAT;
      *out = r;
    }
    return;
  }
  unsigned pk = key_index(st.peak_key);
  if (pk >= (unsigned)(N * N)) pk = 0;
  int py = pk / N, px = pk % N;
  if (2 * py >= N) py -= N;
  if (2 * px >= N) px -= N;
  unsigned gk = key_index(st.grid_key);
  if (gk >= (unsigned)(g.M * g.M)) gk = (unsigned)(g.c * g.M + g.c);
  const int my = gk / g.M, mx = gk % g.M;
  const double dgy = py + (double)(my - g.c) / g.u;
  const double dgx = px + (double)(mx - g.c) / g.u;
  const float2* Xf = g.X + (size_t)f * N * H;

  double sy = dgy, sx = dgx;
  unsigned status = 0;
  for (int it = 0; it < g.newton_iters; ++it) {
    const CEval e = eval_c<N>(Xf, sy, sx, ey, red);
    const double det = e.hyy * e.hxx - e.hxy * e.hxy;
    if (!(e.hyy < 0.0 && det > 0.0)) {
      status |= CCPT_ST_NEWTON_FALLBACK;
      sy = dgy;
      sx = dgx;
      break;
    }
    const double ty = -(e.hxx * e.gy - e.hxy * e.gx) / det;
    const double tx = -(e.hyy * e.gx - e.hxy * e.gy) / det;
    if (fmax(fabs(ty), fabs(tx)) > step_limit) {
      status |= CCPT_ST_NEWTON_FALLBACK;
      sy = dgy;
      sx = dgx;
      break;
    }
    sy += ty;
    sx += tx;
  }
  if (fmax(fabs(sy - py), fabs(sx - px)) > g.half_window) {
    status |= CCPT_ST_WINDOW_EXIT;
    sy = dgy;
    sx = dgx;
  }
  const CEval e = eval_c<N>(Xf, sy, sx, ey, red);
  if (tid == 0) {
    r.d[0] = sy;
    r.d[1] = sx;
    r.peak = e.c;
    r.hess[0] = e.hyy;
    r.hess[1] = e.hxy;
    r.hess[2] = e.hxx;
    r.d_grid[0] = (float)dgy;
    r.d_grid[1] = (float)dgx;
    r.p[0] = py;
    r.p[1] = px;
    r.status = status;
    *out = r;
  }
}

template <int N>
static int newton_n(const GroupParams& g, double step_limit, hipStream_t s) {
  hipLaunchKernelGGL((k_newton<N>), dim3(g.count), dim3(kNThreads), 0, s, g, step_limit);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

#define CCPT_FOR_SIZES(X) \
  X(16) X(18) X(24) X(32) X(36) X(48) X(54) X(64) X(72) X(96) X(108) X(128) X(144) X(162) X(192) \
  X(216) X(256) X(288) X(324) X(384) X(432) X(486) X(512)

int launch_newton(int N, const GroupParams& g, double step_limit, hipStream_t s) {
  switch (N) {
#define CASE(n) \
  case n:       \
    return newton_n<n>(g, step_limit, s);
    CCPT_FOR_SIZES(CASE)
#undef CASE
  }
  return -2;
}

}  // namespace ccpt
