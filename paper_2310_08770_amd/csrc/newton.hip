// FP64 refinement of the upsampled-grid maximum and the result record.
//
// The band-limited correlation (the function the paper's upsampled DFT
// samples, Sec. III) around an expansion centre s0 is
//
//   C(s0 + e) = 1/N^2 sum_kx w_kx Re[ phi_kx(s0x + ex) V_kx(s0y + ey) ],
//   V_kx(s0y + ey) = sum_ky X[ky, kx] phi_ky(s0y) exp(i a_ky ey),
//   phi_k(s) = exp(i a_k s), a_k = 2 pi k~ / N, and for a Nyquist bin
//   phi(s) = cos(pi s) = Re exp(i pi s),
//
// with w = 1 at kx = 0 and N/2, else 2.  Expanding both exponentials in
// powers of e turns C into a polynomial
//
//   C(s0 + e) = sum_{n+m <= K} c_nm ey^n ex^m / (n! m!),
//   c_nm = 1/N^2 sum_kx w Re[ P_m(kx) M_n(kx) ],
//   M_n(kx) = sum_ky X[ky, kx] phi_ky(s0y) (i a_ky)^n,
//   P_m(kx) = phi_kx(s0x) (i b_kx)^m       (real part only for a Nyquist bin)
//
// whose truncation error is below (pi |e|)^(K+1)/(K+1)! relative, i.e. at
// FP64 rounding for |e| <= 0.02 px with K = 7.  One streaming pass over the
// FP32 spectrum (FP64 arithmetic) therefore gives C, its gradient and Hessian
// anywhere near the seed, and the Newton iterations run on the polynomial.
// (In the FP64 mode the spectrum itself is FP64.)
// If an iterate moves farther than the model radius from the centre, the
// model is rebuilt around it (at most three passes).
//
// Safeguards as in the reference definition: a Hessian that is not negative
// definite or a step beyond the step limit falls back to the grid estimate,
// and a result farther than half the window from the integer peak is
// flagged and replaced by the grid estimate.
#include <hip/hip_runtime.h>

#include <math.h>

#include "common.h"

namespace ccpt {

constexpr int kNThreads = 512;
constexpr int kOrder = 7;                               // K
constexpr int kCoef = (kOrder + 1) * (kOrder + 2) / 2;  // pairs with n + m <= K
static_assert(kCoef == kNewtonCoef, "model size");
constexpr double kModelRadius = 0.02;                   // px
constexpr int kMaxPasses = 3;

// pairs ordered by n, then m
__host__ __device__ constexpr int coef_index(int n, int m) {
  return n * (kOrder + 1) - n * (n - 1) / 2 + m;
}

struct Deriv {
  double c, gy, gx, hyy, hxy, hxx;
};

// C and its first and second derivatives of the polynomial model at e.
__device__ Deriv model_eval(const double* coef, double ey, double ex) {
  double py[kOrder + 1], px[kOrder + 1];  // e^j / j!
  py[0] = px[0] = 1.0;
#pragma unroll
  for (int j = 1; j <= kOrder; ++j) {
    py[j] = py[j - 1] * ey / j;
    px[j] = px[j - 1] * ex / j;
  }
  Deriv d{0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int n = 0; n <= kOrder; ++n)
#pragma unroll
    for (int m = 0; n + m <= kOrder; ++m) {
      const double c = coef[coef_index(n, m)];
      d.c += c * py[n] * px[m];
      if (n >= 1) d.gy += c * py[n - 1] * px[m];
      if (m >= 1) d.gx += c * py[n] * px[m - 1];
      if (n >= 2) d.hyy += c * py[n - 2] * px[m];
      if (m >= 2) d.hxx += c * py[n] * px[m - 2];
      if (n >= 1 && m >= 1) d.hxy += c * py[n - 1] * px[m - 1];
    }
  return d;
}

// Accumulates t (i a)^n into M[n], n = 0..K.
__device__ __forceinline__ void add_powers(double2* M, double2 t, double a) {
#pragma unroll
  for (int n = 0; n <= kOrder; ++n) {
    M[n].x += t.x;
    M[n].y += t.y;
    t = make_double2(-a * t.y, a * t.x);
  }
}

// Lane moves inside rows of 16 lanes by DPP (VALU operand modifiers, no
// LDS traffic), on doubles.  CTRL: 0xB1 / 0x4E quad permutations [1,0,3,2] /
// [2,3,0,1], 0x141 half-row mirror, 0x140 row mirror, 0x120 + d rotation by d.
// Every lane of the wave must be active (a lane reading an inactive one
// would receive 0); the callers below run in wave-uniform control flow.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum over each aligned group of G adjacent lanes, every lane of the group
// receiving it; the same additions in the same order as an xor butterfly
// (at the mirror steps the partner lane holds the value the xor partner
// would, the quads or half-rows being uniform by then).
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (G >= 2) v += dpp_f64<0xB1>(v);
  if constexpr (G >= 4) v += dpp_f64<0x4E>(v);
  if constexpr (G >= 8) v += dpp_f64<0x141>(v);
  if constexpr (G >= 16) v += dpp_f64<0x140>(v);
  if constexpr (G >= 32) v += __shfl_xor(v, 16, 64);
  if constexpr (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// Sum over the lanes of a 16-lane row that agree modulo S (S a power of two
// up to 16), every such lane receiving it: rotations by S, 2S, ..., 8.
template <int S>
__device__ __forceinline__ double row_residue_sum(double v) {
  if constexpr (S <= 1) v += dpp_f64<0x120 + 1>(v);
  if constexpr (S <= 2) v += dpp_f64<0x120 + 2>(v);
  if constexpr (S <= 4) v += dpp_f64<0x120 + 4>(v);
  if constexpr (S <= 8) v += dpp_f64<0x120 + 8>(v);
  return v;
}

constexpr int pow2_floor(int x) {
  int p = 1;
  while (2 * p <= x) p *= 2;
  return p;
}

// Work split of one model pass over a spectrum of NY rows and NX/2+1
// columns: each column kx < NX/2 is shared by S adjacent lanes (ky segments
// of length SEG); after their moments are combined, lane `seg` accumulates
// the coefficients with m = seg, seg + S, ... (QM of them).
template <int NY, int NX>
struct ModelSplit {
  static constexpr int NC = NX / 2;
  static constexpr int S0 = kNThreads / NC;
  static constexpr int S = pow2_floor(S0 < 64 ? (S0 < NY ? S0 : NY) : 64);
  static constexpr int SEG = (NY + S - 1) / S;
  static constexpr int QM = (kOrder + S) / S;
};

// One pass: the model coefficients around (sy, sx) into coef (LDS), from
// the spectrum rows ky_lo <= ky < ky_hi (all rows: the full model; a range:
// its share, the coefficients being linear in the spectrum).  CX is the
// spectrum's element type (float2, or double2 in FP64 mode).  Frames are
// NY rows of NX (a_ky = 2 pi ky~ / NY, b_kx = 2 pi kx / NX, 1/N^2 becomes
// 1/(NY NX)).
template <int NY, int NX, typename CX>
__device__ __forceinline__ void build_model(const CX* __restrict__ Xf, double sy, double sx, double2* phy,
                            double* ay, double (*red)[kOrder + 1][kOrder + 1],
                            double (*nred)[2 * (kOrder + 1)], double* coef, int ky_lo = 0,
                            int ky_hi = NY) {
  using MS = ModelSplit<NY, NX>;
  constexpr int H = NX / 2 + 1;
  constexpr int NC = MS::NC, S = MS::S, QM = MS::QM;
  const double pi = 3.14159265358979323846;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int ky = tid; ky < NY; ky += kNThreads) {
    if (2 * ky == NY) {
      phy[ky] = make_double2(0.0, 0.0);  // the Nyquist row is added separately
      ay[ky] = 0.0;
    } else {
      const int kt = 2 * ky < NY ? ky : ky - NY;
      double sn, cs;
      sincospi(2.0 * (double)kt * sy / (double)NY, &sn, &cs);
      phy[ky] = make_double2(cs, sn);
      ay[ky] = 2.0 * pi * (double)kt / (double)NY;
    }
  }
  __syncthreads();
  // Nyquist row: Re[exp(i pi sy) (i pi)^n]
  double ry[kOrder + 1];
  {
    double sn, cs;
    sincospi(sy, &sn, &cs);
    double2 t = make_double2(cs, sn);
#pragma unroll
    for (int n = 0; n <= kOrder; ++n) {
      ry[n] = t.x;
      t = make_double2(-pi * t.y, pi * t.x);
    }
  }
  // ---- moments of column kx over this lane's ky segment
  const int kx = tid / S, seg = tid % S;
  double2 M[kOrder + 1];
#pragma unroll
  for (int n = 0; n <= kOrder; ++n) M[n] = make_double2(0.0, 0.0);
  if (kx < NC) {
    const int segl = (ky_hi - ky_lo + S - 1) / S;  // SEG for the full range
    const int y0 = ky_lo + seg * segl, y1 = min(ky_hi, y0 + segl);
    const CX* col = Xf + kx;
#pragma unroll 4
    for (int ky = y0; ky < y1; ++ky) {
      const CX xf = col[(size_t)ky * H];
      const double2 ph = phy[ky];
      add_powers(M, make_double2((double)xf.x * ph.x - (double)xf.y * ph.y,
                                 (double)xf.x * ph.y + (double)xf.y * ph.x),
                 ay[ky]);
    }
    if (y0 <= NY / 2 && NY / 2 < y1) {
      const CX xf = col[(size_t)(NY / 2) * H];
#pragma unroll
      for (int n = 0; n <= kOrder; ++n) {
        M[n].x += (double)xf.x * ry[n];
        M[n].y += (double)xf.y * ry[n];
      }
    }
  }
#pragma unroll
  for (int n = 0; n <= kOrder; ++n) {
    M[n].x = group_sum<S>(M[n].x);
    M[n].y = group_sum<S>(M[n].y);
  }
  // ---- this lane's share of the coefficients: m = seg + S q
  double acc[QM][kOrder + 1];
#pragma unroll
  for (int q = 0; q < QM; ++q)
#pragma unroll
    for (int n = 0; n <= kOrder; ++n) acc[q][n] = 0.0;
  if (kx < NC) {
    const double b = 2.0 * pi * (double)kx / (double)NX;
    const double w = kx == 0 ? 1.0 : 2.0;
    double sn, cs;
    sincospi(2.0 * (double)kx * sx / (double)NX, &sn, &cs);
    double2 P = make_double2(cs, sn);
    for (int k = 0; k < seg && k <= kOrder; ++k) P = make_double2(-b * P.y, b * P.x);
#pragma unroll
    for (int q = 0; q < QM; ++q) {
      const int m = seg + S * q;
      if (m <= kOrder) {
#pragma unroll
        for (int n = 0; n <= kOrder; ++n)
          if (n + m <= kOrder) acc[q][n] += w * (P.x * M[n].x - P.y * M[n].y);
      }
#pragma unroll
      for (int k = 0; k < S && k <= kOrder; ++k) P = make_double2(-b * P.y, b * P.x);
    }
  }
  // sum over the columns of each 16-lane row (lanes with the same seg); the
  // rows' partials (RP per wave) are added in the final sums
  constexpr int RW = S <= 16 ? 16 : 64, RP = 64 / RW;
  if constexpr (RW == 16) {
#pragma unroll
    for (int q = 0; q < QM; ++q)
#pragma unroll
      for (int n = 0; n <= kOrder; ++n) acc[q][n] = row_residue_sum<S>(acc[q][n]);
  } else {
#pragma unroll
    for (int off = S; off < RW; off <<= 1)
#pragma unroll
      for (int q = 0; q < QM; ++q)
#pragma unroll
        for (int n = 0; n <= kOrder; ++n) acc[q][n] += __shfl_xor(acc[q][n], off, 64);
  }
  if (lane % RW < S) {
#pragma unroll
    for (int q = 0; q < QM; ++q) {
      const int m = lane % RW + S * q;
      if (m <= kOrder)
#pragma unroll
        for (int n = 0; n <= kOrder; ++n) red[wave * RP + lane / RW][m][n] = acc[q][n];
    }
  }
  // ---- Nyquist column kx = NX/2: wave 0, one row per lane at a time
  double2 Mn[kOrder + 1];
#pragma unroll
  for (int n = 0; n <= kOrder; ++n) Mn[n] = make_double2(0.0, 0.0);
  for (int ky = ky_lo + (wave == 0 ? lane : ky_hi); ky < ky_hi; ky += 64) {
    const CX xf = Xf[(size_t)ky * H + NC];
    if (2 * ky == NY) {
#pragma unroll
      for (int n = 0; n <= kOrder; ++n) {
        Mn[n].x += (double)xf.x * ry[n];
        Mn[n].y += (double)xf.y * ry[n];
      }
    } else {
      const double2 ph = phy[ky];
      add_powers(Mn, make_double2((double)xf.x * ph.x - (double)xf.y * ph.y,
                                  (double)xf.x * ph.y + (double)xf.y * ph.x),
                 ay[ky]);
    }
  }
  if (wave == 0) {  // (the other waves hold zeros)
#pragma unroll
    for (int off = 1; off < 64; off <<= 1)
#pragma unroll
      for (int n = 0; n <= kOrder; ++n) {
        Mn[n].x += __shfl_xor(Mn[n].x, off, 64);
        Mn[n].y += __shfl_xor(Mn[n].y, off, 64);
      }
  }
  if (lane == 0)
#pragma unroll
    for (int n = 0; n <= kOrder; ++n) {
      nred[wave][2 * n] = Mn[n].x;
      nred[wave][2 * n + 1] = Mn[n].y;
    }
  __syncthreads();
  // ---- final sums, fixed order
  if (tid < kCoef) {
    int n = 0, m = tid;
    while (m > kOrder - n) {  // invert coef_index
      m -= kOrder + 1 - n;
      ++n;
    }
    double v = 0.0, mr = 0.0;
    for (int w = 0; w < kNThreads / 64 * RP; ++w) v += red[w][m][n];
    for (int w = 0; w < kNThreads / 64; ++w) mr += nred[w][2 * n];
    // Nyquist column: P_m = Re[exp(i pi sx) (i pi)^m], weight 1, real part of M_n
    double sn, cs;
    sincospi(sx, &sn, &cs);
    double2 P = make_double2(cs, sn);
    for (int k = 0; k < m; ++k) P = make_double2(-pi * P.y, pi * P.x);
    v += P.x * mr;
    coef[coef_index(n, m)] = v / ((double)NY * (double)NX);
  }
  __syncthreads();
}

__device__ void write_special(ccpt_result* out, unsigned status) {
  ccpt_result r;
  r.reserved = 0;
  const double v = status == CCPT_ST_NONFINITE ? __builtin_nan("") : 0.0;
  r.d[0] = r.d[1] = v;
  r.peak = v;
  r.hess[0] = r.hess[1] = r.hess[2] = v;
  r.d_grid[0] = r.d_grid[1] = (float)v;
  r.p[0] = r.p[1] = 0;
  r.status = status;
  *out = r;
}

// Integer peak (py, px) and grid estimate (dgy, dgx) of a frame from its
// state, in the axes of the tall image.
template <int NY, int NX>
__device__ void grid_seed(const GroupParams& g, const FrameState& st, int& py, int& px,
                          double& dgy, double& dgx) {
  peak_yx<NY, NX>(key_index(st.peak_key), g.trans, py, px);
  if (2 * py >= NY) py -= NY;
  if (2 * px >= NX) px -= NX;
  unsigned gk = key_index(st.grid_key);
  if (gk >= (unsigned)(g.M * g.M)) gk = (unsigned)(g.c * g.M + g.c);
  // (the grid index is the frame's row-major one: transposed for a wide frame)
  const bool tr = transposed<NY, NX>(g.trans);
  const int my = tr ? gk % g.M : gk / g.M, mx = tr ? gk / g.M : gk % g.M;
  dgy = py + (double)(my - g.c) / g.u;
  dgx = px + (double)(mx - g.c) / g.u;
}

// Small launches: block b of frame f builds the first model's share of the
// spectrum rows b NY / nb <= ky < (b + 1) NY / nb around the grid estimate
// and stores its coefficients to parts[f][b]; the Newton kernel adds the
// shares in block order.
template <int NY, int NX, typename CX>
__global__ void __launch_bounds__(kNThreads) k_newton_part(GroupParams g, double* __restrict__ parts,
                                                           int nb) {
  __shared__ double2 phy[NY];
  __shared__ double ay[NY];
  __shared__ double red[kNThreads / 16][kOrder + 1][kOrder + 1];
  __shared__ double nred[kNThreads / 64][2 * (kOrder + 1)];
  __shared__ double coef[kCoef];
  const int f = blockIdx.y, b = blockIdx.x, tid = threadIdx.x;
  const FrameState st = g.st[f];
  if ((st.flags & CCPT_ST_NONFINITE) || st.amin == st.amax) return;  // no model needed
  int py, px;
  double dgy, dgx;
  grid_seed<NY, NX>(g, st, py, px, dgy, dgx);
  const CX* Xf = (sizeof(CX) == sizeof(float2) ? (const CX*)g.X : (const CX*)g.X64) +
                 (size_t)f * NY * (NX / 2 + 1);
  build_model<NY, NX, CX>(Xf, dgy, dgx, phy, ay, red, nred, coef, b * NY / nb, (b + 1) * NY / nb);
  if (tid < kCoef) parts[((size_t)f * nb + b) * kCoef + tid] = coef[tid];
}

template <int NY, int NX, typename CX>
__global__ void __launch_bounds__(kNThreads) k_newton(GroupParams g, double step_limit,
                                                      const double* __restrict__ parts, int nb) {
  __shared__ double2 phy[NY];
  __shared__ double ay[NY];
  __shared__ double red[kNThreads / 16][kOrder + 1][kOrder + 1];
  __shared__ double nred[kNThreads / 64][2 * (kOrder + 1)];
  __shared__ double coef[kCoef];
  __shared__ double ctl[3];  // next centre y, x; another pass?
  const int f = blockIdx.x;
  const int tid = threadIdx.x;
  const FrameState st = g.st[f];
  const FrameDesc d = g.desc[g.first + f];
  ccpt_result* out = g.out + d.out_idx;
  // the state goes back to its initial value for the next chunk once every
  // thread has read it
  auto reset_state = [&]() {
    __syncthreads();
    if (tid == 0) {
      FrameState z;
      z.peak_key = 0;
      z.grid_key = 0;
      z.second_key = 0;
      z.amin = 0xFFFFFFFFu;
      z.amax = 0;
      z.flags = 0;
      z.pad = 0;
      g.st[f] = z;
    }
  };
  if (st.flags & CCPT_ST_NONFINITE) {
    if (tid == 0) write_special(out, CCPT_ST_NONFINITE);
    reset_state();
    return;
  }
  if (st.amin == st.amax) {
    if (tid == 0) write_special(out, CCPT_ST_FLAT);
    reset_state();
    return;
  }
  reset_state();
  int py, px;
  double dgy, dgx;
  grid_seed<NY, NX>(g, st, py, px, dgy, dgx);
  const CX* Xf = (sizeof(CX) == sizeof(float2) ? (const CX*)g.X : (const CX*)g.X64) +
                 (size_t)f * NY * (NX / 2 + 1);

  // the iterate and the decisions live in thread 0; the centre is broadcast
  double sy = dgy, sx = dgx;
  // near tie of the integer peak: flagged by the FP64 reduction, or from
  // the two largest FP32 keys
  unsigned status = st.flags & CCPT_ST_NEAR_TIE;
  if (st.second_key && near_tie((double)key_value(st.peak_key), (double)key_value(st.second_key)))
    status |= CCPT_ST_NEAR_TIE;
  bool done = false;
  bool checked = false;  // window test applied
  int it_left = g.newton_iters;
  double cy = dgy, cx = dgx;
  Deriv fin{0, 0, 0, 0, 0, 0};
  // iterations run in the first kMaxPasses model passes; one more pass may
  // re-centre the model on the final point (a window exit, or an iterate
  // still moving when the passes ran out) for C and the Hessian there
  for (int pass = 0; pass <= kMaxPasses; ++pass) {
    if (pass == 0 && parts) {
      // the first model from the blocks of k_newton_part, added in block order
      if (tid < kCoef) {
        double v = 0.0;
        for (int b = 0; b < nb; ++b) v += parts[((size_t)f * nb + b) * kCoef + tid];
        coef[tid] = v;
      }
      __syncthreads();
    } else {
      build_model<NY, NX, CX>(Xf, cy, cx, phy, ay, red, nred, coef);
    }
    if (tid == 0) {
      while (!done && it_left > 0) {
        const Deriv e = model_eval(coef, sy - cy, sx - cx);
        const double det = e.hyy * e.hxx - e.hxy * e.hxy;
        if (!(e.hyy < 0.0 && det > 0.0)) {
          status |= CCPT_ST_NEWTON_FALLBACK;
          sy = dgy;
          sx = dgx;
          done = true;
          break;
        }
        const double ty = -(e.hxx * e.gy - e.hxy * e.gx) / det;
        const double tx = -(e.hyy * e.gx - e.hxy * e.gy) / det;
        if (fmax(fabs(ty), fabs(tx)) > step_limit) {
          status |= CCPT_ST_NEWTON_FALLBACK;
          sy = dgy;
          sx = dgx;
          done = true;
          break;
        }
        sy += ty;
        sx += tx;
        --it_left;
        if (fmax(fabs(sy - cy), fabs(sx - cx)) > kModelRadius) break;  // rebuild around sy, sx
      }
      // out of steps or out of iterating passes: the iterate is final, and
      // the window test applies to it whether or not it converged
      if (it_left == 0 || pass >= kMaxPasses - 1) done = true;
      if (done && !checked) {
        checked = true;
        if (fmax(fabs(sy - py), fabs(sx - px)) > g.half_window) {
          status |= CCPT_ST_WINDOW_EXIT;
          sy = dgy;
          sx = dgx;
        }
      }
      const bool again = !done || fmax(fabs(sy - cy), fabs(sx - cx)) > kModelRadius;
      if (!again) fin = model_eval(coef, sy - cy, sx - cx);
      ctl[0] = sy;
      ctl[1] = sx;
      ctl[2] = again ? 1.0 : 0.0;
    }
    __syncthreads();
    const bool again = ctl[2] != 0.0;
    cy = ctl[0];
    cx = ctl[1];
    __syncthreads();
    if (!again) break;
  }
  if (tid == 0) {
    // in the frame's own axes (a wide frame was processed transposed)
    const int a = transposed<NY, NX>(g.trans) ? 1 : 0, b = 1 - a;
    ccpt_result r;
    r.reserved = 0;
    r.d[a] = sy;
    r.d[b] = sx;
    r.peak = fin.c;
    r.hess[2 * a] = fin.hyy;
    r.hess[1] = fin.hxy;
    r.hess[2 * b] = fin.hxx;
    r.d_grid[a] = (float)dgy;
    r.d_grid[b] = (float)dgx;
    r.p[a] = py;
    r.p[b] = px;
    r.status = status;
    *out = r;
  }
}

template <int NY, int NX>
static int newton_n(const GroupParams& g, double step_limit, hipStream_t s) {
  // few frames: the first model is built by kNewtonParts blocks per frame
  const bool split = g.nparts && g.count < kNewtonSplitMax;
  double* parts = split ? g.nparts : nullptr;
  const int nb = split ? kNewtonParts : 0;
  if (g.X64) {
    if (split)
      hipLaunchKernelGGL((k_newton_part<NY, NX, double2>), dim3(nb, g.count), dim3(kNThreads), 0,
                         s, g, parts, nb);
    hipLaunchKernelGGL((k_newton<NY, NX, double2>), dim3(g.count), dim3(kNThreads), 0, s, g,
                       step_limit, (const double*)parts, nb);
  } else {
    if (split)
      hipLaunchKernelGGL((k_newton_part<NY, NX, float2>), dim3(nb, g.count), dim3(kNThreads), 0,
                         s, g, parts, nb);
    hipLaunchKernelGGL((k_newton<NY, NX, float2>), dim3(g.count), dim3(kNThreads), 0, s, g,
                       step_limit, (const double*)parts, nb);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_newton(int ny, int nx, const GroupParams& g, double step_limit, hipStream_t s) {
  if (ny == nx) {
    switch (ny) {
#define CASE(n) \
  case n:       \
    return newton_n<n, n>(g, step_limit, s);
      CCPT_FOR_SIZES(CASE)
#undef CASE
    }
    return -2;
  }
#define CASE(a, b) \
  if (ny == a && nx == b) return newton_n<a, b>(g, step_limit, s);
  CCPT_FOR_RECT(CASE)
#undef CASE
  return -2;
}

}  // namespace ccpt
