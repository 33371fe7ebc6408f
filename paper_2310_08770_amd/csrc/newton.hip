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

constexpr int kNThreads = 256;  // three blocks (frames) per CU: one frame's serial phases overlap the others' loops
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
// columns.  Rows are taken in conjugate pairs q = 1 .. NY/2-1 (rows q and
// NY-q, whose phases and frequencies are conjugate and opposite), plus the
// pair q = 0 of the two rows that pair with themselves (0 and the Nyquist
// row NY/2).  Each column kx < NX/2 is shared by S adjacent lanes (pair
// segments of length SEG), at least four, the block taking its columns in
// NCG groups of CPG; after a column's moments are combined, lane `seg`
// accumulates its share of the coefficients, m = seg, seg + S, ... (QM of
// them), over the lane's columns.
// Spectrum values are loaded in batches of up to 4 pairs, the next batch in
// flight while the current one is summed.
template <int NY, int NX>
struct ModelSplit {
  static constexpr int NC = NX / 2;
  static constexpr int NQ = NY / 2;  // row pairs
  static constexpr int S0 = kNThreads / NC < 4 ? 4 : kNThreads / NC;
  static constexpr int S = pow2_floor(S0 < 64 ? (S0 < NQ ? S0 : NQ) : 64);
  static constexpr int CPG = kNThreads / S;          // columns per group
  static constexpr int NCG = (NC + CPG - 1) / CPG;   // column groups, one after the other
  static constexpr int SEG = (NQ + S - 1) / S;
  static constexpr int QM = (kOrder + S) / S;
  // pairs per lane in one of the kNewtonParts shares of a split model
  static constexpr int SEGP = ((NQ + kNewtonParts - 1) / kNewtonParts + S - 1) / S;
};

// One pass: the model coefficients around (sy, sx) into coef (LDS), from
// the row pairs q_lo <= q < q_hi (all pairs: the full model; a range: its
// share, the coefficients being linear in the spectrum).  CX is the
// spectrum's element type (float2, or double2 in FP64 mode).  Frames are
// NY rows of NX (a_ky = 2 pi ky~ / NY, b_kx = 2 pi kx / NX, 1/N^2 becomes
// 1/(NY NX)).
//
// The lane's first pair and a zero offset pass through an empty asm
// statement in every column group, so that the compiler forms the per-lane
// offsets, frequencies and their powers where they are used instead of
// hoisting them out of the column-group and re-centring loops (hundreds of
// registers).
//
// For a pair q >= 1 with t1 = X[q] phi_q(sy), t2 = X[NY-q] conj(phi_q(sy))
// and a = a_q, the two rows add (i a)^n (t1 + (-1)^n t2) to M_n; the sums
// R_n + i I_n = sum a^n (t1 +- t2) are accumulated with FMAs on real powers
// and M_n = i^n (R_n + i I_n) is formed once per column.
template <int NY, int NX, typename CX, int SEGL = ModelSplit<NY, NX>::SEG>
__device__ __forceinline__ void build_model(const CX* __restrict__ Xf, double sy, double sx, double2* phy,
                            double (*red)[kOrder + 1][kOrder + 1],
                            double (*nred)[2 * (kOrder + 1)], double* coef, int q_lo = 0,
                            int q_hi = NY / 2) {
  using MS = ModelSplit<NY, NX>;
  constexpr int H = NX / 2 + 1;
  constexpr int NC = MS::NC, NQ = MS::NQ, S = MS::S, QM = MS::QM;
  const double pi = 3.14159265358979323846;
  const double a_unit = 2.0 * pi / (double)NY;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int q = tid; q < NQ; q += kNThreads) {
    double sn, cs;
    sincospi(2.0 * (double)q * sy / (double)NY, &sn, &cs);
    phy[q] = make_double2(cs, sn);
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
  const int seg = tid % S;
  double acc[QM][kOrder + 1];
#pragma unroll
  for (int q = 0; q < QM; ++q)
#pragma unroll
    for (int n = 0; n <= kOrder; ++n) acc[q][n] = 0.0;
#pragma unroll 1
  for (int cg = 0; cg < MS::NCG; ++cg) {
  // ---- moments of column kx over this lane's pair segment
  const int kx = cg * MS::CPG + tid / S;
  double R[kOrder + 1], I[kOrder + 1];
#pragma unroll
  for (int n = 0; n <= kOrder; ++n) R[n] = I[n] = 0.0;
  if (kx < NC) {
    // this lane's pairs qa <= q < qb (at most SEGL of them); q = 0 stands for
    // row 0 (phase 1, a = 0) and the Nyquist row, which is loaded in the
    // second slot and added separately
    const int segl = (q_hi - q_lo + S - 1) / S;
    int qa = q_lo + seg * segl;
    const int qb = min(q_hi, qa + segl);
    // (32-bit offsets from the frame's uniform base)
    unsigned fo = 0;
    asm volatile("" : "+s"(fo), "+v"(qa));
    constexpr int BQ = SEGL < 4 ? SEGL : 4;
    constexpr int NB = (SEGL + BQ - 1) / BQ;
    CX b0[2 * BQ], b1[2 * BQ];
    // unconditional loads from clamped addresses (no branches between the
    // loads, so the next batch stays in flight while this one is summed);
    // values past the segment are masked where they are used
    auto load = [&](CX* b, int base) {
#pragma unroll
      for (int e = 0; e < BQ; ++e) {
        const int q = min(base + e, NQ - 1);
        b[2 * e] = Xf[fo + (unsigned)(q * H + kx)];
        b[2 * e + 1] = Xf[fo + (unsigned)((q == 0 ? NQ : NY - q) * H + kx)];
      }
    };
    auto sum = [&](const CX* b, int base) {
#pragma unroll
      for (int e = 0; e < BQ; ++e) {
        const int q = base + e;
        const bool v1 = q < qb, v2 = v1 && q > 0;
        const double2 ph = phy[min(q, NQ - 1)];
        const double x1 = v1 ? (double)b[2 * e].x : 0.0, y1 = v1 ? (double)b[2 * e].y : 0.0;
        const double x2 = v2 ? (double)b[2 * e + 1].x : 0.0, y2 = v2 ? (double)b[2 * e + 1].y : 0.0;
        const double t1x = x1 * ph.x - y1 * ph.y, t1y = x1 * ph.y + y1 * ph.x;
        const double t2x = x2 * ph.x + y2 * ph.y, t2y = y2 * ph.x - x2 * ph.y;
        const double sxv = t1x + t2x, syv = t1y + t2y, dxv = t1x - t2x, dyv = t1y - t2y;
        const double a = (double)q * a_unit;
        double pw = 1.0;
#pragma unroll
        for (int n = 0; n <= kOrder; ++n) {
          R[n] = fma((n & 1) ? dxv : sxv, pw, R[n]);
          I[n] = fma((n & 1) ? dyv : syv, pw, I[n]);
          pw *= a;
        }
      }
    };
    load(b0, qa);
    // a rolled loop: two batches live at a time (unrolled, the scheduler
    // hoists every load and runs out of registers)
#pragma unroll 1
    for (int bi = 0; bi < NB; bi += 2) {
      if (bi + 1 < NB) load(b1, qa + (bi + 1) * BQ);
      sum(b0, qa + bi * BQ);
      if (bi == 0) {
        // the Nyquist row (second slot of pair 0, masked elsewhere; no branch),
        // rotated by (-i)^n into the R + i I form
        const bool nq = qa == 0 && qb > 0;
        const double xn = nq ? (double)b0[1].x : 0.0, yn = nq ? (double)b0[1].y : 0.0;
#pragma unroll
        for (int n = 0; n <= kOrder; ++n) {
          const double vx = xn * ry[n], vy = yn * ry[n];
          switch (n & 3) {
            case 0: R[n] += vx; I[n] += vy; break;
            case 1: R[n] += vy; I[n] -= vx; break;
            case 2: R[n] -= vx; I[n] -= vy; break;
            default: R[n] -= vy; I[n] += vx; break;
          }
        }
      }
      if (bi + 1 < NB) {
        if (bi + 2 < NB) load(b0, qa + (bi + 2) * BQ);
        sum(b1, qa + (bi + 1) * BQ);
      }
    }
  }
  double2 M[kOrder + 1];
#pragma unroll
  for (int n = 0; n <= kOrder; ++n) {
    const double r = group_sum<S>(R[n]), i = group_sum<S>(I[n]);
    switch (n & 3) {  // M_n = i^n (R_n + i I_n)
      case 0: M[n] = make_double2(r, i); break;
      case 1: M[n] = make_double2(-i, r); break;
      case 2: M[n] = make_double2(-r, -i); break;
      default: M[n] = make_double2(i, -r); break;
    }
  }
  // ---- this lane's share of the coefficients: m = seg + S q
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
  // ---- Nyquist column kx = NX/2: wave 0, one row pair per lane at a time
  double2 Mn[kOrder + 1];
#pragma unroll
  for (int n = 0; n <= kOrder; ++n) Mn[n] = make_double2(0.0, 0.0);
  for (int q = q_lo + (wave == 0 ? lane : q_hi); q < q_hi; q += 64) {
    if (q == 0) {
      const CX x0 = Xf[NC], xn = Xf[(size_t)NQ * H + NC];
      Mn[0].x += (double)x0.x;
      Mn[0].y += (double)x0.y;
#pragma unroll
      for (int n = 0; n <= kOrder; ++n) {
        Mn[n].x += (double)xn.x * ry[n];
        Mn[n].y += (double)xn.y * ry[n];
      }
    } else {
      const double2 ph = phy[q];
      const double a = (double)q * a_unit;
      const CX x1 = Xf[(size_t)q * H + NC], x2 = Xf[(size_t)(NY - q) * H + NC];
      add_powers(Mn, make_double2((double)x1.x * ph.x - (double)x1.y * ph.y,
                                  (double)x1.x * ph.y + (double)x1.y * ph.x), a);
      add_powers(Mn, make_double2((double)x2.x * ph.x + (double)x2.y * ph.y,
                                  (double)x2.y * ph.x - (double)x2.x * ph.y), -a);
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
// row pairs b (NY/2) / nb <= q < (b + 1) (NY/2) / nb around the grid estimate
// and stores its coefficients to parts[f][b]; the Newton kernel adds the
// shares in block order.
template <int NY, int NX, typename CX>
__global__ void __launch_bounds__(kNThreads) k_newton_part(GroupParams g, double* __restrict__ parts,
                                                           int nb) {
  __shared__ double2 phy[NY / 2];
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
  build_model<NY, NX, CX, ModelSplit<NY, NX>::SEGP>(Xf, dgy, dgx, phy, red, nred, coef, b * (NY / 2) / nb,
                          (b + 1) * (NY / 2) / nb);
  if (tid < kCoef) parts[((size_t)f * nb + b) * kCoef + tid] = coef[tid];
}

template <int NY, int NX, typename CX>
__global__ void __launch_bounds__(kNThreads, 3) k_newton(GroupParams g, double step_limit,
                                                      const double* __restrict__ parts, int nb) {
  __shared__ double2 phy[NY / 2];
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
      z.xmax = 0;
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
  // still moving when the passes ran out) for C and the Hessian there.
  // After each pass thread 0 iterates on the model and says whether another
  // pass is needed.  The first pass, which every frame runs, is outside the
  // loop of re-centring passes, which few frames need.
  auto iterate = [&](int pass) -> bool {
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
    return again;
  };
  if (parts) {
    // the first model from the blocks of k_newton_part, added in block order
    if (tid < kCoef) {
      double v = 0.0;
      for (int b = 0; b < nb; ++b) v += parts[((size_t)f * nb + b) * kCoef + tid];
      coef[tid] = v;
    }
    __syncthreads();
  } else {
    build_model<NY, NX, CX>(Xf, cy, cx, phy, red, nred, coef);
  }
  bool again = iterate(0);
  for (int pass = 1; again && pass <= kMaxPasses; ++pass) {
    build_model<NY, NX, CX>(Xf, cy, cx, phy, red, nred, coef);
    again = iterate(pass);
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
