// Upsampled matrix DFT of the FP64 (accuracy) mode, Sec. III first
// paragraph: the band-limited correlation sampled on the M x M grid
// p + (m - c)/u around the integer peak p,
//
//   U[my][mx] = 1/N^2 sum_kx w_kx Re[ Y'[my][kx] phi_kx(p_x + d_mx) ],
//   Y'[my][kx] = sum_ky phi_ky(p_y + d_my) X[ky][kx],
//
// with phi_k(s) = exp(2 pi i k~ s / N), cos(pi s) for a Nyquist bin, and
// w = 1 at kx = 0 and N/2, else 2.  For integer p, phi_k(p + d) =
// phi_k(p) phi_k(d) exactly (the Nyquist bin gives (-1)^p cos(pi d)), so the
// tables K[m][ky] = phi_ky(d_m) and W[kx][mx] = w phi_kx(d_mx) / N^2 stay
// frame independent and the peak phase is applied per frame.
//
// One block per frame, one thread per spectrum column kx; the grid rows are
// processed in chunks of kRC: Stage A accumulates kRC rows of Y' in
// registers (K tiles staged in LDS, X streamed from L2), Stage B contracts
// them with W into kRC grid rows and keeps the running maximum.  Everything
// is FP64 on the vector units: this mode trades speed for agreement with an
// FP64 definition.
//
// The integer peak arrives as one candidate per row block of the inverse
// row pass; the first step reduces them in a fixed order (ties to the lower
// row-major index), as the FP32 path's 64-bit atomic key does.
#include <hip/hip_runtime.h>

#include <math.h>

#include "common.h"
#include "fft.h"

namespace ccpt {

constexpr int kRC = 16;  // grid rows per chunk
constexpr int kKT = 32;  // ky per staged K tile

// phi_k(p) for an integer p: exp(2 pi i (k p mod N) / N), which is also the
// Nyquist bin's (-1)^p (sinpi of an integer is exactly zero).
__device__ __forceinline__ double2 phase_int(int k, int p, int N) {
  long t = ((long)k * (long)p) % N;
  if (t < 0) t += N;
  double sn, cs;
  sincospi(2.0 * (double)t / (double)N, &sn, &cs);
  return make_double2(cs, sn);
}

template <int N>
constexpr int updft64_threads() {
  return ((N / 2 + 1) + 63) / 64 * 64;
}

template <int N>
__global__ void __launch_bounds__(updft64_threads<N>())
    k_updft_f64(GroupParams g, const double2* __restrict__ K, const double2* __restrict__ W,
                int Mp, int nb) {
  constexpr int H = N / 2 + 1;
  constexpr int BD = updft64_threads<N>();
  constexpr int NW = BD / 64;
  __shared__ double2 fy[N];
  __shared__ double2 fx[H];
  __shared__ double2 Ks[kRC][kKT];
  __shared__ double2 Ys[kRC][H];
  __shared__ double rv[NW];
  __shared__ unsigned ri[NW];
  __shared__ int pk[2];
  const int f = blockIdx.x;
  const int tid = threadIdx.x;
  const int M = g.M;
  FrameState* st = g.st + f;

  double bv = -__builtin_inf();
  unsigned bi = 0xFFFFFFFFu;
  auto take = [&](double v, unsigned i) {
    if (v > bv || (v == bv && i < bi)) {
      bv = v;
      bi = i;
    }
  };

  if (tid == 0) {
    const PeakCand* cd = g.cand + (size_t)f * nb;
    // runner-up: the largest block runner-up or a block maximum that lost
    double sv = -__builtin_inf();
    for (int j = 0; j < nb; ++j) {
      const double v = cd[j].v;
      const unsigned i = cd[j].idx;
      if (v > bv || (v == bv && i < bi)) {
        sv = bv > sv ? bv : sv;
        bv = v;
        bi = i;
      } else if (v > sv) {
        sv = v;
      }
      sv = cd[j].v2 > sv ? cd[j].v2 : sv;
    }
    st->peak_key = peak_key((float)bv, bi);
    if (near_tie(bv, sv)) st->flags |= CCPT_ST_NEAR_TIE;
    const unsigned q = bi < (unsigned)(N * N) ? bi : 0u;
    int py = (int)(q / N), px = (int)(q % N);
    if (2 * py >= N) py -= N;
    if (2 * px >= N) px -= N;
    pk[0] = py;
    pk[1] = px;
    bv = -__builtin_inf();
    bi = 0xFFFFFFFFu;
  }
  __syncthreads();
  const int py = pk[0], px = pk[1];
  for (int k = tid; k < N; k += BD) fy[k] = phase_int(k, py, N);
  for (int k = tid; k < H; k += BD) fx[k] = phase_int(k, px, N);
  __syncthreads();

  const double2* Xf = g.X64 + (size_t)f * N * H;
  const int kx = tid;
  const double2 zero = make_double2(0.0, 0.0);
  for (int m0 = 0; m0 < M; m0 += kRC) {
    // ---- Stage A: rows m0 .. m0 + kRC - 1 of Y' for column kx
    double2 acc[kRC];
#pragma unroll
    for (int r = 0; r < kRC; ++r) acc[r] = zero;
    for (int ky0 = 0; ky0 < N; ky0 += kKT) {
      __syncthreads();
      for (int i = tid; i < kRC * kKT; i += BD) {
        const int r = i / kKT, j = i - r * kKT;
        const int m = m0 + r, ky = ky0 + j;
        Ks[r][j] = (m < M && ky < N) ? cmul(K[(size_t)m * N + ky], fy[ky]) : zero;
      }
      __syncthreads();
      if (kx < H) {
        const int jn = min(kKT, N - ky0);
        for (int j = 0; j < jn; ++j) {
          const double2 xv = Xf[(size_t)(ky0 + j) * H + kx];
#pragma unroll
          for (int r = 0; r < kRC; ++r) {
            const double2 kv = Ks[r][j];
            acc[r].x = fma(kv.x, xv.x, fma(-kv.y, xv.y, acc[r].x));
            acc[r].y = fma(kv.x, xv.y, fma(kv.y, xv.x, acc[r].y));
          }
        }
      }
    }
    if (kx < H) {
      const double2 ph = fx[kx];
#pragma unroll
      for (int r = 0; r < kRC; ++r) Ys[r][kx] = cmul(acc[r], ph);
    }
    __syncthreads();
    // ---- Stage B: grid rows m0 .. m0 + kRC - 1, columns mx
    for (int mx = tid; mx < M; mx += BD) {
      double u[kRC];
#pragma unroll
      for (int r = 0; r < kRC; ++r) u[r] = 0.0;
      for (int k = 0; k < H; ++k) {
        const double2 w = W[(size_t)k * Mp + mx];
#pragma unroll
        for (int r = 0; r < kRC; ++r) u[r] = fma(Ys[r][k].x, w.x, fma(-Ys[r][k].y, w.y, u[r]));
      }
#pragma unroll
      for (int r = 0; r < kRC; ++r)
        if (m0 + r < M) take(u[r], (unsigned)((m0 + r) * M + mx));
    }
  }
  // ---- grid maximum of the block
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) take(__shfl_xor(bv, o, 64), (unsigned)__shfl_xor((int)bi, o, 64));
  if ((tid & 63) == 0) {
    rv[tid >> 6] = bv;
    ri[tid >> 6] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < NW; ++w) take(rv[w], ri[w]);
    st->grid_key = peak_key((float)bv, bi);
  }
}

template <int N>
static int updft64_n(const GroupParams& g, const double2* K, const double2* W, int Mp,
                     hipStream_t s) {
  hipLaunchKernelGGL((k_updft_f64<N>), dim3(g.count), dim3(updft64_threads<N>()), 0, s, g, K, W,
                     Mp, N / row_block64(N));
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_updft64(int N, const GroupParams& g, const double2* K, const double2* W, int Mp,
                   hipStream_t s) {
  switch (N) {
#define CASE(n) \
  case n:       \
    return updft64_n<n>(g, K, W, Mp, s);
    CCPT_FOR_SIZES(CASE)
#undef CASE
  }
  return -2;
}

}  // namespace ccpt
