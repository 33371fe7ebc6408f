// Upsampled matrix-multiply DFT around the integer peak and its maximum
// (Sec. III, first paragraph; the matrix DFT of Guizar-Sicairos et al.).
//
// With the cross-power spectrum X of a frame and its integer peak p, the
// band-limited correlation on the 1.5-px window is
//
//   U[my, mx] = 1/N^2 sum_kx w_kx Re[ phi_kx(dx_mx) Y[my, kx] ],
//   Y[my, kx] = sum_ky phi_ky(dy_my) X'[ky, kx],
//   X'[ky, kx] = X[ky, kx] exp(2 pi i (ky p_y + kx p_x) / N)       (phase fold)
//
// over the half spectrum kx = 0..N/2 (w = 1 at kx = 0 and N/2, else 2).  The
// fold makes the DFT tables K[m, ky] = phi_ky(dy_m) and W[j, mx] the same for
// every frame, so both stages are dense products with shared operands:
//
//   Stage A  (complex)  Y  = K  X'   : Mp x N  times N x N/2  on matrix cores,
//                                       plus the Nyquist column kx = N/2 on VALU
//   Stage B  (real)     U  = Ymat W  : Ymat[my, j] = Yr (j <= N/2), Yi (j > N/2)
//
// The imaginary parts of Y at kx = 0 and N/2 never enter U (their W is real),
// so Stage B's contraction length is exactly N.
//
// One block handles one 32-row tile of my for one frame; its grid maximum is
// merged into the frame's key with a 64-bit atomic max (value, lowest index).
#include <hip/hip_runtime.h>

#include "common.h"
#include "fft.h"

namespace ccpt {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kUThreads = 256;

template <typename T>
__device__ __forceinline__ T wmax64(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

__device__ __forceinline__ bool frame_skipped(const FrameState& s) {
  return (s.flags & CCPT_ST_NONFINITE) || s.amin == s.amax;
}

// ky-chunk of the Stage A contraction held in LDS: the largest divisor of N
// not above 32 (16 for the largest sizes, to bound LDS)
constexpr int a_chunk(int N) {
  const int cap = N >= 384 ? 16 : 32;
  int best = 1;
  for (int d = 1; d <= cap; ++d)
    if (N % d == 0) best = d;
  return best;
}

// ---------------------------------------------------------------- FP32
// K table: float2 [Mp][N]  (K[m][ky] = phi_ky((m - c)/u))
// W table: float  [Kb][Mp], Kb = N rounded up to 32 (zero rows past N)
template <int N>
__global__ void __launch_bounds__(kUThreads) k_updft_f32(GroupParams g, const float2* __restrict__ Ktab,
                                                         const float* __restrict__ Wtab, int Mp) {
  constexpr int H = N / 2 + 1;
  constexpr int NC = N / 2;                 // columns on matrix cores
  constexpr int NT = (NC + 31) / 32;        // 32-wide column tiles
  constexpr int TPW = (NT + 3) / 4;         // tiles per wave
  constexpr int KC = a_chunk(N);
  constexpr int XS = KC * H;                // folded X' chunk (float2)
  constexpr int KS = 32 * KC;               // K chunk (float2)
  constexpr int KB = (N + 31) / 32 * 32;    // Stage B contraction, zero padded
  constexpr int YS = 32 * KB / 2;           // Ymat as float2 count (32 x KB floats)
  constexpr int RAW = (XS + KS) > YS ? (XS + KS) : YS;
  __shared__ float2 raw[RAW];
  __shared__ float2 twf[N];                 // exp(+2 pi i m / N)
  __shared__ float nyq[8][32];
  __shared__ unsigned long long red[kUThreads / 64];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = blockIdx.y;
  const int m0 = blockIdx.x * 32;
  const FrameState st = g.st[f];
  if (frame_skipped(st)) return;
  unsigned pk = key_index(st.peak_key);
  if (pk >= (unsigned)(N * N)) pk = 0;  // never set: cannot happen for a frame that got here
  const int iy = pk / N, ix = pk % N;
  for (int i = tid; i < N; i += kUThreads) twf[i] = cconj(g.tw[i]);

  float2* xs = raw;
  float2* ks = raw + XS;
  const float2* Xf = g.X + (size_t)f * N * H;

  f32x16 accr[TPW], acci[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) accr[t][v] = acci[t][v] = 0.f;
  float nacc = 0.f;
  const int half = lane >> 5, l32 = lane & 31;
  __syncthreads();

  for (int k0 = 0; k0 < N; k0 += KC) {
    for (int i = tid; i < XS; i += kUThreads) {
      const int kk = i / H, kx = i - kk * H;
      const int ky = k0 + kk;
      float2 v = Xf[(size_t)ky * H + kx];
      v = cmul(v, twf[(ky * iy + kx * ix) % N]);
      if (ky == 0 && kx == 0) v = make_float2(0.f, 0.f);  // DC only shifts U by a constant
      xs[i] = v;
    }
    for (int i = tid; i < KS; i += kUThreads) {
      const int m = i / KC, kk = i - m * KC;
      ks[i] = Ktab[(size_t)(m0 + m) * N + k0 + kk];
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KC; ++kk) {
      const float2 kv = ks[l32 * KC + kk];
      const float ar = half ? -kv.y : kv.x;
      const float ai = half ? kv.x : kv.y;
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int kx = (wave + 4 * t) * 32 + l32;
        float b = 0.f;
        if (kx < NC) {
          const float2 xv = xs[kk * H + kx];
          b = half ? xv.y : xv.x;
        }
        accr[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, b, accr[t], 0, 0, 0);
        acci[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, b, acci[t], 0, 0, 0);
      }
    }
    // Nyquist column kx = N/2: Yr only
    {
      const int m = tid & 31, grp = tid >> 5;
      for (int kk = grp; kk < KC; kk += 8) {
        const float2 kv = ks[m * KC + kk];
        const float2 xv = xs[kk * H + NC];
        nacc += kv.x * xv.x - kv.y * xv.y;
      }
    }
    __syncthreads();
  }
  nyq[tid >> 5][tid & 31] = nacc;
  // Ymat[32][KB] (floats) aliases the chunk buffers
  float* ym = (float*)raw;
  for (int i = tid; i < 32 * (KB - N); i += kUThreads) {
    const int r = i / (KB - N), j = N + i % (KB - N);
    ym[r * KB + j] = 0.f;
  }
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int kx = (wave + 4 * t) * 32 + l32;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = (v >> 2) * 8 + half * 4 + (v & 3);
      if (kx < NC) ym[i * KB + kx] = accr[t][v];
      if (kx >= 1 && kx < NC) ym[i * KB + NC + kx] = acci[t][v];
    }
  }
  __syncthreads();
  if (tid < 32) {
    float s = 0.f;
    for (int q = 0; q < 8; ++q) s += nyq[q][tid];
    ym[tid * KB + NC] = s;
  }
  __syncthreads();

  // Stage B: U[32][Mp] = ym[32][KB] x W[KB][Mp], 16x16x4 tiles
  const int ntb = 2 * (Mp / 16);
  unsigned long long best = 0;
  const int l16 = lane & 15, q4 = lane >> 4;
  for (int T = wave; T < ntb; T += 4) {
    const int mt = T & 1, nt = T >> 1;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const float* arow = ym + (mt * 16 + l16) * KB + q4;
    const float* bcol = Wtab + (size_t)q4 * Mp + nt * 16 + l16;
#pragma unroll 8
    for (int k = 0; k < KB; k += 4) {
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(arow[k], bcol[(size_t)k * Mp], acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int my = m0 + mt * 16 + q4 * 4 + v;
      const int mx = nt * 16 + l16;
      if (my < g.M && mx < g.M) {
        const unsigned long long key = peak_key(acc[v], (unsigned)(my * g.M + mx));
        best = key > best ? key : best;
      }
    }
  }
  best = wmax64(best);
  if (lane == 0) red[wave] = best;
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < kUThreads / 64; ++w) best = red[w] > best ? red[w] : best;
    atomicMax(&g.st[f].grid_key, best);
  }
}

template <int N>
static int updft_n(const GroupParams& g, const UpdftTables& t, hipStream_t s) {
  const int mtiles = t.Mp / 32;
  if (t.precision == CCPT_PREC_FP32) {
    hipLaunchKernelGGL((k_updft_f32<N>), dim3(mtiles, g.count), dim3(kUThreads), 0, s, g,
                       (const float2*)t.ky, (const float*)t.wb, t.Mp);
  } else {
    return -2;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

#define CCPT_FOR_SIZES(X) \
  X(16) X(18) X(24) X(32) X(36) X(48) X(54) X(64) X(72) X(96) X(108) X(128) X(144) X(162) X(192) \
  X(216) X(256) X(288) X(324) X(384) X(432) X(486) X(512)

int launch_updft(int N, const GroupParams& g, const UpdftTables& t, hipStream_t s) {
  switch (N) {
#define CASE(n) \
  case n:       \
    return updft_n<n>(g, t, s);
    CCPT_FOR_SIZES(CASE)
#undef CASE
  }
  return -2;
}

}  // namespace ccpt
