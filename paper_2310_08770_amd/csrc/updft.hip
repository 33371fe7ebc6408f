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


// ---------------------------------------------------------------- BF16 x 2
// Split precision: every operand x is carried as bf16 hi + lo (x ~ hi + lo to
// ~16 significant bits) and each product as hi*hi + hi*lo + lo*hi, accumulated
// in FP32 on the matrix cores (the lo*lo term is below the FP32 rounding of
// the sum).  The frame's X arrives already split (unfolded, DC dropped) from
// the column FFT; the integer-peak phase is folded into the shared K table
// instead: K'[m, ky] = K[m, ky] exp(2 pi i ky p_y / N) (split per block), and
// the kx phase exp(2 pi i kx p_x / N) multiplies Y after Stage A.
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 as_bf(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }
// (re, im) word pairs -> (re, -im)
__device__ __forceinline__ u32x4 neg_im(u32x4 w) { return w ^ 0x80000000u; }
// (re, im) word pairs -> (im, re)
__device__ __forceinline__ u32x4 swap_ri(u32x4 w) { return (w >> 16) | (w << 16); }

// Stage B operand: W^T as bf16 planes [2][Mp][KB] (hi, lo)
template <int N>
__global__ void __launch_bounds__(kUThreads) k_updft_bf16x2(GroupParams g, const float2* __restrict__ Ktab,
                                                            const unsigned short* __restrict__ WbT, int Mp) {
  constexpr int H = N / 2 + 1;
  constexpr int NC = N / 2;
  constexpr int NT = (NC + 31) / 32;
  constexpr int TPW = (NT + 3) / 4;
  constexpr int P = xb_pitch(N);
  constexpr int KC = N >= 384 ? 16 : 32;   // ky per LDS chunk (multiple of 8)
  constexpr int KCS = KC + 4;              // LDS row stride, words
  constexpr int XROWS = NT * 32;
  constexpr int KB = (N + 31) / 32 * 32;
  constexpr int YST = KB + 8;              // Ymat row stride, bf16 elements
  constexpr int XW = 2 * XROWS * KCS;
  constexpr int KW = 2 * 32 * KCS;
  constexpr int YW = 32 * YST;             // two bf16 planes of 32 x YST
  constexpr int RAWW = (XW + KW) > YW ? (XW + KW) : YW;
  __shared__ __attribute__((aligned(16))) unsigned raw[RAWW];
  __shared__ float2 kf[32][KC + 1];
  __shared__ float2 twf[N];
  __shared__ float nyq[8][32];
  __shared__ unsigned long long red[kUThreads / 64];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = blockIdx.y;
  const int m0 = blockIdx.x * 32;
  const FrameState st = g.st[f];
  if (frame_skipped(st)) return;
  unsigned pk = key_index(st.peak_key);
  if (pk >= (unsigned)(N * N)) pk = 0;
  const int iy = pk / N, ix = pk % N;
  for (int i = tid; i < N; i += kUThreads) twf[i] = cconj(g.tw[i]);

  unsigned* xs_hi = raw;
  unsigned* xs_lo = raw + XROWS * KCS;
  unsigned* ks_hi = raw + XW;
  unsigned* ks_lo = ks_hi + 32 * KCS;
  const unsigned* Xbh = g.Xb + (size_t)f * 2 * NC * P;
  const unsigned* Xbl = Xbh + (size_t)NC * P;
  const float2* Xf = g.X + (size_t)f * N * H;

  f32x16 accr[TPW], acci[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) accr[t][v] = acci[t][v] = 0.f;
  float nacc = 0.f;
  const int h = lane >> 5, j = lane & 31;
  __syncthreads();

  for (int k0 = 0; k0 < P; k0 += KC) {
    for (int i = tid; i < XROWS * (KC / 4); i += kUThreads) {
      const int r = i / (KC / 4), q = i - r * (KC / 4);
      u32x4 vh = {0u, 0u, 0u, 0u}, vl = {0u, 0u, 0u, 0u};
      if (r < NC) {
        vh = *(const u32x4*)(Xbh + (size_t)r * P + k0 + 4 * q);
        vl = *(const u32x4*)(Xbl + (size_t)r * P + k0 + 4 * q);
      }
      *(u32x4*)(xs_hi + r * KCS + 4 * q) = vh;
      *(u32x4*)(xs_lo + r * KCS + 4 * q) = vl;
    }
    for (int i = tid; i < 32 * KC; i += kUThreads) {
      const int m = i / KC, kk = i - m * KC;
      const int ky = k0 + kk;
      float2 kv = make_float2(0.f, 0.f);
      if (ky < N) kv = cmul(Ktab[(size_t)(m0 + m) * N + ky], twf[(ky * iy) % N]);
      kf[m][kk] = kv;
      unsigned wh, wl;
      split_pair(kv, wh, wl);
      ks_hi[m * KCS + kk] = wh;
      ks_lo[m * KCS + kk] = wl;
    }
    __syncthreads();
#pragma unroll
    for (int s8 = 0; s8 < KC / 8; ++s8) {
      const int col = s8 * 8 + 4 * h;
      const u32x4 ah = *(const u32x4*)(ks_hi + j * KCS + col);
      const u32x4 al = *(const u32x4*)(ks_lo + j * KCS + col);
      const bf16x8 arh = as_bf(neg_im(ah)), aih = as_bf(swap_ri(ah));
      const bf16x8 arl = as_bf(neg_im(al)), ail = as_bf(swap_ri(al));
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        if (wave + 4 * t < NT) {
          const int row = (wave + 4 * t) * 32 + j;
          const bf16x8 bh = as_bf(*(const u32x4*)(xs_hi + row * KCS + col));
          const bf16x8 bl = as_bf(*(const u32x4*)(xs_lo + row * KCS + col));
          accr[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, bh, accr[t], 0, 0, 0);
          accr[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, bl, accr[t], 0, 0, 0);
          accr[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arl, bh, accr[t], 0, 0, 0);
          acci[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, bh, acci[t], 0, 0, 0);
          acci[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, bl, acci[t], 0, 0, 0);
          acci[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ail, bh, acci[t], 0, 0, 0);
        }
      }
    }
    {  // Nyquist column kx = N/2 in FP32 on the VALU
      const int m = tid & 31, grp = tid >> 5;
      for (int kk = grp; kk < KC; kk += 8) {
        const int ky = k0 + kk;
        if (ky < N) {
          const float2 kv = kf[m][kk];
          const float2 xv = Xf[(size_t)ky * H + NC];
          nacc += kv.x * xv.x - kv.y * xv.y;
        }
      }
    }
    __syncthreads();
  }
  nyq[tid >> 5][tid & 31] = nacc;
  // kx phase of the fold
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    if (wave + 4 * t < NT) {
      const int kx = (wave + 4 * t) * 32 + j;
      const float2 ph = twf[(kx * ix) % N];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float yr = accr[t][v], yi = acci[t][v];
        accr[t][v] = yr * ph.x - yi * ph.y;
        acci[t][v] = yr * ph.y + yi * ph.x;
      }
    }
  }
  unsigned short* ymh = (unsigned short*)raw;
  unsigned short* yml = ymh + 32 * YST;
  for (int i = tid; i < 32 * (KB - N); i += kUThreads) {
    const int r = i / (KB - N), c = N + i % (KB - N);
    ymh[r * YST + c] = 0;
    yml[r * YST + c] = 0;
  }
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int kx = (wave + 4 * t) * 32 + j;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = (v >> 2) * 8 + h * 4 + (v & 3);
      if (kx < NC) {
        const unsigned a = bf16_bits(accr[t][v]);
        ymh[i * YST + kx] = (unsigned short)a;
        yml[i * YST + kx] = (unsigned short)bf16_bits(accr[t][v] - bf16_float(a));
      }
      if (kx >= 1 && kx < NC) {
        const unsigned b = bf16_bits(acci[t][v]);
        ymh[i * YST + NC + kx] = (unsigned short)b;
        yml[i * YST + NC + kx] = (unsigned short)bf16_bits(acci[t][v] - bf16_float(b));
      }
    }
  }
  __syncthreads();
  if (tid < 32) {
    float sacc = 0.f;
    for (int q = 0; q < 8; ++q) sacc += nyq[q][tid];
    if (ix & 1) sacc = -sacc;  // exp(i pi p_x)
    const unsigned a = bf16_bits(sacc);
    ymh[tid * YST + NC] = (unsigned short)a;
    yml[tid * YST + NC] = (unsigned short)bf16_bits(sacc - bf16_float(a));
  }
  __syncthreads();

  // Stage B: U[32][Mp] = Ymat[32][KB] x W[KB][Mp] on 16x16x32 bf16 tiles
  const int ntb = 2 * (Mp / 16);
  unsigned long long best = 0;
  const int l16 = lane & 15, q4 = lane >> 4;
  const unsigned short* WbL = WbT + (size_t)Mp * KB;
  for (int T = wave; T < ntb; T += 4) {
    const int mt = T & 1, nt = T >> 1;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const unsigned short* ah_p = ymh + (mt * 16 + l16) * YST + 8 * q4;
    const unsigned short* al_p = yml + (mt * 16 + l16) * YST + 8 * q4;
    const unsigned short* bh_p = WbT + (size_t)(nt * 16 + l16) * KB + 8 * q4;
    const unsigned short* bl_p = WbL + (size_t)(nt * 16 + l16) * KB + 8 * q4;
#pragma unroll 4
    for (int k = 0; k < KB; k += 32) {
      const bf16x8 ah = as_bf(*(const u32x4*)(ah_p + k));
      const bf16x8 al = as_bf(*(const u32x4*)(al_p + k));
      const bf16x8 bh = as_bf(*(const u32x4*)(bh_p + k));
      const bf16x8 bl = as_bf(*(const u32x4*)(bl_p + k));
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
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


// Wide variant for N >= 256: one block per frame and group of up to MT
// 32-row m-tiles, one wave per 32-column kx tile.  Each frame's split
// spectrum is streamed once from memory straight into the B operands (no
// LDS staging, each fragment feeds 6 MT matrix instructions); the folded
// K' rows of the block are built per 32-ky chunk in LDS and shared by all
// waves.  The Nyquist column is accumulated in FP32 by the thread that
// builds the row.  Stage B then runs m-tile by m-tile.
template <int N, int MT>
__global__ void __launch_bounds__(64 * ((N / 2 + 31) / 32))
    k_updft_bf16x2_wide(GroupParams g, const float2* __restrict__ Ktab,
                        const unsigned short* __restrict__ WbT, int Mp) {
  constexpr int H = N / 2 + 1;
  constexpr int NC = N / 2;
  constexpr int NW = (NC + 31) / 32;  // waves = kx tiles
  constexpr int NTH = 64 * NW;
  constexpr int P = xb_pitch(N);
  constexpr int KC = 32;
  constexpr int KCS = KC + 4;
  constexpr int ROWS = MT * 32;
  constexpr int KB = (N + 31) / 32 * 32;
  constexpr int YST = KB + 8;
  constexpr int KW = 2 * ROWS * KCS;
  constexpr int YW = 32 * YST;
  constexpr int RAWW = KW > YW ? KW : YW;
  static_assert(ROWS <= NTH, "one thread per K' row");
  __shared__ __attribute__((aligned(16))) unsigned raw[RAWW];
  __shared__ float2 twf[N];
  __shared__ float2 xnyq[N];  // Nyquist column X[ky, N/2] of the frame
  __shared__ float nyq[ROWS];
  __shared__ unsigned long long red[NW];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = blockIdx.y;
  const int m0 = blockIdx.x * ROWS;
  const int mt_here = min(MT, (Mp - m0) / 32);
  const FrameState st = g.st[f];
  if (frame_skipped(st)) return;
  unsigned pk = key_index(st.peak_key);
  if (pk >= (unsigned)(N * N)) pk = 0;
  const int iy = pk / N, ix = pk % N;
  for (int i = tid; i < N; i += NTH) {
    twf[i] = cconj(g.tw[i]);
    xnyq[i] = g.X[(size_t)f * N * H + (size_t)i * H + NC];
  }

  unsigned* ks_hi = raw;
  unsigned* ks_lo = raw + ROWS * KCS;
  const unsigned* Xbh = g.Xb + (size_t)f * 2 * NC * P;
  const unsigned* Xbl = Xbh + (size_t)NC * P;
  const int h = lane >> 5, j = lane & 31;
  const int kxrow = wave * 32 + j;
  const bool bvalid = kxrow < NC;

  f32x16 accr[MT], acci[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) accr[t][v] = acci[t][v] = 0.f;
  float nacc = 0.f;
  const bool krow = tid < mt_here * 32;
  __syncthreads();

  for (int k0 = 0; k0 < P; k0 += KC) {
    u32x4 bh[KC / 8], bl[KC / 8];
#pragma unroll
    for (int s8 = 0; s8 < KC / 8; ++s8) {
      const int col = k0 + s8 * 8 + 4 * h;
      if (bvalid) {
        bh[s8] = *(const u32x4*)(Xbh + (size_t)kxrow * P + col);
        bl[s8] = *(const u32x4*)(Xbl + (size_t)kxrow * P + col);
      } else {
        bh[s8] = u32x4{0u, 0u, 0u, 0u};
        bl[s8] = u32x4{0u, 0u, 0u, 0u};
      }
    }
    if (krow) {
      // this thread's K row segment, fetched with 16-byte loads before use
      const int m = tid;
      const float4* krow_p = (const float4*)(Ktab + (size_t)(m0 + m) * N + k0);
      constexpr int Q = KC / 2;  // float4 = two complex values
      float4 kq[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q)
        kq[q] = (k0 + 2 * q < N) ? krow_p[q] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int q = 0; q < Q; ++q) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int kk = 2 * q + e;
          const int ky = k0 + kk;
          float2 kv = make_float2(0.f, 0.f);
          if (ky < N) {
            const float2 kr = e ? make_float2(kq[q].z, kq[q].w) : make_float2(kq[q].x, kq[q].y);
            kv = cmul(kr, twf[(ky * iy) % N]);
            const float2 xn = xnyq[ky];
            nacc += kv.x * xn.x - kv.y * xn.y;
          }
          unsigned wh, wl;
          split_pair(kv, wh, wl);
          ks_hi[m * KCS + kk] = wh;
          ks_lo[m * KCS + kk] = wl;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int s8 = 0; s8 < KC / 8; ++s8) {
      const int col = s8 * 8 + 4 * h;
      const bf16x8 b_h = as_bf(bh[s8]), b_l = as_bf(bl[s8]);
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        if (t < mt_here) {
          const u32x4 ah = *(const u32x4*)(ks_hi + (t * 32 + j) * KCS + col);
          const u32x4 al = *(const u32x4*)(ks_lo + (t * 32 + j) * KCS + col);
          const bf16x8 arh = as_bf(neg_im(ah)), aih = as_bf(swap_ri(ah));
          const bf16x8 arl = as_bf(neg_im(al)), ail = as_bf(swap_ri(al));
          accr[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, b_h, accr[t], 0, 0, 0);
          accr[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arh, b_l, accr[t], 0, 0, 0);
          accr[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(arl, b_h, accr[t], 0, 0, 0);
          acci[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, b_h, acci[t], 0, 0, 0);
          acci[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aih, b_l, acci[t], 0, 0, 0);
          acci[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ail, b_h, acci[t], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  if (krow) nyq[tid] = (ix & 1) ? -nacc : nacc;  // kx phase exp(i pi p_x) of the Nyquist column
  // kx phase of the fold
  if (bvalid) {
    const float2 ph = twf[(kxrow * ix) % N];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float yr = accr[t][v], yi = acci[t][v];
        accr[t][v] = yr * ph.x - yi * ph.y;
        acci[t][v] = yr * ph.y + yi * ph.x;
      }
  }
  unsigned short* ymh = (unsigned short*)raw;
  unsigned short* yml = ymh + 32 * YST;
  const int ntb = 2 * (Mp / 16);
  unsigned long long best = 0;
  const int l16 = lane & 15, q4 = lane >> 4;
  const unsigned short* WbL = WbT + (size_t)Mp * KB;
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    if (t >= mt_here) break;
    __syncthreads();
    for (int i = tid; i < 32 * (KB - N); i += NTH) {
      const int r = i / (KB - N), c = N + i % (KB - N);
      ymh[r * YST + c] = 0;
      yml[r * YST + c] = 0;
    }
    if (tid < 32) {
      const float v = nyq[t * 32 + tid];
      const unsigned a = bf16_bits(v);
      ymh[tid * YST + NC] = (unsigned short)a;
      yml[tid * YST + NC] = (unsigned short)bf16_bits(v - bf16_float(a));
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = (v >> 2) * 8 + h * 4 + (v & 3);
      if (bvalid) {
        const unsigned a = bf16_bits(accr[t][v]);
        ymh[i * YST + kxrow] = (unsigned short)a;
        yml[i * YST + kxrow] = (unsigned short)bf16_bits(accr[t][v] - bf16_float(a));
        if (kxrow >= 1) {
          const unsigned b = bf16_bits(acci[t][v]);
          ymh[i * YST + NC + kxrow] = (unsigned short)b;
          yml[i * YST + NC + kxrow] = (unsigned short)bf16_bits(acci[t][v] - bf16_float(b));
        }
      }
    }
    __syncthreads();
    const int mrow0 = m0 + t * 32;
    for (int T = wave; T < ntb; T += NW) {
      const int mt = T & 1, nt = T >> 1;
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      const unsigned short* ah_p = ymh + (mt * 16 + l16) * YST + 8 * q4;
      const unsigned short* al_p = yml + (mt * 16 + l16) * YST + 8 * q4;
      const unsigned short* bh_p = WbT + (size_t)(nt * 16 + l16) * KB + 8 * q4;
      const unsigned short* bl_p = WbL + (size_t)(nt * 16 + l16) * KB + 8 * q4;
#pragma unroll 4
      for (int k = 0; k < KB; k += 32) {
        const bf16x8 a_h = as_bf(*(const u32x4*)(ah_p + k));
        const bf16x8 a_l = as_bf(*(const u32x4*)(al_p + k));
        const bf16x8 w_h = as_bf(*(const u32x4*)(bh_p + k));
        const bf16x8 w_l = as_bf(*(const u32x4*)(bl_p + k));
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h, w_h, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h, w_l, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_l, w_h, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int my = mrow0 + mt * 16 + q4 * 4 + v;
        const int mx = nt * 16 + l16;
        if (my < g.M && mx < g.M) {
          const unsigned long long key = peak_key(acc[v], (unsigned)(my * g.M + mx));
          best = key > best ? key : best;
        }
      }
    }
  }
  best = wmax64(best);
  if (lane == 0) red[wave] = best;
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < NW; ++w) best = red[w] > best ? red[w] : best;
    atomicMax(&g.st[f].grid_key, best);
  }
}

template <int N>
static int updft_n(const GroupParams& g, const UpdftTables& t, hipStream_t s) {
  const int mtiles = t.Mp / 32;
  if (t.precision == CCPT_PREC_FP32) {
    hipLaunchKernelGGL((k_updft_f32<N>), dim3(mtiles, g.count), dim3(kUThreads), 0, s, g,
                       (const float2*)t.ky, (const float*)t.wb, t.Mp);
  } else if (t.precision == CCPT_PREC_BF16X2) {
    if (!g.Xb) return -1;
    if constexpr (N >= 256) {
      constexpr int MT = 5;
      constexpr int NW = (N / 2 + 31) / 32;
      hipLaunchKernelGGL((k_updft_bf16x2_wide<N, MT>), dim3((mtiles + MT - 1) / MT, g.count),
                         dim3(64 * NW), 0, s, g, (const float2*)t.ky, (const unsigned short*)t.wb,
                         t.Mp);
    } else {
      hipLaunchKernelGGL((k_updft_bf16x2<N>), dim3(mtiles, g.count), dim3(kUThreads), 0, s, g,
                         (const float2*)t.ky, (const unsigned short*)t.wb, t.Mp);
    }
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
