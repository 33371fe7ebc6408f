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
// For a rectangular frame of NY rows of NX pixels, ky runs over NY, kx over
// NX/2+1, 1/N^2 becomes 1/(NY NX), and the Stage B contraction length is NX.
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

// ky-chunk of the Stage A contraction held in LDS: the largest divisor of NY
// not above 32 (16 for the longest rows, to bound LDS)
constexpr int a_chunk(int NY, int NX) {
  const int cap = NX >= 384 ? 16 : 32;
  int best = 1;
  for (int d = 1; d <= cap; ++d)
    if (NY % d == 0) best = d;
  return best;
}

// Row stride (floats) of the FP32 path's Ymat in LDS: KB + 1, so the 16 rows
// and 4 lane groups (16 floats apart) of one Stage B MFMA read fall in
// distinct banks.
template <int NX>
constexpr int ym_stride() {
  return (NX + 31) / 32 * 32 + 1;
}

// Stage B of the FP32 path for one 32-row tile: U[32][Mp] = ym[32][KB] x
// W[KB][Mp] on 16x16x4 tiles, then the tile's grid maximum merged into the
// frame's key.  ym is in LDS (row stride ym_stride); W comes transposed
// ([Mp][KB]).  Within each 64-wide block of K, lane group q4 takes the 16
// consecutive k = 16 q4 + i over the block's 16 MFMA steps (the same k for
// A and B), so a lane loads its W values as four 16-byte runs per block.
// Every thread of the block calls this.
// Whole 64-wide K blocks of Stage B whose W values a lane loads at once: the
// largest divisor of the block count not above 4.
constexpr int stage_b_batch(int nb) {
  int b = 1;
  for (int d = 1; d <= 4 && d <= nb; ++d)
    if (nb % d == 0) b = d;
  return b;
}

template <int NY, int NX>
__device__ void stage_b_f32(const GroupParams& g, const float* ym, const float* __restrict__ WtT,
                            int Mp, int m0, int f, unsigned long long* red, int nt0, int nt1) {
  const bool tr = transposed<NY, NX>(g.trans);
  constexpr int KB = (NX + 31) / 32 * 32;
  constexpr int YR = ym_stride<NX>();
  constexpr int NB = KB / 64;            // whole 64-wide blocks of K
  constexpr bool TAIL = (KB % 64) != 0;  // then one of 32
  constexpr int BB = stage_b_batch(NB);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ntb = 2 * (nt1 - nt0);
  unsigned long long best = 0;
  const int l16 = lane & 15, q4 = lane >> 4;
  for (int T = wave; T < ntb; T += 4) {
    const int mt = T & 1, nt = nt0 + (T >> 1);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const float* arow = ym + (mt * 16 + l16) * YR + 16 * q4;
    const float* bcol = WtT + (size_t)(nt * 16 + l16) * KB + 16 * q4;
    // the W values of BB blocks are requested together (one memory round trip
    // per BB blocks, not per block), then the blocks' products in k order
    if constexpr (NB > 0) {
#pragma unroll
      for (int b0 = 0; b0 < NB; b0 += BB) {
        float4 w[BB][4];
#pragma unroll
        for (int b = 0; b < BB; ++b)
#pragma unroll
          for (int i = 0; i < 4; ++i) w[b][i] = *(const float4*)(bcol + (b0 + b) * 64 + 4 * i);
#pragma unroll
        for (int b = 0; b < BB; ++b) {
          const int k0 = (b0 + b) * 64;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(arow[k0 + 4 * i], w[b][i].x, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(arow[k0 + 4 * i + 1], w[b][i].y, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(arow[k0 + 4 * i + 2], w[b][i].z, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(arow[k0 + 4 * i + 3], w[b][i].w, acc, 0, 0, 0);
          }
        }
      }
    }
    if constexpr (TAIL) {
      // last 32 of K: lane group q4 takes k = k0 + 8 q4 + i
      constexpr int k0 = NB * 64;
      const float* ar = arow - 8 * q4;
      const float* bc = bcol - 8 * q4;
      float4 w[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) w[i] = *(const float4*)(bc + k0 + 4 * i);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[k0 + 4 * i], w[i].x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[k0 + 4 * i + 1], w[i].y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[k0 + 4 * i + 2], w[i].z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[k0 + 4 * i + 3], w[i].w, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int my = m0 + mt * 16 + q4 * 4 + v;
      const int mx = nt * 16 + l16;
      if (my < g.M && mx < g.M) {
        const unsigned long long key = peak_key(acc[v], grid_index(my, mx, g.M, tr));
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

// ---------------------------------------------------------------- FP32
// Frames of NY rows of NX (the spectrum is NY x (NX/2+1)).
// K table: float2 [Mp][NY]  (K[m][ky] = phi_ky((m - c)/u))
// W table: float  [Mp][Kb] (transposed), Kb = NX rounded up to 32 (zero columns past NX)
// SPLIT (few frames, latency): blockIdx.z is one of `nsl` ky slices; the
// block stores its partial Ymat to `ypart` and k_updft_f32_sum finishes.
template <int NY, int NX, bool SPLIT>
__global__ void __launch_bounds__(kUThreads) k_updft_f32(GroupParams g, const float2* __restrict__ Ktab,
                                                         const float* __restrict__ Wtab, int Mp,
                                                         float* __restrict__ ypart, int nsl) {
  constexpr int H = NX / 2 + 1;
  constexpr int NC = NX / 2;                // columns on matrix cores
  constexpr int NT = (NC + 31) / 32;        // 32-wide column tiles
  constexpr int TPW = (NT + 3) / 4;         // tiles per wave
  constexpr int KC = a_chunk(NY, NX);
  constexpr int KCS = KC + 1;               // K chunk row stride (float2): lanes on distinct banks
  constexpr int XS = KC * H;                // folded X' chunk (float2)
  constexpr int KS = 32 * KCS;              // K chunk (float2)
  constexpr int KB = (NX + 31) / 32 * 32;   // Stage B contraction, zero padded
  constexpr int YR = ym_stride<NX>();       // Ymat row stride (floats)
  constexpr int YS = 32 * YR / 2;           // Ymat as float2 count
  constexpr int RAW = (XS + KS) > YS ? (XS + KS) : YS;
  constexpr int RX = NY / NX;               // kx phase index step in the NY table
  __shared__ float2 raw[RAW];
  __shared__ float2 twf[NY];                // exp(+2 pi i m / NY)
  __shared__ float nyq[8][32];
  __shared__ unsigned long long red[kUThreads / 64];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = blockIdx.y;
  const int m0 = blockIdx.x * 32;
  const FrameState st = g.st[f];
  if (frame_skipped(st)) return;
  int iy, ix;
  peak_yx<NY, NX>(key_index(st.peak_key), g.trans, iy, ix);
  for (int i = tid; i < NY; i += kUThreads) twf[i] = cconj(g.tw[i]);

  float2* xs = raw;
  float2* ks = raw + XS;
  const float2* Xf = g.X + (size_t)f * NY * H;

  f32x16 accr[TPW], acci[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) accr[t][v] = acci[t][v] = 0.f;
  float nacc = 0.f;
  const int half = lane >> 5, l32 = lane & 31;
  __syncthreads();

  constexpr int NCH = NY / KC;
  const int ch0 = SPLIT ? (int)blockIdx.z * NCH / nsl : 0;
  const int ch1 = SPLIT ? ((int)blockIdx.z + 1) * NCH / nsl : NCH;
  // A chunk's X and K values are held in registers between their loads and
  // the LDS stores, so the next chunk's loads are in flight during this
  // chunk's matrix instructions (indices clamped: every load in bounds)
  constexpr int XQ = (XS + kUThreads - 1) / kUThreads;
  constexpr int KQ = (32 * KC + kUThreads - 1) / kUThreads;
  float2 xr[XQ], kr[KQ];
  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int q = 0; q < XQ; ++q) {
      const int i = min(tid + q * kUThreads, XS - 1);
      const int kk = i / H, kx = i - kk * H;
      xr[q] = Xf[(size_t)(k0 + kk) * H + kx];
    }
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      const int i = min(tid + q * kUThreads, 32 * KC - 1);
      const int m = i / KC, kk = i - m * KC;
      kr[q] = Ktab[(size_t)(m0 + m) * NY + k0 + kk];
    }
  };
  auto store_chunk = [&](int k0) {
#pragma unroll
    for (int q = 0; q < XQ; ++q) {
      const int i = tid + q * kUThreads;
      if (XS % kUThreads == 0 || i < XS) {
        const int kk = i / H, kx = i - kk * H;
        const int ky = k0 + kk;
        float2 v = cmul(xr[q], twf[(ky * iy + kx * ix * RX) % NY]);
        if (ky == 0 && kx == 0) v = make_float2(0.f, 0.f);  // DC only shifts U by a constant
        xs[i] = v;
      }
    }
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      const int i = tid + q * kUThreads;
      if ((32 * KC) % kUThreads == 0 || i < 32 * KC) {
        const int m = i / KC, kk = i - m * KC;
        ks[m * KCS + kk] = kr[q];
      }
    }
  };
  load_chunk(ch0 * KC);
  for (int k0 = ch0 * KC; k0 < ch1 * KC; k0 += KC) {
    store_chunk(k0);
    __syncthreads();
    load_chunk(min(k0 + KC, (ch1 - 1) * KC));  // (the last chunk reloads itself)
#pragma unroll 4
    for (int kk = 0; kk < KC; ++kk) {
      const float2 kv = ks[l32 * KCS + kk];
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
    // Nyquist column kx = NX/2: Yr only
    {
      const int m = tid & 31, grp = tid >> 5;
      for (int kk = grp; kk < KC; kk += 8) {
        const float2 kv = ks[m * KCS + kk];
        const float2 xv = xs[kk * H + NC];
        nacc += kv.x * xv.x - kv.y * xv.y;
      }
    }
    __syncthreads();
  }
  nyq[tid >> 5][tid & 31] = nacc;
  // Ymat[32][KB] (floats) aliases the chunk buffers
  float* ym = (float*)raw;
  for (int i = tid; i < 32 * (KB - NX); i += kUThreads) {
    const int r = i / (KB - NX), j = NX + i % (KB - NX);
    ym[r * YR + j] = 0.f;
  }
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int kx = (wave + 4 * t) * 32 + l32;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = (v >> 2) * 8 + half * 4 + (v & 3);
      if (kx < NC) ym[i * YR + kx] = accr[t][v];
      if (kx >= 1 && kx < NC) ym[i * YR + NC + kx] = acci[t][v];
    }
  }
  __syncthreads();
  if (tid < 32) {
    float s = 0.f;
    for (int q = 0; q < 8; ++q) s += nyq[q][tid];
    ym[tid * YR + NC] = s;
  }
  __syncthreads();
  if constexpr (SPLIT) {
    const int mtiles = Mp / 32;
    float* dst = ypart + (((size_t)f * mtiles + blockIdx.x) * nsl + blockIdx.z) * 32 * KB;
    for (int i = tid; i < 32 * KB; i += kUThreads) dst[i] = ym[(i / KB) * YR + i % KB];
  } else {
    stage_b_f32<NY, NX>(g, ym, Wtab, Mp, m0, f, red, 0, Mp / 16);
  }
}

// Sums the ky-slice partials of one 32-row tile in a fixed order, then Stage B
// over kSumColTiles 16-column tiles of the grid (blockIdx.z picks them: a
// single frame's Stage B is spread over (Mp/32) x (Mp/16/kSumColTiles) blocks,
// each summing the partials of its rows).
constexpr int kSumColTiles = 2;
template <int NY, int NX>
__global__ void __launch_bounds__(kUThreads) k_updft_f32_sum(GroupParams g, const float* __restrict__ Wtab,
                                                             int Mp, const float* __restrict__ ypart,
                                                             int nsl) {
  constexpr int KB = (NX + 31) / 32 * 32;
  constexpr int YR = ym_stride<NX>();
  __shared__ float ym[32 * YR];
  __shared__ unsigned long long red[kUThreads / 64];
  const int f = blockIdx.y;
  const FrameState st = g.st[f];
  if (frame_skipped(st)) return;
  const int mtiles = Mp / 32;
  const float* src = ypart + ((size_t)f * mtiles + blockIdx.x) * nsl * 32 * KB;
  // every element a thread owns is loaded at once per slice (the partials
  // come from other XCDs: one round trip per slice, not per element); each
  // element is summed over the slices in order
  constexpr int PER = 32 * KB / kUThreads;  // KB is a multiple of 32
  // SG slices are requested together (a clamped slice index keeps every load
  // in bounds; slices past nsl are not added)
  constexpr int SG = PER >= 128 ? 1 : (128 / PER < kSplitSlices ? 128 / PER : kSplitSlices);
  float v[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) v[e] = 0.f;
  for (int q0 = 0; q0 < nsl; q0 += SG) {
    float p[SG][PER];
#pragma unroll
    for (int j = 0; j < SG; ++j) {
      const int q = min(q0 + j, nsl - 1);
#pragma unroll
      for (int e = 0; e < PER; ++e) p[j][e] = src[(size_t)q * 32 * KB + threadIdx.x + e * kUThreads];
    }
#pragma unroll
    for (int j = 0; j < SG; ++j)
      if (q0 + j < nsl) {
#pragma unroll
        for (int e = 0; e < PER; ++e) v[e] += p[j][e];
      }
  }
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    const int i = threadIdx.x + e * kUThreads;
    ym[(i / KB) * YR + i % KB] = v[e];
  }
  __syncthreads();
  const int nt0 = (int)blockIdx.z * kSumColTiles;
  stage_b_f32<NY, NX>(g, ym, Wtab, Mp, blockIdx.x * 32, f, red, nt0, min(nt0 + kSumColTiles, Mp / 16));
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
template <int NY, int NX>
__global__ void __launch_bounds__(kUThreads) k_updft_bf16x2(GroupParams g, const float2* __restrict__ Ktab,
                                                            const unsigned short* __restrict__ WbT, int Mp) {
  constexpr int H = NX / 2 + 1;
  constexpr int NC = NX / 2;
  constexpr int NT = (NC + 31) / 32;
  constexpr int TPW = (NT + 3) / 4;
  constexpr int P = xb_pitch(NY);
  constexpr int KC = NX >= 384 ? 16 : 32;  // ky per LDS chunk (multiple of 8)
  constexpr int KCS = KC + 4;              // LDS row stride, words
  constexpr int XROWS = NT * 32;
  constexpr int KB = (NX + 31) / 32 * 32;
  constexpr int RX = NY / NX;              // kx phase index step in the NY table
  constexpr int YST = KB + 8;              // Ymat row stride, bf16 elements
  constexpr int XW = 2 * XROWS * KCS;
  constexpr int KW = 2 * 32 * KCS;
  constexpr int YW = 32 * YST;             // two bf16 planes of 32 x YST
  constexpr int RAWW = (XW + KW) > YW ? (XW + KW) : YW;
  __shared__ __attribute__((aligned(16))) unsigned raw[RAWW];
  __shared__ float2 kf[32][KC + 1];
  __shared__ float2 twf[NY];
  __shared__ float nyq[8][32];
  __shared__ unsigned long long red[kUThreads / 64];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = blockIdx.y;
  const int m0 = blockIdx.x * 32;
  const FrameState st = g.st[f];
  if (frame_skipped(st)) return;
  int iy, ix;
  peak_yx<NY, NX>(key_index(st.peak_key), g.trans, iy, ix);
  const bool tr = transposed<NY, NX>(g.trans);
  for (int i = tid; i < NY; i += kUThreads) twf[i] = cconj(g.tw[i]);

  unsigned* xs_hi = raw;
  unsigned* xs_lo = raw + XROWS * KCS;
  unsigned* ks_hi = raw + XW;
  unsigned* ks_lo = ks_hi + 32 * KCS;
  const unsigned* Xbh = g.Xb + (size_t)f * 2 * NC * P;
  const unsigned* Xbl = Xbh + (size_t)NC * P;
  const float2* Xf = g.X + (size_t)f * NY * H;

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
      if (ky < NY) kv = cmul(Ktab[(size_t)(m0 + m) * NY + ky], twf[(ky * iy) % NY]);
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
    {  // Nyquist column kx = NX/2 in FP32 on the VALU
      const int m = tid & 31, grp = tid >> 5;
      for (int kk = grp; kk < KC; kk += 8) {
        const int ky = k0 + kk;
        if (ky < NY) {
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
      const float2 ph = twf[(kx * ix * RX) % NY];
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
  for (int i = tid; i < 32 * (KB - NX); i += kUThreads) {
    const int r = i / (KB - NX), c = NX + i % (KB - NX);
    ymh[r * YST + c] = 0;
    yml[r * YST + c] = 0;
  }
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int kx = (wave + 4 * t) * 32 + j;
#pragma unroll
    for (int v = 0; v < 16; v += 2) {
      const int i = (v >> 2) * 8 + h * 4 + (v & 3);  // rows i and i + 1
      if (kx < NC) {
        unsigned a, al;
        split2(accr[t][v], accr[t][v + 1], a, al);
        ymh[i * YST + kx] = (unsigned short)a;
        ymh[(i + 1) * YST + kx] = (unsigned short)(a >> 16);
        yml[i * YST + kx] = (unsigned short)al;
        yml[(i + 1) * YST + kx] = (unsigned short)(al >> 16);
      }
      if (kx >= 1 && kx < NC) {
        unsigned b, bl;
        split2(acci[t][v], acci[t][v + 1], b, bl);
        ymh[i * YST + NC + kx] = (unsigned short)b;
        ymh[(i + 1) * YST + NC + kx] = (unsigned short)(b >> 16);
        yml[i * YST + NC + kx] = (unsigned short)bl;
        yml[(i + 1) * YST + NC + kx] = (unsigned short)(bl >> 16);
      }
    }
  }
  __syncthreads();
  if (tid < 32) {
    float sacc = 0.f;
    for (int q = 0; q < 8; ++q) sacc += nyq[q][tid];
    if (ix & 1) sacc = -sacc;  // exp(i pi p_x)
    unsigned a, al;
    split2(sacc, 0.f, a, al);
    ymh[tid * YST + NC] = (unsigned short)a;
    yml[tid * YST + NC] = (unsigned short)al;
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
        const unsigned long long key = peak_key(acc[v], grid_index(my, mx, g.M, tr));
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


// Wide variant for rows of NX > 256: one block per frame and group of up to MT
// 32-row m-tiles, one wave per 32-column kx tile.  Each frame's split
// spectrum is streamed once from memory straight into the B operands (each
// fragment feeds 6 MT matrix instructions).  The A operands come from the
// precomputed folded table K'_p[m, ky] = phi_ky(p + (m - c)/u) for the
// frame's integer peak row p (bf16 hi/lo words), copied per 32-ky chunk into
// LDS and shared by all waves.  Row 0 of the split spectrum carries the
// Nyquist column in its imaginary part, so Yi(., 0) is the Nyquist output.
// The three products of each K step are issued pass by pass over all tiles
// so consecutive matrix instructions never depend on each other.  Where a
// block's waves fit one per SIMD (NX <= 256) Stage A is software pipelined:
// the next chunk's B fragments and K' rows are loaded while the current
// chunk's MFMAs run, and K' chunks alternate between two LDS buffers.
// Stage B converts Y to bf16 hi/lo for up to GB row tiles at a time into
// LDS, so every W fragment a wave loads from L2 serves 2*GB row halves (W
// is read 2 times per frame instead of 2*MT); its three products accumulate
// into one register tile per row half (separate ones per product left the
// compiler shuffling accumulators beside the pending Stage A tiles).
template <int NY, int NX, int MT>
__global__ void __launch_bounds__(64 * ((NX / 2 + 31) / 32))
    k_updft_bf16x2_wide(GroupParams g, const unsigned* __restrict__ kfold,
                        const unsigned short* __restrict__ WbT, int Mp) {
  constexpr int NC = NX / 2;
  constexpr int NW = (NC + 31) / 32;  // waves = kx tiles
  constexpr int NTH = 64 * NW;
  constexpr int P = xb_pitch(NY);
  constexpr int KC = 32;
  constexpr int KCS = KC + 4;
  constexpr int ROWS = MT * 32;
  constexpr int KB = (NX + 31) / 32 * 32;
  constexpr int RX = NY / NX;  // kx phase index step in the NY table
  constexpr int YST = KB + 8;
  constexpr int KW = 2 * ROWS * KCS;
  constexpr int YW = 32 * YST;
  // the pipelined Stage A needs registers for a second chunk of operands:
  // used where a block's waves fit one per SIMD (NX <= 256)
  constexpr bool PIPE = NW <= 4;
  constexpr int GB = 3 * YW * 4 <= 120000 ? 3 : 2;  // row tiles per Stage B group
  constexpr int KWT = PIPE ? 2 * KW : KW;
  constexpr int RAWW = KWT > GB * YW ? KWT : GB * YW;
  __shared__ __attribute__((aligned(16))) unsigned raw[RAWW];
  __shared__ float2 twf[NY];
  __shared__ unsigned long long red[NW];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = blockIdx.y;
  const int m0 = blockIdx.x * ROWS;  // the folded table has rows up to a whole block
  const FrameState st = g.st[f];
  if (frame_skipped(st)) return;
  int iy, ix;
  peak_yx<NY, NX>(key_index(st.peak_key), g.trans, iy, ix);
  const bool tr = transposed<NY, NX>(g.trans);
  for (int i = tid; i < NY; i += NTH) twf[i] = cconj(g.tw[i]);

  const size_t kplane = (size_t)kfold_rows(Mp) * P;
  const unsigned* Kh = kfold + (size_t)iy * 2 * kplane;
  const unsigned* Kl = Kh + kplane;
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
  constexpr int NCH = P / KC;
  constexpr int KCOPY = ROWS * (KC / 4);                 // 16-byte K' copies per chunk
  constexpr int KQ = (KCOPY + NTH - 1) / NTH;            // per thread
  constexpr bool BFULL = NC % 32 == 0;                   // every wave's kx tile is full

  // B fragments of this wave's kx tile for the ky chunk at k0 (global -> registers)
  auto load_b = [&](int k0, u32x4* dh, u32x4* dl) {
#pragma unroll
    for (int s8 = 0; s8 < KC / 8; ++s8) {
      const int col = k0 + s8 * 8 + 4 * h;
      if (BFULL || bvalid) {
        dh[s8] = *(const u32x4*)(Xbh + (size_t)kxrow * P + col);
        dl[s8] = *(const u32x4*)(Xbl + (size_t)kxrow * P + col);
      } else {
        dh[s8] = u32x4{0u, 0u, 0u, 0u};
        dl[s8] = u32x4{0u, 0u, 0u, 0u};
      }
    }
  };
  // the block's K' rows for the ky chunk at k0: global -> registers -> LDS
  u32x4 kh[KQ], kl[KQ];
  auto load_k = [&](int k0) {
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      const int i = tid + q * NTH;
      if (KCOPY % NTH == 0 || i < KCOPY) {
        const int r = i / (KC / 4), c4 = i - r * (KC / 4);
        const size_t src = (size_t)(m0 + r) * P + k0 + 4 * c4;
        kh[q] = *(const u32x4*)(Kh + src);
        kl[q] = *(const u32x4*)(Kl + src);
      }
    }
  };
  auto store_k = [&](unsigned* dh) {
    unsigned* dl = dh + ROWS * KCS;
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      const int i = tid + q * NTH;
      if (KCOPY % NTH == 0 || i < KCOPY) {
        const int r = i / (KC / 4), c4 = i - r * (KC / 4);
        *(u32x4*)(dh + r * KCS + 4 * c4) = kh[q];
        *(u32x4*)(dl + r * KCS + 4 * c4) = kl[q];
      }
    }
  };
  // Stage A products of one ky chunk: three passes (hi*hi, hi*lo, lo*hi) per tile
  auto mma_chunk = [&](const unsigned* ks_hi, const u32x4* bh, const u32x4* bl) {
    const unsigned* ks_lo = ks_hi + ROWS * KCS;
#pragma unroll
    for (int s8 = 0; s8 < KC / 8; ++s8) {
      const int col = s8 * 8 + 4 * h;
      // B as (re, -im) for Re(K X) and as (im, re) for Im(K X); A is used as stored
      const bf16x8 bh_r = as_bf(neg_im(bh[s8])), bh_i = as_bf(swap_ri(bh[s8]));
      const bf16x8 bl_r = as_bf(neg_im(bl[s8])), bl_i = as_bf(swap_ri(bl[s8]));
      bf16x8 ah[MT], al[MT];
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        ah[t] = as_bf(*(const u32x4*)(ks_hi + (t * 32 + j) * KCS + col));
        al[t] = as_bf(*(const u32x4*)(ks_lo + (t * 32 + j) * KCS + col));
      }
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        accr[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[t], bh_r, accr[t], 0, 0, 0);
        acci[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[t], bh_i, acci[t], 0, 0, 0);
      }
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        accr[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[t], bl_r, accr[t], 0, 0, 0);
        acci[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[t], bl_i, acci[t], 0, 0, 0);
      }
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        accr[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[t], bh_r, accr[t], 0, 0, 0);
        acci[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[t], bh_i, acci[t], 0, 0, 0);
      }
    }
  };

  u32x4 bh[KC / 8], bl[KC / 8];
  if constexpr (PIPE) {
    // software pipeline: chunk c + 1's operands are loaded while chunk c's
    // MFMAs run; K' chunks alternate between two LDS buffers
    u32x4 nh[KC / 8], nl[KC / 8];
    load_b(0, bh, bl);
    load_k(0);
    store_k(raw);
    __syncthreads();
    for (int c = 0; c < NCH; ++c) {
      const bool more = c + 1 < NCH;
      if (more) {
        load_b((c + 1) * KC, nh, nl);
        load_k((c + 1) * KC);
      }
      // keep the next chunk's loads ahead of this chunk's MFMAs and their LDS
      // stores (which wait for the loads) behind them
      __builtin_amdgcn_sched_barrier(0);
      mma_chunk(raw + (c & 1) * KW, bh, bl);
      __builtin_amdgcn_sched_barrier(0);
      if (more) store_k(raw + ((c + 1) & 1) * KW);
      __syncthreads();
      if (more) {
#pragma unroll
        for (int s8 = 0; s8 < KC / 8; ++s8) {
          bh[s8] = nh[s8];
          bl[s8] = nl[s8];
        }
      }
    }
  } else {
    for (int c = 0; c < NCH; ++c) {
      load_b(c * KC, bh, bl);
      load_k(c * KC);
      store_k(raw);
      __syncthreads();
      mma_chunk(raw, bh, bl);
      __syncthreads();
    }
  }
  // kx phase of the fold; column 0 holds (Y[., 0], Y[., N/2]) and its phase is 1
  if ((BFULL || bvalid) && kxrow > 0) {
    const float2 ph = twf[(kxrow * ix * RX) % NY];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float yr = accr[t][v], yi = acci[t][v];
        accr[t][v] = yr * ph.x - yi * ph.y;
        acci[t][v] = yr * ph.y + yi * ph.x;
      }
  }
  const float nyq_sign = (ix & 1) ? -1.f : 1.f;  // exp(i pi p_x)
  // Stage B in groups of up to GB row tiles: their Y (bf16 hi/lo planes) sits in
  // LDS together, so each W fragment a wave loads serves 2 * GB row halves
  constexpr int SLOT = 2 * 32 * YST;  // u16 elements per row tile (hi, lo planes)
  unsigned short* ybase = (unsigned short*)raw;
  const int nnt = Mp / 16;
  unsigned long long best = 0;
  const int l16 = lane & 15, q4 = lane >> 4;
  const unsigned short* WbL = WbT + (size_t)Mp * KB;
#pragma unroll
  for (int t0 = 0; t0 < MT; t0 += GB) {
    const int gn = min(GB, MT - t0);  // a constant once the loop is unrolled
    __syncthreads();
#pragma unroll
    for (int t = t0; t < t0 + GB && t < MT; ++t) {
      unsigned short* ymh = ybase + (t - t0) * SLOT;
      unsigned short* yml = ymh + 32 * YST;
      for (int i = tid; i < 32 * (KB - NX); i += NTH) {
        const int r = i / (KB - NX), c = NX + i % (KB - NX);
        ymh[r * YST + c] = 0;
        yml[r * YST + c] = 0;
      }
#pragma unroll
      for (int v = 0; v < 16; v += 2) {
        const int i = (v >> 2) * 8 + h * 4 + (v & 3);  // rows i and i + 1
        if (BFULL || bvalid) {
          unsigned a, al;
          split2(accr[t][v], accr[t][v + 1], a, al);
          ymh[i * YST + kxrow] = (unsigned short)a;
          ymh[(i + 1) * YST + kxrow] = (unsigned short)(a >> 16);
          yml[i * YST + kxrow] = (unsigned short)al;
          yml[(i + 1) * YST + kxrow] = (unsigned short)(al >> 16);
          const float sg = kxrow == 0 ? nyq_sign : 1.f;
          const int col = NC + kxrow;  // Yi of kx, or the Nyquist output for kx = 0
          unsigned b, bl;
          split2(sg * acci[t][v], sg * acci[t][v + 1], b, bl);
          ymh[i * YST + col] = (unsigned short)b;
          ymh[(i + 1) * YST + col] = (unsigned short)(b >> 16);
          yml[i * YST + col] = (unsigned short)bl;
          yml[(i + 1) * YST + col] = (unsigned short)(bl >> 16);
        }
      }
    }
    __syncthreads();
    // this wave's 16-column W tiles nt = wave, wave + NW, ...; every row half of the group
    for (int nt = wave; nt < nnt; nt += NW) {
      f32x4 acc[2 * GB];
#pragma unroll
      for (int r = 0; r < 2 * GB; ++r) acc[r] = f32x4{0.f, 0.f, 0.f, 0.f};
      const unsigned short* bh_p = WbT + (size_t)(nt * 16 + l16) * KB + 8 * q4;
      const unsigned short* bl_p = WbL + (size_t)(nt * 16 + l16) * KB + 8 * q4;
      // Y fragments of the group's row halves for a k step (LDS).  Where waves
      // share SIMDs (NW > 4) the next step's load during this step's MFMAs,
      // which also keeps those sizes from spilling registers.
      constexpr bool YPRE = NW > 4;
      bf16x8 a_h[2 * GB], a_l[2 * GB], n_h[2 * GB], n_l[2 * GB];
      auto load_a = [&](int k, bf16x8* dh, bf16x8* dl) {
#pragma unroll
        for (int r = 0; r < 2 * GB; ++r) {
          if (r < 2 * gn) {
            const unsigned short* ah_p = ybase + (r >> 1) * SLOT + ((r & 1) * 16 + l16) * YST + 8 * q4;
            dh[r] = as_bf(*(const u32x4*)(ah_p + k));
            dl[r] = as_bf(*(const u32x4*)(ah_p + 32 * YST + k));
          }
        }
      };
      if constexpr (YPRE) load_a(0, a_h, a_l);
#pragma unroll 4
      for (int k = 0; k < KB; k += 32) {
        const bf16x8 w_h = as_bf(*(const u32x4*)(bh_p + k));
        const bf16x8 w_l = as_bf(*(const u32x4*)(bl_p + k));
        if constexpr (YPRE) {
          if (k + 32 < KB) load_a(k + 32, n_h, n_l);
          __builtin_amdgcn_sched_barrier(0);
        } else {
          load_a(k, a_h, a_l);
        }
        // the three products pass by pass over the row halves, into one
        // accumulator per half (consecutive MFMAs never depend on each other)
#pragma unroll
        for (int r = 0; r < 2 * GB; ++r)
          if (r < 2 * gn) acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h[r], w_h, acc[r], 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 2 * GB; ++r)
          if (r < 2 * gn) acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h[r], w_l, acc[r], 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 2 * GB; ++r)
          if (r < 2 * gn) acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_l[r], w_h, acc[r], 0, 0, 0);
        if constexpr (YPRE) {
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int r = 0; r < 2 * GB; ++r) {
            a_h[r] = n_h[r];
            a_l[r] = n_l[r];
          }
        }
      }
#pragma unroll
      for (int r = 0; r < 2 * GB; ++r) {
        if (r < 2 * gn) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float uval = acc[r][v];
            const int my = m0 + (t0 + (r >> 1)) * 32 + (r & 1) * 16 + q4 * 4 + v;
            const int mx = nt * 16 + l16;
            if (my < g.M && mx < g.M) {
              const unsigned long long key = peak_key(uval, grid_index(my, mx, g.M, tr));
              best = key > best ? key : best;
            }
          }
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

// Variant for rows of NX = 256 (four 32-column kx tiles): the same Stage A as
// k_updft_bf16x2_wide with the operands of every matrix instruction swapped,
// so each wave holds Y^T of its kx tile: lane l has grid row m = l mod 32 of
// each row tile and, across its registers, the kx values
// (v / 4) 8 + 4 (l / 32) + v mod 4 of the tile.  That is the layout of a
// Stage B A operand whose k index runs over the kx of the tile, so Stage B
// takes Y from registers (split into bf16 hi/lo in place) against the W
// table stored in the matching order (tables.h, the 256-column layout), with
// no staging of Y in LDS.  Each wave contracts its own kx slice (its 32
// columns of Yr and of Yi, four k steps) for every grid point, so the four
// waves do equal work; per 32-column tile of the grid the four partial
// grids meet in LDS and are added in wave order (a fixed order), and the
// grid maximum is taken from the sums.
//
// FROMX: the frame's spectrum comes as FP32 X (row-major) plus the packed
// column Zc instead of the split copy Xb, and each chunk's A fragments are
// split into bf16 hi/lo here, after the matrix instructions of the chunk
// before (the same words the split copy would hold).
//
// F16 (with FROMX): the fp16 hi + lo split instead (about 22 significant
// bits): X scaled by a power of two from the frame's largest component (the
// correlation kernel records it), Y by 2^-8 before Stage B, and the K' and W
// tables stored as fp16 hi/lo (W scaled by 2^16 on the host); every scale is a
// positive power of two, so the grid and its maximum are those of the
// unscaled products up to rounding.
// One 32x32x16 matrix instruction on packed bf16 (F16 = false) or fp16
// operands, FP32 accumulation.
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
template <bool F16>
__device__ __forceinline__ f32x16 mfma32(u32x4 a, u32x4 b, f32x16 c) {
  if constexpr (F16)
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

template <int NY, int MT, bool FROMX, bool F16>
__global__ void __launch_bounds__(256)
    k_updft_bf16x2_t256(GroupParams g, const unsigned* __restrict__ kfold,
                        const unsigned short* __restrict__ WP, int Mp) {
  constexpr int NX = 256, NC = 128, NKT = 4, NTH = 256;
  constexpr int P = xb_pitch(NY);
  constexpr int KC = 32;
  constexpr int KCS = KC + 4;
  constexpr int ROWS = MT * 32;
  constexpr int RX = NY / NX;  // kx phase index step in the NY table
  constexpr int KW = 2 * ROWS * KCS;
  constexpr int UST = ROWS + 4;  // floats per grid column of a kx slice's partial grid
  constexpr int UW = 32 * UST;   // floats per kx slice's partial grid (one 32-column tile)
  constexpr int RAWW = 2 * KW > NKT * UW ? 2 * KW : NKT * UW;
  __shared__ __attribute__((aligned(16))) unsigned raw[RAWW];
  __shared__ float2 twf[NY];
  __shared__ unsigned long long red[NTH / 64];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kt = wave;  // kx tile
  const int f = blockIdx.y;
  const int m0 = blockIdx.x * ROWS;  // the folded table has rows up to a whole block
  const FrameState st = g.st[f];
  if (frame_skipped(st)) return;
  int iy, ix;
  peak_yx<NY, NX>(key_index(st.peak_key), g.trans, iy, ix);
  const bool tr = transposed<NY, NX>(g.trans);
  for (int i = tid; i < NY; i += NTH) twf[i] = cconj(g.tw[i]);

  const size_t kplane = (size_t)kfold_rows(Mp) * P;
  const unsigned* Kh = kfold + (size_t)iy * 2 * kplane;
  const unsigned* Kl = Kh + kplane;
  const unsigned* Xbh = g.Xb + (size_t)f * 2 * NC * P;
  const unsigned* Xbl = Xbh + (size_t)NC * P;
  const int h = lane >> 5, j = lane & 31;
  const int kxrow = kt * 32 + j;

  f32x16 accr[MT], acci[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int v = 0; v < 16; ++v) accr[t][v] = acci[t][v] = 0.f;
  constexpr int NCH = P / KC;
  constexpr int KCOPY = ROWS * (KC / 4);
  constexpr int KQ = (KCOPY + NTH - 1) / NTH;

  auto load_b = [&](int k0, u32x4* dh, u32x4* dl) {
#pragma unroll
    for (int s8 = 0; s8 < KC / 8; ++s8) {
      const int col = k0 + s8 * 8 + 4 * h;
      dh[s8] = *(const u32x4*)(Xbh + (size_t)kxrow * P + col);
      dl[s8] = *(const u32x4*)(Xbl + (size_t)kxrow * P + col);
    }
  };
  u32x4 kh[KQ], kl[KQ];
  auto load_k = [&](int k0) {
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      const int i = tid + q * NTH;
      if (KCOPY % NTH == 0 || i < KCOPY) {
        const int r = i / (KC / 4), c4 = i - r * (KC / 4);
        const size_t src = (size_t)(m0 + r) * P + k0 + 4 * c4;
        kh[q] = *(const u32x4*)(Kh + src);
        kl[q] = *(const u32x4*)(Kl + src);
      }
    }
  };
  auto store_k = [&](unsigned* dh) {
    unsigned* dl = dh + ROWS * KCS;
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      const int i = tid + q * NTH;
      if (KCOPY % NTH == 0 || i < KCOPY) {
        const int r = i / (KC / 4), c4 = i - r * (KC / 4);
        *(u32x4*)(dh + r * KCS + 4 * c4) = kh[q];
        *(u32x4*)(dl + r * KCS + 4 * c4) = kl[q];
      }
    }
  };
  // Stage A products of one ky chunk, transposed: the spectrum fragment is the
  // A operand (rows kx), the K' fragment the B operand (columns m)
  // hook(slot) after each pair of matrix instructions (slot 15 s8 + j for
  // MT = 5): work the caller places in the shadow of the instructions
  auto mma_chunk = [&](const unsigned* ks_hi, const u32x4* bh, const u32x4* bl, auto&& hook) {
    const unsigned* ks_lo = ks_hi + ROWS * KCS;
    int slot = 0;
#pragma unroll
    for (int s8 = 0; s8 < KC / 8; ++s8) {
      const int col = s8 * 8 + 4 * h;
      // (the sign flip and the half swap act alike on packed bf16 and fp16)
      const u32x4 bh_r = neg_im(bh[s8]), bh_i = swap_ri(bh[s8]);
      const u32x4 bl_r = neg_im(bl[s8]), bl_i = swap_ri(bl[s8]);
      u32x4 ah[MT], al[MT];
#pragma unroll
      for (int t = 0; t < MT; ++t)
        {
          ah[t] = *(const u32x4*)(ks_hi + (t * 32 + j) * KCS + col);
          al[t] = *(const u32x4*)(ks_lo + (t * 32 + j) * KCS + col);
        }
#pragma unroll
      for (int t = 0; t < MT; ++t)
        {
          accr[t] = mfma32<F16>(bh_r, ah[t], accr[t]);
          acci[t] = mfma32<F16>(bh_i, ah[t], acci[t]);
          hook(slot++);
        }
#pragma unroll
      for (int t = 0; t < MT; ++t)
        {
          accr[t] = mfma32<F16>(bl_r, ah[t], accr[t]);
          acci[t] = mfma32<F16>(bl_i, ah[t], acci[t]);
          hook(slot++);
        }
#pragma unroll
      for (int t = 0; t < MT; ++t)
        {
          accr[t] = mfma32<F16>(bh_r, al[t], accr[t]);
          acci[t] = mfma32<F16>(bh_i, al[t], acci[t]);
          hook(slot++);
        }
    }
  };

  u32x4 bh[KC / 8], bl[KC / 8];
  if constexpr (FROMX) {
    static_assert(xb_pitch(NY) == NY, "FP32 operands: rows of whole chunks");
    constexpr int H = NX / 2 + 1;
    const float2* Xc = kxrow == 0 ? g.Zc + (size_t)f * NY : g.X + (size_t)f * NY * H + kxrow;
    const int xs = kxrow == 0 ? 1 : H;
    float2 xr[KC / 8][4];
    auto load_x = [&](int k0) {
#pragma unroll
      for (int s8 = 0; s8 < KC / 8; ++s8)
#pragma unroll
        for (int e = 0; e < 4; ++e) xr[s8][e] = Xc[(size_t)(k0 + s8 * 8 + 4 * h + e) * xs];
    };
    // fp16: the frame's spectrum scaled by a power of two that brings its
    // largest component (without DC) below 2^13 (exact; the grid maximum does
    // not depend on a positive scale, and Newton reads the unscaled X)
    float xsc = 1.f;
    if constexpr (F16) {
      const float xm = __uint_as_float(st.xmax);
      int ex = 0;
      (void)frexpf(xm, &ex);
      if (xm > 0.f && xm <= 3.4e38f) xsc = ldexpf(1.f, min(13 - ex, 120));  // (finite X only)
    }
    // Stage A pipelined by k step: at the top of chunk c, bh/bl[0] hold the
    // split of X(c)'s k step 0, xr[1..3] its raw k steps 1..3 and xr[0] the
    // raw k step 0 of chunk c + 1.  Between the matrix instructions of k step
    // s < 3 the split of k step s + 1 is made and its register group reloaded
    // with the next chunk's values; between those of the last k step the next
    // chunk's K' fragments go to the other LDS buffer, its k step 0 is split
    // (bh/bl[0] are free once k step 0 is done) and xr[0] reloaded with the
    // chunk after it.  So every X load has a whole chunk to arrive and nothing
    // but the barrier separates two chunks' matrix instructions.  The last
    // chunks request themselves again (no branch in the loop body).
    auto load_x8 = [&](int k0, int s8) {
#pragma unroll
      for (int e = 0; e < 4; ++e) xr[s8][e] = Xc[(size_t)(k0 + s8 * 8 + 4 * h + e) * xs];
    };
    auto split_x8 = [&](int s8, int e) {
      unsigned wh, wl;
      if constexpr (F16)
        split2_f16(xr[s8][e].x * xsc, xr[s8][e].y * xsc, wh, wl);
      else
        split_pair(xr[s8][e], wh, wl);
      bh[s8][e] = wh;
      bl[s8][e] = wl;
    };
    static_assert(KC / 8 == 4 && MT == 5 && KQ <= 6, "hook slots laid out for 4 k steps of 15 pairs");
    load_x(0);
    load_k(0);
#pragma unroll
    for (int e = 0; e < 4; ++e) split_x8(0, e);
    load_x8((NCH > 1 ? 1 : 0) * KC, 0);
    store_k(raw);
    __syncthreads();
    for (int c = 0; c < NCH; ++c) {
      const int cn = (c + 1 < NCH ? c + 1 : c) * KC;
      const int cnn = (c + 2 < NCH ? c + 2 : NCH - 1) * KC;
      unsigned* knext = raw + ((c + 1) & 1) * KW;
      load_k(cn);
      __builtin_amdgcn_sched_barrier(0);
      mma_chunk(raw + (c & 1) * KW, bh, bl, [&](int slot) {
        const int s8 = slot / 15, j = slot - 15 * s8;
        if (s8 < 3) {
          if (j == 2 || j == 4 || j == 6 || j == 8) {
            __builtin_amdgcn_sched_barrier(0);
            split_x8(s8 + 1, (j - 2) / 2);
            __builtin_amdgcn_sched_barrier(0);
          } else if (j == 10) {
            __builtin_amdgcn_sched_barrier(0);
            load_x8(cn, s8 + 1);
            __builtin_amdgcn_sched_barrier(0);
          }
        } else if (j >= 2 && (j & 1) == 0 && (j - 2) / 2 < KQ) {
          const int q = (j - 2) / 2;
          const int i = tid + q * NTH;
          if (KCOPY % NTH == 0 || i < KCOPY) {
            __builtin_amdgcn_sched_barrier(0);
            const int r = i / (KC / 4), c4 = i - r * (KC / 4);
            *(u32x4*)(knext + r * KCS + 4 * c4) = kh[q];
            *(u32x4*)(knext + ROWS * KCS + r * KCS + 4 * c4) = kl[q];
            __builtin_amdgcn_sched_barrier(0);
          }
        } else if (j == 3 || j == 5 || j == 7 || j == 9) {
          __builtin_amdgcn_sched_barrier(0);
          split_x8(0, (j - 3) / 2);
          __builtin_amdgcn_sched_barrier(0);
        } else if (j == 11) {
          __builtin_amdgcn_sched_barrier(0);
          load_x8(cnn, 0);
          __builtin_amdgcn_sched_barrier(0);
        }
      });
      __builtin_amdgcn_sched_barrier(0);
      __syncthreads();
    }
  } else {
    u32x4 nh[KC / 8], nl[KC / 8];
    load_b(0, bh, bl);
    load_k(0);
    store_k(raw);
    __syncthreads();
    for (int c = 0; c < NCH; ++c) {
      const bool more = c + 1 < NCH;
      if (more) {
        load_b((c + 1) * KC, nh, nl);
        load_k((c + 1) * KC);
      }
      __builtin_amdgcn_sched_barrier(0);
      mma_chunk(raw + (c & 1) * KW, bh, bl, [](int) {});
      __builtin_amdgcn_sched_barrier(0);
      if (more) store_k(raw + ((c + 1) & 1) * KW);
      __syncthreads();
      if (more) {
#pragma unroll
        for (int s8 = 0; s8 < KC / 8; ++s8) {
          bh[s8] = nh[s8];
          bl[s8] = nl[s8];
        }
      }
    }
  }
  // kx phase of the fold, per register (kx of register v); column 0 holds
  // (Y[., 0], Y[., N/2]): phase 1 (the table's entry 0), and the Nyquist
  // output takes exp(i pi p_x)
  const float nyq_sign = (ix & 1) ? -1.f : 1.f;
  auto rotate = [&](int v) {
    const int kx = kt * 32 + (v >> 2) * 8 + 4 * h + (v & 3);
    const float2 ph = twf[(kx * ix * RX) % NY];
    const float sg = kx > 0 ? 1.f : nyq_sign;
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      const float yr = accr[t][v], yi = acci[t][v];
      accr[t][v] = yr * ph.x - yi * ph.y;
      acci[t][v] = (yr * ph.y + yi * ph.x) * sg;
    }
  };
  // Y as bf16 hi/lo A operands: k step s < 2 takes Yr, s >= 2 Yi, registers
  // 8 (s mod 2) .. 8 (s mod 2) + 7
  u32x4 yh[MT][4], yl[MT][4];
  auto split_y = [&](int t, int s4, int q) {
    const int v = 8 * (s4 & 1) + 2 * q;
    const f32x16& a = s4 < 2 ? accr[t] : acci[t];
    unsigned wh, wl;
    if constexpr (F16)  // |Y| <= 256 * 2^13: scaled by 2^-8 into the fp16 range (exact)
      split2_f16(a[v] * 0x1p-8f, a[v + 1] * 0x1p-8f, wh, wl);
    else
      split2(a[v], a[v + 1], wh, wl);
    yh[t][s4][q] = wh;
    yl[t][s4][q] = wl;
  };
  // before the first round only what its first k step needs (registers
  // 0..7 rotated, k step 0 split); the rest is placed between the first
  // round's matrix instructions (transition_hook below)
#pragma unroll
  for (int v = 0; v < 8; ++v) rotate(v);
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) split_y(t, 0, q);
  // Stage B per 32-column tile r of the grid: this wave's partial over its kx
  // slice, then the four partials added in wave order
  const int nr = Mp / 32;
  const size_t wplane = (size_t)nr * NKT * 4 * 64 * 8;
  const unsigned short* WPl = WP + wplane;
  u32x4 wh[4], wl[4], nwh[4], nwl[4];
  auto load_w = [&](int r, u32x4* dh, u32x4* dl) {
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const size_t off = ((((size_t)r * NKT + kt) * 4 + s4) * 64 + lane) * 8;
      dh[s4] = *(const u32x4*)(WP + off);
      dl[s4] = *(const u32x4*)(WPl + off);
    }
  };
  float* up = (float*)raw;
  unsigned long long best = 0;
  // One round's products: au = this wave's partial grid of one 32-column
  // tile over its kx slice; hook(slot) after each of the 60 instructions.
  auto round_mma = [&](f32x16* au, auto&& hook) {
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) au[t][v] = 0.f;
    int slot = 0;
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const u32x4 w_h = wh[s4], w_l = wl[s4];
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        au[t] = mfma32<F16>(yh[t][s4], w_h, au[t]);
        hook(slot++);
      }
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        au[t] = mfma32<F16>(yh[t][s4], w_l, au[t]);
        hook(slot++);
      }
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        au[t] = mfma32<F16>(yl[t][s4], w_h, au[t]);
        hook(slot++);
      }
    }
  };
  // the same products tile by tile (each tile's accumulation order as above,
  // so the sums are identical); hook(slot) after each instruction
  auto round_mma_t = [&](f32x16* au, auto&& hook) {
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) au[t][v] = 0.f;
    int slot = 0;
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        au[t] = mfma32<F16>(yh[t][s4], wh[s4], au[t]);
        hook(slot++);
        au[t] = mfma32<F16>(yh[t][s4], wl[s4], au[t]);
        hook(slot++);
        au[t] = mfma32<F16>(yl[t][s4], wh[s4], au[t]);
        hook(slot++);
      }
  };
  // this wave's partial grid, column-major: up[kt][mx][my] (mx = lane mod 32)
  auto write_tile = [&](const f32x16* au, int t) {
#pragma unroll
    for (int v4 = 0; v4 < 4; ++v4)
      *(f32x4*)(up + kt * UW + j * UST + t * 32 + v4 * 8 + 4 * h) =
          f32x4{au[t][4 * v4], au[t][4 * v4 + 1], au[t][4 * v4 + 2], au[t][4 * v4 + 3]};
  };
  auto write_up = [&](const f32x16* au) {
#pragma unroll
    for (int t = 0; t < MT; ++t) write_tile(au, t);
  };
  // The four partials of round r are added in wave order and their maximum
  // taken in MT items per thread (item it: four grid rows of one column),
  // each split into phases: its LDS reads, the sums, then one grid point's
  // key at a time.
  static_assert(32 * ROWS / 4 == MT * NTH, "MT reduction items per thread");
  f32x4 rq[NKT];
  f32x4 rsum;
  float rbv;  // the item's largest sum and its row offset
  int rbe;
  auto reduce_phase = [&](int r, int it, int ph) {
    const int i = tid + it * NTH;
    const int mxl = i / (ROWS / 4), my4 = i - mxl * (ROWS / 4);
    if (ph == 0) {
      const float* q = up + mxl * UST + 4 * my4;
#pragma unroll
      for (int w = 0; w < NKT; ++w) rq[w] = *(const f32x4*)(q + w * UW);
    } else if (ph == 1) {
      rsum = rq[0];
#pragma unroll
      for (int w = 1; w < NKT; ++w) {
        rsum[0] += rq[w][0];
        rsum[1] += rq[w][1];
        rsum[2] += rq[w][2];
        rsum[3] += rq[w][3];
      }
    } else if (ph == 2) {
      // the item's four grid points share a column and have increasing rows,
      // so increasing grid indices in either orientation: a strict compare in
      // that order keeps the lowest index among equal values, as the key
      // order does; points past M take part as -inf
      const int mx = r * 32 + mxl;
      const int my0 = m0 + 4 * my4;
      const bool cin = mx < g.M;
      rbv = (cin && my0 < g.M) ? rsum[0] : -INFINITY;
      rbe = 0;
#pragma unroll
      for (int e = 1; e < 4; ++e) {
        const float v = (cin && my0 + e < g.M) ? rsum[e] : -INFINITY;
        const bool gt = v > rbv;
        rbv = gt ? v : rbv;
        rbe = gt ? e : rbe;
      }
    } else if (ph == 3) {
      const int mx = r * 32 + mxl;
      // one key per item (a select, not a branch: an item with no grid point counts as key 0)
      unsigned long long key = peak_key(rbv, grid_index(m0 + 4 * my4 + rbe, mx, g.M, tr));
      key = rbv > -INFINITY ? key : 0ull;
      best = key > best ? key : best;
    }
  };
  // the first round's k steps 0..2 carry the rest of the rotation (registers
  // 8..15, before the split of k step 1) and the splits of k steps 1..3, each
  // done before the k step that reads it
  auto transition_hook = [&](int slot) {
    __builtin_amdgcn_sched_barrier(0);
    if (slot < 15) {
#pragma unroll
      for (int p = 2 * slot; p < 2 * slot + 2; ++p) {
        if (p < 8)
          rotate(8 + p);
        else if (p < 28)
          split_y((p - 8) / 4, 1, (p - 8) % 4);
      }
    } else if (slot < 45) {
      const int s4 = slot < 30 ? 2 : 3, base = slot < 30 ? 15 : 30;
#pragma unroll
      for (int i = 0; i < 4 * MT; ++i)
        if (base + (i * 15) / (4 * MT) == slot) split_y(i / 4, s4, i % 4);
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  static_assert(8 + 4 * MT <= 30, "the first k step's slots hold the rotation and the k step 1 split");
  f32x16 au[MT];
  load_w(0, wh, wl);
  if (nr > 1) load_w(1, nwh, nwl);
  round_mma(au, transition_hook);
  __syncthreads();  // Stage A's chunks are done with LDS
  write_up(au);
  __syncthreads();
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) {
    wh[s4] = nwh[s4];
    wl[s4] = nwl[s4];
  }
  // rounds after the first, tile by tile: round r's reduction in the first
  // 30 instruction slots (item it: reads after slot 6 it, sums after 6 it + 3,
  // its largest point after 6 it + 4, its key after 6 it + 5), then a barrier (every wave is done
  // reading round r's partials), then each finished tile's partial written
  // two instructions after its last one; the last tile's after the round
  static_assert(MT == 5, "tile-by-tile rounds laid out for five row tiles");
  auto round_hook = [&](int r, const f32x16* au) {
    return [&, r, au](int slot) {
      if (slot < 30) {
        const int it = slot / 6, k = slot - 6 * it;
        if (k == 0 || k == 3 || k == 4 || k == 5) {
          __builtin_amdgcn_sched_barrier(0);
          reduce_phase(r, it, k == 0 ? 0 : k - 2);
          __builtin_amdgcn_sched_barrier(0);
        }
        if (slot == 29) {
          __builtin_amdgcn_sched_barrier(0);
          __syncthreads();
          __builtin_amdgcn_sched_barrier(0);
        }
      } else {
        // tiles 0 and 1 are complete by the barrier; tile t >= 2 after slot 12 t + 11
        const int t = slot == 30 ? 0 : slot == 31 ? 1 : (slot >= 37 && (slot - 37) % 12 == 0) ? 2 + (slot - 37) / 12 : -1;
        if (t >= 0 && t < MT - 1) {
          __builtin_amdgcn_sched_barrier(0);
          write_tile(au, t);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    };
  };
  for (int r = 0; r < nr; ++r) {
    const bool more = r + 1 < nr;
    if (r + 2 < nr) load_w(r + 2, nwh, nwl);
    if (more) {
      round_mma_t(au, round_hook(r, au));
      write_tile(au, MT - 1);
      __syncthreads();
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        wh[s4] = nwh[s4];
        wl[s4] = nwl[s4];
      }
    } else {
#pragma unroll
      for (int it = 0; it < MT; ++it)
#pragma unroll
        for (int ph = 0; ph < 4; ++ph) reduce_phase(r, it, ph);
    }
  }
  best = wmax64(best);
  if (lane == 0) red[wave] = best;
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < NTH / 64; ++w) best = red[w] > best ? red[w] : best;
    atomicMax(&g.st[f].grid_key, best);
  }
}

// Folded split table for the wide kernels: K'_p[m, ky] = phi_ky(p + (m - c)/u)
// for every integer peak row p of frames of N rows, as bf16 (f16: fp16) hi/lo
// words (re | im << 16), [N][2][Mp][xb_pitch(N)], computed in FP64 with
// exactly reduced phases.
__global__ void k_build_kfold(unsigned* __restrict__ out, int N, int u, int M, int c, int rows, int P,
                              int f16) {
  const size_t plane = (size_t)rows * P;
  const size_t total = (size_t)N * plane;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int iy = (int)(e / plane);
    const size_t rem = e - (size_t)iy * plane;
    const int m = (int)(rem / P), ky = (int)(rem % P);
    double re = 0.0, im = 0.0;
    if (m < M && ky < N) {
      const long t = (long)iy * u + (m - c);  // position in units of 1/u
      if (2 * ky == N) {
        const long per = 2L * u;  // cos(pi t / u)
        const long r = ((t % per) + per) % per;
        re = cospi((double)r / (double)u);
      } else {
        const int kt = 2 * ky < N ? ky : ky - N;
        const long per = (long)u * N;  // angle 2 pi kt t / (u N)
        const long r = (((long)kt * t) % per + per) % per;
        double sn, cs;
        sincospi(2.0 * (double)r / (double)per, &sn, &cs);
        re = cs;
        im = sn;
      }
    }
    const size_t base = (size_t)iy * 2 * plane + (size_t)m * P + ky;
    if (f16) {  // fp16 hi/lo words (the fp16 split)
      const unsigned h = f16_pack((float)re, (float)im);
      out[base] = h;
      out[base + plane] = f16_pack((float)(re - (double)f16_lo_float(h)), (float)(im - (double)f16_hi_float(h)));
      continue;
    }
    const unsigned hr = bf16_bits((float)re), hm = bf16_bits((float)im);
    const unsigned lr = bf16_bits((float)(re - (double)bf16_float(hr)));
    const unsigned lm = bf16_bits((float)(im - (double)bf16_float(hm)));
    out[base] = hr | (hm << 16);
    out[base + plane] = lr | (lm << 16);
  }
}

int launch_build_kfold(unsigned* out, int N, int u, int M, int c, int rows, int f16, hipStream_t s) {
  hipLaunchKernelGGL(k_build_kfold, dim3(4096), dim3(256), 0, s, out, N, u, M, c, rows, xb_pitch(N), f16);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int NY, int NX>
static int updft_n(const GroupParams& g, const UpdftTables& t, hipStream_t s) {
  const int mtiles = t.Mp / 32;
  if (t.precision == CCPT_PREC_FP32) {
    constexpr int NCH = NY / a_chunk(NY, NX);
    const int nsl = NCH < kSplitSlices ? NCH : kSplitSlices;
    if (g.ypart && nsl > 1) {  // (the plan decided the split: a partials buffer)
      hipLaunchKernelGGL((k_updft_f32<NY, NX, true>), dim3(mtiles, g.count, nsl), dim3(kUThreads),
                         0, s, g, (const float2*)t.ky, (const float*)t.wb, t.Mp, g.ypart, nsl);
      const int ncg = (t.Mp / 16 + kSumColTiles - 1) / kSumColTiles;
      hipLaunchKernelGGL((k_updft_f32_sum<NY, NX>), dim3(mtiles, g.count, ncg), dim3(kUThreads), 0, s,
                         g, (const float*)t.wb, t.Mp, (const float*)g.ypart, nsl);
    } else {
      hipLaunchKernelGGL((k_updft_f32<NY, NX, false>), dim3(mtiles, g.count), dim3(kUThreads), 0,
                         s, g, (const float2*)t.ky, (const float*)t.wb, t.Mp, (float*)nullptr, 1);
    }
  } else if (t.precision == CCPT_PREC_FP16X2) {
    // the fp16 split: 256 x 256 frames through the one-kernel correlation only
    if constexpr (NY == 256 && NX == 256) {
      if (g.Xb || !g.Zc || !t.kfold) return -2;
      hipLaunchKernelGGL((k_updft_bf16x2_t256<NY, kWideMT, true, true>),
                         dim3((mtiles + kWideMT - 1) / kWideMT, g.count), dim3(256), 0, s, g,
                         (const unsigned*)t.kfold, (const unsigned short*)t.wb, t.Mp);
    } else {
      return -2;
    }
  } else if (t.precision == CCPT_PREC_BF16X2) {
    if (!g.Xb && !(NY == 256 && NX == 256 && g.Zc)) return -1;
    if constexpr (NX >= kWideMinN) {
      constexpr int MT = kWideMT;
      constexpr int NW = (NX / 2 + 31) / 32;
      if (!t.kfold) return -1;
      if constexpr (NX == 256) {
        static_assert(NW == 4, "four kx tiles");
        if constexpr (NY == 256) {
          if (!g.Xb) {  // the one-kernel correlation left X and its packed column
            if (!g.Zc) return -1;
            hipLaunchKernelGGL((k_updft_bf16x2_t256<NY, MT, true, false>),
                               dim3((mtiles + MT - 1) / MT, g.count), dim3(256), 0, s, g,
                               (const unsigned*)t.kfold, (const unsigned short*)t.wb, t.Mp);
            return hipGetLastError() == hipSuccess ? 0 : -1;
          }
        }
        hipLaunchKernelGGL((k_updft_bf16x2_t256<NY, MT, false, false>), dim3((mtiles + MT - 1) / MT, g.count),
                           dim3(256), 0, s, g, (const unsigned*)t.kfold, (const unsigned short*)t.wb,
                           t.Mp);
      } else {
        hipLaunchKernelGGL((k_updft_bf16x2_wide<NY, NX, MT>),
                           dim3((mtiles + MT - 1) / MT, g.count), dim3(64 * NW), 0, s, g,
                           (const unsigned*)t.kfold, (const unsigned short*)t.wb, t.Mp);
      }
    } else {
      hipLaunchKernelGGL((k_updft_bf16x2<NY, NX>), dim3(mtiles, g.count), dim3(kUThreads), 0, s,
                         g, (const float2*)t.ky, (const unsigned short*)t.wb, t.Mp);
    }
  } else {
    return -2;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_updft(int ny, int nx, const GroupParams& g, const UpdftTables& t, hipStream_t s) {
  if (ny == nx) {
    switch (ny) {
#define CASE(n) \
  case n:       \
    return updft_n<n, n>(g, t, s);
      CCPT_FOR_SIZES(CASE)
#undef CASE
    }
    return -2;
  }
#define CASE(a, b) \
  if (ny == a && nx == b) return updft_n<a, b>(g, t, s);
  CCPT_FOR_RECT(CASE)
#undef CASE
  return -2;
}

}  // namespace ccpt
