// Correlation stage of the tracker (Sec. II Eq. 4 / Eq. 7, Sec. III first
// paragraph): prologue A = I or (I+eps)^2, forward 2-D r2c FFT, product with
// the resident conj F[B], inverse 2-D c2r FFT and the integer-lag maximum.
//
// The 2-D transforms are split into a row pass (each row of N reals is
// packed as N/2 complex values, transformed, and unpacked into N/2+1 bins)
// and a column pass over the N/2+1 columns.  Both passes keep their data in
// LDS and exchange it through a per-frame workspace that stays in the
// L2/Infinity-Cache for the chunk sizes used.
#include <hip/hip_runtime.h>

#include "common.h"
#include "fft.h"

namespace ccpt {

// 512 threads (8 waves) per block: the passes are bound by memory latency
// and LDS, so more resident waves per CU (16 to 32) hide more of it
constexpr int kThreads = 512;

// Frames are NY rows of NX pixels (NY = NX, or NY = 2^k NX).

// largest divisor of NY whose block of rows (NX/2 complex values each) holds
// at most `budget` complex values
constexpr int rows_per_block(int NY, int NX, int budget) {
  int best = 1;
  for (int r = 1; r <= NY; ++r)
    if (NY % r == 0 && r * (NX / 2) <= budget) best = r;
  return best;
}

// columns per block of the column pass: at most 2048 complex values per
// LDS buffer (8 columns of 256: 37 KB of LDS, so four blocks share a CU),
// no wider than the NX/2+1 columns need
constexpr int cols_per_block(int NY, int NX) {
  int cb = 1;
  while (cb * 2 * NY <= 2048 && cb < NX / 2) cb *= 2;
  return cb;
}

// rows per block of the row passes: 16 rows (128-byte runs of the
// column-major intermediate) when they fit, else the largest divisor of NY
constexpr int row_block(int NY, int NX) {
  return (NY % 16 == 0 && 16 * (NX / 2 + 1) <= 4200) ? 16 : rows_per_block(NY, NX, 2048);
}

// the same choices for FP64 data (square frames; half the values per LDS buffer)
constexpr int cols_per_block64(int N) {
  int cb = 1;
  while (cb * 2 * N <= 2048 && cb < N / 2) cb *= 2;
  return cb;
}
template <typename C>
constexpr int row_block_of(int NY, int NX) {
  return sizeof(C) == sizeof(float2) ? row_block(NY, NX) : row_block64(NY);
}
template <typename C>
constexpr int cols_block_of(int NY, int NX) {
  return sizeof(C) == sizeof(float2) ? cols_per_block(NY, NX) : cols_per_block64(NY);
}

template <typename R>
__device__ __forceinline__ R load_px(const void* p, int dtype, long idx) {
  if (dtype == CCPT_U16) return (R)((const unsigned short*)p)[idx];
  if (dtype == CCPT_F64) return (R)((const double*)p)[idx];
  return (R)((const float*)p)[idx];
}

// Where a row pass reads its images from.
struct ImgSrc {
  const FrameDesc* desc;  // frames (desc[first + f]) or null
  int first;
  const void* data;  // when desc is null: image f at data + f * img_stride elements
  int dtype;
  int pitch;
  long img_stride;
  int trans;  // read each image transposed (a wide frame held tall)
};

__device__ __forceinline__ void img_of(const ImgSrc& s, int f, const void*& data, int& dtype,
                                       int& pitch) {
  if (s.desc) {
    const FrameDesc d = s.desc[s.first + f];
    data = d.data;
    dtype = d.dtype;
    pitch = d.pitch;
  } else {
    dtype = s.dtype;
    pitch = s.pitch;
    data = (const char*)s.data + (size_t)f * s.img_stride * dtype_bytes(dtype);
  }
}

template <typename T>
__device__ __forceinline__ T wave_max_u64(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

__device__ __forceinline__ unsigned wave_min_u32(unsigned v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, (unsigned)__shfl_xor((int)v, o, 64));
  return v;
}
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, o, 64));
  return v;
}

__global__ void k_init_state(FrameState* st, int count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    FrameState s;
    s.peak_key = 0;
    s.grid_key = 0;
    s.second_key = 0;
    s.amin = 0xFFFFFFFFu;
    s.amax = 0;
    s.flags = 0;
    s.xmax = 0;
    st[i] = s;
  }
}

// Row pass, forward.  weight: 0 A = I, 1 B = -1/(E+eps), 2 A = (I+eps)^2.
// Writes T[f][k][y] (column-major), k < NX/2+1.  With st != null records
// min/max of A (as FP32 keys) and non-finite pixels per frame.  C = float2
// or double2 sets the arithmetic.
template <int NY, int NX, int RPB, typename C>
__global__ void __launch_bounds__(kThreads) k_rows_fwd(ImgSrc src, int weight, double eps_in,
                                                       C* __restrict__ T, FrameState* st,
                                                       const C* __restrict__ gtw) {
  using R = real_t<C>;
  constexpr int L = NX / 2, H = NX / 2 + 1;
  constexpr int LS = lds_len(L) + 1;  // row stride in LDS
  const R eps = (R)eps_in;
  __shared__ C tw[NX];
  __shared__ C bufA[RPB * LS];
  __shared__ C bufB[RPB * LS];
  __shared__ unsigned red[3][kThreads / 64];
  const int tid = threadIdx.x;
  const int f = blockIdx.y;
  const int y0 = blockIdx.x * RPB;
  for (int i = tid; i < NX; i += kThreads) tw[i] = gtw[i * (NY / NX)];
  const void* data;
  int dtype, pitch;
  img_of(src, f, data, dtype, pitch);
  unsigned kmin = 0xFFFFFFFFu, kmax = 0, bad = 0;
  auto pro = [&](R a) {
    if (weight == 1) a = R(-1) / (a + eps);
    else if (weight == 2) a = (a + eps) * (a + eps);
    if (!isfinite(a)) bad = 1;
    kmin = min(kmin, f2key((float)a));
    kmax = max(kmax, f2key((float)a));
    return a;
  };
  const bool trans = transposed<NY, NX>(src.trans);
  const bool vec16 = !trans && dtype == CCPT_U16 && NX % 8 == 0 && pitch % 8 == 0 &&
                     ((uintptr_t)data & 15) == 0;
  const bool vec32 = !trans && dtype == CCPT_F32 && NX % 4 == 0 && pitch % 4 == 0 &&
                     ((uintptr_t)data & 15) == 0;
  if (vec16) {
    // 8 pixels (16 bytes) per load
    for (int i = tid; i < RPB * (NX / 8); i += kThreads) {
      const int r = i / (NX / 8), q = i - r * (NX / 8);
      const uint4 v = *(const uint4*)((const unsigned short*)data + (long)(y0 + r) * pitch + 8 * q);
      const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 4; ++e)
        bufA[r * LS + lds_idx(4 * q + e)] = mkc<C>(pro((R)(w[e] & 0xFFFFu)), pro((R)(w[e] >> 16)));
    }
  } else if (vec32) {
    for (int i = tid; i < RPB * (NX / 4); i += kThreads) {
      const int r = i / (NX / 4), q = i - r * (NX / 4);
      const float4 v = *(const float4*)((const float*)data + (long)(y0 + r) * pitch + 4 * q);
      bufA[r * LS + lds_idx(2 * q)] = mkc<C>(pro((R)v.x), pro((R)v.y));
      bufA[r * LS + lds_idx(2 * q + 1)] = mkc<C>(pro((R)v.z), pro((R)v.w));
    }
  } else if (trans) {
    // row y of the tall image is column y of the wide frame: adjacent threads
    // take adjacent columns of one frame row
    for (int i = tid; i < RPB * L; i += kThreads) {
      const int c = i / RPB, r = i - c * RPB;
      const long idx = (long)(2 * c) * pitch + (y0 + r);
      const R a0 = pro(load_px<R>(data, dtype, idx));
      const R a1 = pro(load_px<R>(data, dtype, idx + pitch));
      bufA[r * LS + lds_idx(c)] = mkc<C>(a0, a1);
    }
  } else {
    for (int i = tid; i < RPB * L; i += kThreads) {
      const int r = i / L, c = i - r * L;
      const long idx = (long)(y0 + r) * pitch + 2 * c;
      const R a0 = pro(load_px<R>(data, dtype, idx));
      const R a1 = pro(load_px<R>(data, dtype, idx + 1));
      bufA[r * LS + lds_idx(c)] = mkc<C>(a0, a1);
    }
  }
  if (st) {
    kmin = wave_min_u32(kmin);
    kmax = wave_max_u32(kmax);
    bad = wave_max_u32(bad);
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = kmin;
      red[1][tid >> 6] = kmax;
      red[2][tid >> 6] = bad;
    }
  }
  __syncthreads();
  if (st && tid == 0) {
    for (int w = 1; w < kThreads / 64; ++w) {
      kmin = min(kmin, red[0][w]);
      kmax = max(kmax, red[1][w]);
      bad |= red[2][w];
    }
    atomicMin(&st[f].amin, kmin);
    atomicMax(&st[f].amax, kmax);
    if (bad) atomicOr(&st[f].flags, (unsigned)CCPT_ST_NONFINITE);
  }
  C* z = fft_lds<L, -1, NX>(bufA, bufB, RPB, LS, tw);
  // unpack: X[k] = E[k] + W^k O[k], E = (Z[k] + conj Z[L-k]) / 2,
  // O = (Z[k] - conj Z[L-k]) / (2i), W = exp(-2 pi i / NX); stored column-major
  // T[k][y] so each column k receives RPB consecutive rows
  C* Tf = T + (size_t)f * NY * H;
  const R half = R(0.5);
  for (int i = tid; i < RPB * H; i += kThreads) {
    const int k = i / RPB, r = i - k * RPB;
    const C zk = z[r * LS + lds_idx(k == L ? 0 : k)];
    const C zc = cconj(z[r * LS + lds_idx(k == 0 ? 0 : L - k)]);
    const C e = cscale(cadd(zk, zc), half);
    const C d = csub(zk, zc);
    const C o = mkc<C>(half * d.y, -half * d.x);  // d / (2i)
    Tf[(size_t)k * NY + y0 + r] = cadd(e, cmul(tw[k], o));
  }
}

enum ColKind { COL_XCORR = 0, COL_FWD = 1, COL_FWD_CONJ = 2, COL_INV = 3 };

// Column pass over the NX/2+1 columns of length NY: block b takes columns
// b*CB .. b*CB+CB-1 of the first NX/2, and block 0 also takes the Nyquist
// column NX/2 (so no
// block is left with a single column, and block 0 holds both real-output
// columns 0 and N/2 for the packed split-precision copy).
//  COL_XCORR:    forward FFT, X = F[A] * rspec (stored to X), inverse FFT back into T
//  COL_FWD:      forward FFT stored to `spec`
//  COL_FWD_CONJ: conjugate of the forward FFT stored to `spec`
//  COL_INV:      inverse FFT of `spec` stored to T
template <int NY, int NX, int CB, int KIND, typename C>
__global__ void __launch_bounds__(kThreads) k_cols(const FrameDesc* __restrict__ desc, int first,
                                                   C* __restrict__ T, C* __restrict__ X,
                                                   unsigned* __restrict__ Xb,
                                                   C* __restrict__ spec, long spec_stride,
                                                   const C* __restrict__ gtw) {
  constexpr int H = NX / 2 + 1, S = lds_len(NY) + 1, NC = NX / 2;
  constexpr int CS = CB + 1;  // column slots: CB regular + the Nyquist slot of block 0
  const C zero = mkc<C>(0, 0);
  __shared__ C tw[NY];
  __shared__ C bufA[CS * S];
  __shared__ C bufB[CS * S];
  const int tid = threadIdx.x;
  const int f = blockIdx.y;
  const int c0 = blockIdx.x * CB;
  const int nreg = min(CB, NC - c0);       // regular columns of this block
  const bool has_nyq = blockIdx.x == 0;
  const int nseq = has_nyq ? CS : CB;
  // slot -> column index (-1 when empty)
  auto col_of = [&](int c) { return c < nreg ? c0 + c : (c == CB && has_nyq ? NC : -1); };
  for (int i = tid; i < NY; i += kThreads) tw[i] = gtw[i];
  // T is column-major: column kx holds NY consecutive rows
  C* Tf = T + (size_t)f * NY * H;
  if constexpr (KIND == COL_INV) {
    const C* inp = spec + (size_t)f * spec_stride;  // row-major spectrum
    for (int i = tid; i < NY * nseq; i += kThreads) {
      const int y = i / nseq, c = i - y * nseq;
      const int kx = col_of(c);
      bufA[c * S + lds_idx(y)] = kx >= 0 ? inp[(size_t)y * H + kx] : mkc<C>(0, 0);
    }
  } else {
    for (int i = tid; i < NY * nseq; i += kThreads) {
      const int c = i / NY, y = i - c * NY;
      const int kx = col_of(c);
      bufA[c * S + lds_idx(y)] = kx >= 0 ? Tf[(size_t)kx * NY + y] : mkc<C>(0, 0);
    }
  }
  __syncthreads();
  if constexpr (KIND == COL_INV) {
    C* r = fft_lds<NY, +1, NY>(bufA, bufB, nseq, S, tw);
    for (int i = tid; i < NY * nseq; i += kThreads) {
      const int c = i / NY, y = i - c * NY;
      const int kx = col_of(c);
      if (kx >= 0) Tf[(size_t)kx * NY + y] = r[c * S + lds_idx(y)];
    }
  } else {
    C* r = fft_lds<NY, -1, NY>(bufA, bufB, nseq, S, tw);
    if constexpr (KIND == COL_FWD || KIND == COL_FWD_CONJ) {
      C* out = spec + (size_t)f * spec_stride;
      for (int i = tid; i < NY * nseq; i += kThreads) {
        const int y = i / nseq, c = i - y * nseq;
        const int kx = col_of(c);
        if (kx >= 0) {
          C v = r[c * S + lds_idx(y)];
          if (KIND == COL_FWD_CONJ) v.y = -v.y;
          out[(size_t)y * H + kx] = v;
        }
      }
    } else {
      const C* R = (const C*)desc[first + f].rspec;
      C* Xf = X + (size_t)f * NY * H;
      for (int i = tid; i < NY * nseq; i += kThreads) {
        const int y = i / nseq, c = i - y * nseq;
        const int kx = col_of(c);
        if (kx >= 0) {
          const C v = cmul(r[c * S + lds_idx(y)], R[(size_t)y * H + kx]);
          Xf[(size_t)y * H + kx] = v;
          r[c * S + lds_idx(y)] = v;
        } else {
          r[c * S + lds_idx(y)] = zero;
        }
      }
      __syncthreads();
      if constexpr (sizeof(C) == sizeof(float2)) {
      if (Xb) {
        // bf16 hi/lo split of X for the matrix cores: one row per column
        // kx < NX/2, ky contiguous, rows padded to xb_pitch(NY) with zeros.
        // Row 0 carries Z = X[., 0] + i X[., NX/2]: both columns give real
        // Stage A outputs, so Re and Im of the product with Z are the two of
        // them.  The DC term X[0, 0] is dropped.
        constexpr int P = xb_pitch(NY);
        unsigned* hi = Xb + (size_t)f * 2 * NC * P;
        unsigned* lo = hi + (size_t)NC * P;
        for (int i = tid; i < nreg * P; i += kThreads) {
          const int c = i / P, y = i - c * P;
          const int kx = c0 + c;
          float2 v = make_float2(0.f, 0.f);
          if (y < NY) {
            v = r[c * S + lds_idx(y)];
            if (kx == 0) {
              if (y == 0) v.x = 0.f;
              const float2 nq = r[CB * S + lds_idx(y)];
              v = make_float2(v.x - nq.y, v.y + nq.x);  // + i * X[y, N/2]
            }
          }
          unsigned wh, wl;
          split_pair(v, wh, wl);
          hi[(size_t)kx * P + y] = wh;
          lo[(size_t)kx * P + y] = wl;
        }
      }
      }
      C* o = (r == bufA) ? bufB : bufA;
      C* q = fft_lds<NY, +1, NY>(r, o, nseq, S, tw);
      for (int i = tid; i < NY * nseq; i += kThreads) {
        const int c = i / NY, y = i - c * NY;
        const int kx = col_of(c);
        if (kx >= 0) Tf[(size_t)kx * NY + y] = q[c * S + lds_idx(y)];
      }
    }
  }
}

// Row pass, inverse (c2r).  Each row's NX/2+1 bins are packed into NX/2
// complex values Z = E + i O with E = (X[k] + conj X[L-k]) / 2 and
// O = (X[k] - conj X[L-k]) W^-k / 2, transformed, and read out as the NX
// reals z[n] = a[2n] + i a[2n+1].
// ARGMAX: per-frame maximum with ties to the lowest row-major index of the
// frame (trans: of the wide frame, whose row-major order is the tall image's
// column-major order): in FP32 one 64-bit atomic key per frame, in FP64 one
// candidate per row block (cand[f][blockIdx.x]).  Otherwise the real row is
// scaled and stored to img (NY x NX per frame, FP32 only).
template <int NY, int NX, int RPB, bool ARGMAX, typename C>
__global__ void __launch_bounds__(kThreads) k_rows_inv(const C* __restrict__ T, FrameState* st,
                                                       float* img, float scale,
                                                       const C* __restrict__ gtw,
                                                       PeakCand* __restrict__ cand, int trans_in) {
  using R = real_t<C>;
  constexpr bool FP64 = sizeof(C) != sizeof(float2);
  constexpr int L = NX / 2, H = NX / 2 + 1;
  constexpr int LS = lds_len(L) + 1;
  __shared__ C tw[NX];
  __shared__ C raw[RPB * H];
  __shared__ C bufA[RPB * LS];
  __shared__ C bufB[RPB * LS];
  __shared__ unsigned long long red[kThreads / 64], red2[kThreads / 64];
  __shared__ double redv[kThreads / 64], redv2[kThreads / 64];
  const int tid = threadIdx.x;
  const int f = blockIdx.y;
  const int y0 = blockIdx.x * RPB;
  for (int i = tid; i < NX; i += kThreads) tw[i] = gtw[i * (NY / NX)];
  // column-major T: column k holds rows y0..y0+RPB-1 consecutively
  const C* Tf = T + (size_t)f * NY * H + y0;
  for (int i = tid; i < RPB * H; i += kThreads) {
    const int k = i / RPB, r = i - k * RPB;
    raw[r * H + k] = Tf[(size_t)k * NY + r];
  }
  // frame row-major index of tall pixel (y, x), and the step to (y, x + 1)
  const bool trans = transposed<NY, NX>(trans_in);
  auto flat_of = [&](int y, int x) {
    return trans ? (unsigned)(x * NY + y) : (unsigned)(y * NX + x);
  };
  const unsigned xstep = trans ? (unsigned)NY : 1u;
  __syncthreads();
  const R half = R(0.5);
  for (int i = tid; i < RPB * L; i += kThreads) {
    const int r = i / L, k = i - r * L;
    const C xk = raw[r * H + k];
    const C xc = cconj(raw[r * H + L - k]);
    const C e = cscale(cadd(xk, xc), half);
    const C o = cmul(cscale(csub(xk, xc), half), cconj(tw[k]));
    bufA[r * LS + lds_idx(k)] = mkc<C>(e.x - o.y, e.y + o.x);  // e + i o
  }
  __syncthreads();
  C* z = fft_lds<L, +1, NX>(bufA, bufB, RPB, LS, tw);
  if constexpr (ARGMAX && !FP64) {
    // the two largest keys of the block (keys are unique: they hold the index)
    unsigned long long best = 0, second = 0;
    auto push = [&](unsigned long long k) {  // branch-free top-two insertion
      const unsigned long long lo = k < best ? k : best;
      best = k < best ? best : k;
      second = second < lo ? lo : second;
    };
    for (int i = tid; i < RPB * L; i += kThreads) {
      const int r = i / L, n = i - r * L;
      const C v = z[r * LS + lds_idx(n)];
      const unsigned flat = flat_of(y0 + r, 2 * n);
      push(peak_key(v.x, flat));
      push(peak_key(v.y, flat + xstep));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long b1 = __shfl_xor(best, o, 64), b2 = __shfl_xor(second, o, 64);
      const unsigned long long lo = b1 < best ? b1 : best;
      second = second > b2 ? second : b2;
      second = second > lo ? second : lo;
      best = b1 > best ? b1 : best;
    }
    if ((tid & 63) == 0) {
      red[tid >> 6] = best;
      red2[tid >> 6] = second;
    }
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < kThreads / 64; ++w) {
        push(red[w]);
        push(red2[w]);
      }
      // the frame's runner-up is some block's second or the smaller of two
      // block maxima meeting in the atomic: submit both
      const unsigned long long old = atomicMax(&st[f].peak_key, best);
      const unsigned long long lose = old < best ? old : best;
      atomicMax(&st[f].second_key, second > lose ? second : lose);
    }
  } else if constexpr (ARGMAX) {
    // (value, index) pairs: larger value wins, equal values go to the lower
    // index; NaN never wins.  sv: the runner-up value.
    double bv = -__builtin_inf(), sv = -__builtin_inf();
    unsigned bi = 0xFFFFFFFFu;
    auto take = [&](double v, unsigned i) {
      if (v > bv || (v == bv && i < bi)) {
        sv = bv;
        bv = v;
        bi = i;
      } else if (v > sv) {
        sv = v;
      }
    };
    for (int i = tid; i < RPB * L; i += kThreads) {
      const int r = i / L, n = i - r * L;
      const C v = z[r * LS + lds_idx(n)];
      const unsigned flat = flat_of(y0 + r, 2 * n);
      take(v.x, flat);
      take(v.y, flat + xstep);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64), os = __shfl_xor(sv, o, 64);
      const unsigned oi = (unsigned)__shfl_xor((int)bi, o, 64);
      take(ov, oi);
      sv = os > sv ? os : sv;
    }
    if ((tid & 63) == 0) {
      redv[tid >> 6] = bv;
      redv2[tid >> 6] = sv;
      red[tid >> 6] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < kThreads / 64; ++w) {
        take(redv[w], (unsigned)red[w]);
        sv = redv2[w] > sv ? redv2[w] : sv;
      }
      PeakCand pc;
      pc.v = bv;
      pc.v2 = sv;
      pc.idx = bi;
      pc.pad = 0;
      cand[(size_t)f * gridDim.x + blockIdx.x] = pc;
    }
  } else if constexpr (!FP64) {
    float* out = img + (size_t)f * NY * NX + (size_t)y0 * NX;
    for (int i = tid; i < RPB * L; i += kThreads) {
      const int r = i / L, n = i - r * L;
      const C v = z[r * LS + lds_idx(n)];
      out[r * NX + 2 * n] = v.x * scale;
      out[r * NX + 2 * n + 1] = v.y * scale;
    }
  }
}

template <int NY, int NX>
static int xcorr_n(const GroupParams& g, hipStream_t s, const Marker& mark) {
  constexpr int RPB = row_block(NY, NX);
  constexpr int CB = cols_per_block(NY, NX);
  ImgSrc src{g.desc, g.first, nullptr, 0, 0, 0, g.trans};
  mark(CCPT_STAGE_ROWS_FWD, 1);
  hipLaunchKernelGGL((k_rows_fwd<NY, NX, RPB, float2>), dim3(NY / RPB, g.count), dim3(kThreads), 0,
                     s, src, g.mode == CCPT_MODE_CCSN ? 2 : 0, (double)g.eps, g.T, g.st, g.tw);
  mark(CCPT_STAGE_ROWS_FWD, 0);
  mark(CCPT_STAGE_COLS, 1);
  hipLaunchKernelGGL((k_cols<NY, NX, CB, COL_XCORR, float2>), dim3((NX / 2 + CB - 1) / CB, g.count),
                     dim3(kThreads), 0, s, g.desc, g.first, g.T, g.X, g.Xb, (float2*)nullptr, 0L,
                     g.tw);
  mark(CCPT_STAGE_COLS, 0);
  mark(CCPT_STAGE_ROWS_INV, 1);
  hipLaunchKernelGGL((k_rows_inv<NY, NX, RPB, true, float2>), dim3(NY / RPB, g.count),
                     dim3(kThreads), 0, s, g.T, g.st, (float*)nullptr, 1.0f, g.tw,
                     (PeakCand*)nullptr, g.trans);
  mark(CCPT_STAGE_ROWS_INV, 0);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int N>
static int xcorr64_n(const GroupParams& g, hipStream_t s, const Marker& mark) {
  constexpr int RPB = row_block64(N);
  constexpr int CB = cols_per_block64(N);
  ImgSrc src{g.desc, g.first, nullptr, 0, 0, 0, 0};
  mark(CCPT_STAGE_ROWS_FWD, 1);
  hipLaunchKernelGGL((k_rows_fwd<N, N, RPB, double2>), dim3(N / RPB, g.count), dim3(kThreads), 0,
                     s, src, g.mode == CCPT_MODE_CCSN ? 2 : 0, g.eps64, g.T64, g.st, g.tw64);
  mark(CCPT_STAGE_ROWS_FWD, 0);
  mark(CCPT_STAGE_COLS, 1);
  hipLaunchKernelGGL((k_cols<N, N, CB, COL_XCORR, double2>), dim3((N / 2 + CB - 1) / CB, g.count),
                     dim3(kThreads), 0, s, g.desc, g.first, g.T64, g.X64, (unsigned*)nullptr,
                     (double2*)nullptr, 0L, g.tw64);
  mark(CCPT_STAGE_COLS, 0);
  mark(CCPT_STAGE_ROWS_INV, 1);
  hipLaunchKernelGGL((k_rows_inv<N, N, RPB, true, double2>), dim3(N / RPB, g.count),
                     dim3(kThreads), 0, s, g.T64, g.st, (float*)nullptr, 1.0f, g.tw64, g.cand, 0);
  mark(CCPT_STAGE_ROWS_INV, 0);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int NY, int NX, typename C>
static int spectrum_n(const void* data, int dtype, int pitch, long img_stride, int trans, int n,
                      int weight, double eps, int conj_out, C* T, C* spec, const C* tw,
                      hipStream_t s) {
  constexpr int RPB = row_block_of<C>(NY, NX);
  constexpr int CB = cols_block_of<C>(NY, NX);
  constexpr int H = NX / 2 + 1;
  ImgSrc src{nullptr, 0, data, dtype, pitch, img_stride, trans};
  hipLaunchKernelGGL((k_rows_fwd<NY, NX, RPB, C>), dim3(NY / RPB, n), dim3(kThreads), 0, s, src,
                     weight, eps, T, (FrameState*)nullptr, tw);
  if (conj_out)
    hipLaunchKernelGGL((k_cols<NY, NX, CB, COL_FWD_CONJ, C>), dim3((NX / 2 + CB - 1) / CB, n),
                       dim3(kThreads), 0, s, (const FrameDesc*)nullptr, 0, T, (C*)nullptr,
                       (unsigned*)nullptr, spec, (long)NY * H, tw);
  else
    hipLaunchKernelGGL((k_cols<NY, NX, CB, COL_FWD, C>), dim3((NX / 2 + CB - 1) / CB, n),
                       dim3(kThreads), 0, s, (const FrameDesc*)nullptr, 0, T, (C*)nullptr,
                       (unsigned*)nullptr, spec, (long)NY * H, tw);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Spectra of frames given by descriptors, held tall (trans: the frames are
// wide and read transposed): T and spec as in the tracking passes.
template <int NY, int NX>
static int frame_spectra_n(const FrameDesc* desc, int first, int count, int mode, float eps,
                           int trans, float2* T, float2* spec, const float2* tw, hipStream_t s) {
  constexpr int RPB = row_block(NY, NX);
  constexpr int CB = cols_per_block(NY, NX);
  constexpr int H = NX / 2 + 1;
  ImgSrc src{desc, first, nullptr, 0, 0, 0, trans};
  hipLaunchKernelGGL((k_rows_fwd<NY, NX, RPB, float2>), dim3(NY / RPB, count), dim3(kThreads), 0,
                     s, src, mode == CCPT_MODE_CCSN ? 2 : 0, (double)eps, T, (FrameState*)nullptr,
                     tw);
  hipLaunchKernelGGL((k_cols<NY, NX, CB, COL_FWD, float2>), dim3((NX / 2 + CB - 1) / CB, count),
                     dim3(kThreads), 0, s, (const FrameDesc*)nullptr, 0, T, (float2*)nullptr,
                     (unsigned*)nullptr, spec, (long)NY * H, tw);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Real images (NY rows of NX, the tall layout) from half spectra.
template <int NY, int NX>
static int inverse_n(const float2* spec, int n, float scale, float2* T, float* img,
                     const float2* tw, hipStream_t s) {
  constexpr int RPB = row_block(NY, NX);
  constexpr int CB = cols_per_block(NY, NX);
  constexpr int H = NX / 2 + 1;
  hipLaunchKernelGGL((k_cols<NY, NX, CB, COL_INV, float2>), dim3((NX / 2 + CB - 1) / CB, n),
                     dim3(kThreads), 0, s, (const FrameDesc*)nullptr, 0, T, (float2*)nullptr,
                     (unsigned*)nullptr, (float2*)spec, (long)NY * H, tw);
  hipLaunchKernelGGL((k_rows_inv<NY, NX, RPB, false, float2>), dim3(NY / RPB, n), dim3(kThreads), 0,
                     s, T, (FrameState*)nullptr, img, scale, tw, (PeakCand*)nullptr, 0);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_xcorr(int ny, int nx, const GroupParams& g, hipStream_t s, const Marker& mark) {
  if (xcorr_fused(ny, nx, g.pairs_ok != 0, g.count, g.fused_min)) {
    mark(CCPT_STAGE_XCORR, 1);
    const int rc = launch_xcorr256(g, s);
    mark(CCPT_STAGE_XCORR, 0);
    return rc;
  }
  if (ny == nx) {
    switch (ny) {
#define CASE(n) \
  case n:       \
    return xcorr_n<n, n>(g, s, mark);
      CCPT_FOR_SIZES(CASE)
#undef CASE
    }
    return -2;
  }
#define CASE(a, b) \
  if (ny == a && nx == b) return xcorr_n<a, b>(g, s, mark);
  CCPT_FOR_RECT(CASE)
#undef CASE
  return -2;
}

int launch_init_state(FrameState* st, int count, hipStream_t s) {
  if (count <= 0) return 0;
  hipLaunchKernelGGL(k_init_state, dim3((count + 255) / 256), dim3(256), 0, s, st, count);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_xcorr64(int N, const GroupParams& g, hipStream_t s, const Marker& mark) {
  switch (N) {
#define CASE(n) \
  case n:       \
    return xcorr64_n<n>(g, s, mark);
    CCPT_FOR_SIZES(CASE)
#undef CASE
  }
  return -2;
}

int launch_spectrum(int ny, int nx, const void* data, int dtype, int pitch, long img_stride,
                    int trans, int n, int weight, float eps, int conj_out, float2* T, float2* spec,
                    const float2* tw, hipStream_t s) {
  if (ny == nx) {
    switch (ny) {
#define CASE(nn)                                                                                 \
  case nn:                                                                                       \
    return spectrum_n<nn, nn, float2>(data, dtype, pitch, img_stride, 0, n, weight, (double)eps, \
                                      conj_out, T, spec, tw, s);
      CCPT_FOR_SIZES(CASE)
#undef CASE
    }
    return -2;
  }
#define CASE(a, b)                                                                            \
  if (ny == a && nx == b)                                                                     \
    return spectrum_n<a, b, float2>(data, dtype, pitch, img_stride, trans, n, weight,         \
                                    (double)eps, conj_out, T, spec, tw, s);
  CCPT_FOR_RECT(CASE)
#undef CASE
  return -2;
}

int launch_spectrum64(int N, const void* data, int dtype, int pitch, long img_stride, int n,
                      int weight, double eps, int conj_out, double2* T, double2* spec,
                      const double2* tw, hipStream_t s) {
  switch (N) {
#define CASE(nn)                                                                                \
  case nn:                                                                                      \
    return spectrum_n<nn, nn, double2>(data, dtype, pitch, img_stride, 0, n, weight, eps,       \
                                       conj_out, T, spec, tw, s);
    CCPT_FOR_SIZES(CASE)
#undef CASE
  }
  return -2;
}

int launch_frame_spectra(int ny, int nx, int trans, const FrameDesc* desc, int first, int count,
                         int mode, float eps, float2* T, float2* spec, const float2* tw,
                         hipStream_t s) {
  if (ny == nx) {
    switch (ny) {
#define CASE(nn) \
  case nn:       \
    return frame_spectra_n<nn, nn>(desc, first, count, mode, eps, 0, T, spec, tw, s);
      CCPT_FOR_SIZES(CASE)
#undef CASE
    }
    return -2;
  }
#define CASE(a, b) \
  if (ny == a && nx == b) return frame_spectra_n<a, b>(desc, first, count, mode, eps, trans, T, spec, tw, s);
  CCPT_FOR_RECT(CASE)
#undef CASE
  return -2;
}

int launch_inverse(int ny, int nx, const float2* spec, int n, float scale, float2* T, float* img,
                   const float2* tw, hipStream_t s) {
  if (ny == nx) {
    switch (ny) {
#define CASE(nn) \
  case nn:       \
    return inverse_n<nn, nn>(spec, n, scale, T, img, tw, s);
      CCPT_FOR_SIZES(CASE)
#undef CASE
    }
    return -2;
  }
#define CASE(a, b) \
  if (ny == a && nx == b) return inverse_n<a, b>(spec, n, scale, T, img, tw, s);
  CCPT_FOR_RECT(CASE)
#undef CASE
  return -2;
}

__global__ void k_zero(unsigned* p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}

int launch_zero(void* p, size_t bytes, hipStream_t s) {
  size_t n = bytes / 4;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, (unsigned*)p, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ccpt
