// Batched complex FFTs of length L = 2^a 3^b held in LDS, in Stockham
// (self-sorting) form: each stage reads its inputs with unit stride across
// butterflies and writes them back already in order, so no bit reversal
// pass is needed.  Radix 3 for the factors of 3, then radix 8, closing with
// radix 4 or 2.  Twiddles come from an LDS table of exp(-2 pi i m / N) for
// the transform size N of the kernel (L divides N).
#pragma once

#include <hip/hip_runtime.h>

namespace ccpt {

// Complex arithmetic on float2 (FP32 path) and double2 (FP64 path).
template <typename C>
struct cplx;
template <>
struct cplx<float2> {
  using real = float;
  static constexpr float sin60 = 0.86602540378443864676f;
  static constexpr float sqrt_half = 0.70710678118654752440f;
};
template <>
struct cplx<double2> {
  using real = double;
  static constexpr double sin60 = 0.86602540378443864676;
  static constexpr double sqrt_half = 0.70710678118654752440;
};
template <typename C>
using real_t = typename cplx<C>::real;

template <typename C>
__device__ __forceinline__ C mkc(real_t<C> x, real_t<C> y) {
  if constexpr (sizeof(C) == sizeof(float2))
    return make_float2(x, y);
  else
    return make_double2(x, y);
}
template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { return mkc<C>(a.x + b.x, a.y + b.y); }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { return mkc<C>(a.x - b.x, a.y - b.y); }
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  return mkc<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C>
__device__ __forceinline__ C cconj(C a) { return mkc<C>(a.x, -a.y); }
template <typename C>
__device__ __forceinline__ C cscale(C a, real_t<C> s) { return mkc<C>(a.x * s, a.y * s); }
// multiply by i * SIGN
template <int SIGN, typename C>
__device__ __forceinline__ C mul_i(C a) {
  return SIGN > 0 ? mkc<C>(-a.y, a.x) : mkc<C>(a.y, -a.x);
}

// bf16 (round to nearest even) of a float, as the high 16 bits of its pattern
__device__ __forceinline__ unsigned bf16_bits(float f) {
  unsigned b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return b >> 16;
}
__device__ __forceinline__ float bf16_float(unsigned h) { return __uint_as_float(h << 16); }

typedef __bf16 bf16x2_v __attribute__((ext_vector_type(2)));
typedef float f32x2_v __attribute__((ext_vector_type(2)));

// bf16 (round to nearest even) of two floats, packed a | b << 16: the same
// bits as bf16_bits for finite values, in one conversion instruction
__device__ __forceinline__ unsigned bf16_pack(float a, float b) {
  const f32x2_v v = {a, b};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2_v));
}
// the low and high halves of a packed pair as floats
__device__ __forceinline__ float bf16_lo_float(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi_float(unsigned w) { return __uint_as_float(w & 0xFFFF0000u); }

// bf16 hi + lo split of two floats (x ~ hi + lo to about 16 significant
// bits), each packed as a | b << 16.
__device__ __forceinline__ void split2(float a, float b, unsigned& hi, unsigned& lo) {
  hi = bf16_pack(a, b);
  lo = bf16_pack(a - bf16_lo_float(hi), b - bf16_hi_float(hi));
}

// Splits a complex value into bf16 hi + lo words (re in the low half, im in
// the high half of each word): v ~ hi + lo to about 16 significant bits.
__device__ __forceinline__ void split_pair(float2 v, unsigned& hi, unsigned& lo) {
  split2(v.x, v.y, hi, lo);
}

// fp16 hi + lo split of two floats (x ~ hi + lo to about 22 significant bits
// while |x| stays inside the fp16 range), each packed as a | b << 16.
__device__ __forceinline__ unsigned f16_pack(float a, float b) {
  const _Float16 ha = (_Float16)a, hb = (_Float16)b;
  return (unsigned)__builtin_bit_cast(unsigned short, ha) |
         ((unsigned)__builtin_bit_cast(unsigned short, hb) << 16);
}
__device__ __forceinline__ float f16_lo_float(unsigned w) {
  return (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xFFFFu));
}
__device__ __forceinline__ float f16_hi_float(unsigned w) {
  return (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
}
__device__ __forceinline__ void split2_f16(float a, float b, unsigned& hi, unsigned& lo) {
  hi = f16_pack(a, b);
  lo = f16_pack(a - f16_lo_float(hi), b - f16_hi_float(hi));
}

// LDS layout of an FFT sequence: element i sits at lds_idx(i), with one
// unused slot after every 2^kLdsPadShift elements when the shift is nonzero,
// so the strided writes of the early Stockham stages spread over the LDS
// banks.  lds_len(n) slots hold a sequence of n elements.
constexpr int kLdsPadShift = 4;
__host__ __device__ constexpr int lds_idx(int i) {
  return kLdsPadShift ? i + (i >> kLdsPadShift) : i;
}
__host__ __device__ constexpr int lds_len(int n) {
  return kLdsPadShift ? n + (n >> kLdsPadShift) : n;
}

constexpr int fft_radix(int L, int stage) {
  int i = 0;
  while (L % 3 == 0) {
    if (i == stage) return 3;
    L /= 3;
    ++i;
  }
  while (L % 8 == 0) {
    if (i == stage) return 8;
    L /= 8;
    ++i;
  }
  if (L % 4 == 0) {
    if (i == stage) return 4;
    L /= 4;
    ++i;
  }
  if (L % 2 == 0) {
    if (i == stage) return 2;
    L /= 2;
    ++i;
  }
  return 1;
}

constexpr int fft_stages(int L) {
  int s = 0;
  while (fft_radix(L, s) > 1) ++s;
  return s;
}

// In-register DFT of size R with exponent sign SIGN (-1 forward, +1 inverse).
template <int R, int SIGN, typename C>
__device__ __forceinline__ void dft(C* v) {
  using Rt = real_t<C>;
  if constexpr (R == 2) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 3) {
    const Rt c = Rt(-0.5);
    const Rt s = SIGN * cplx<C>::sin60;
    C a = v[0], b = v[1], d = v[2];
    C t = cadd(b, d);
    C u = csub(b, d);
    v[0] = cadd(a, t);
    C m = mkc<C>(a.x + c * t.x, a.y + c * t.y);
    // i * s * u
    C r = mkc<C>(-s * u.y, s * u.x);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
  } else if constexpr (R == 4) {
    C a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
    C s02 = cadd(a0, a2), d02 = csub(a0, a2);
    C s13 = cadd(a1, a3), d13 = mul_i<SIGN>(csub(a1, a3));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
  } else if constexpr (R == 8) {
    C e[4] = {v[0], v[2], v[4], v[6]};
    C o[4] = {v[1], v[3], v[5], v[7]};
    dft<4, SIGN>(e);
    dft<4, SIGN>(o);
    const Rt h = cplx<C>::sqrt_half;
    // w8^k = exp(SIGN * 2 pi i k / 8)
    C o1 = mkc<C>(h * (o[1].x - SIGN * o[1].y), h * (o[1].y + SIGN * o[1].x));
    C o2 = mul_i<SIGN>(o[2]);
    C o3 = mkc<C>(h * (-o[3].x - SIGN * o[3].y), h * (-o[3].y + SIGN * o[3].x));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
}

// One Stockham stage of radix R on `nseq` sequences of length L (sequence
// q at src/dst + q*stride).  NS = product of the radices already applied.
// tw: exp(-2 pi i m / NTW), m < NTW, with L | NTW.
template <int L, int R, int SIGN, int NTW, typename C>
__device__ __forceinline__ void fft_stage(const C* __restrict__ src, C* __restrict__ dst,
                                          int nseq, int stride, int NS, const C* tw,
                                          int tid, int nthr) {
  constexpr int B = L / R;
  const int total = nseq * B;
  for (int b = tid; b < total; b += nthr) {
    const int q = b / B;
    const int j = b - q * B;
    const C* in = src + q * stride;
    C* out = dst + q * stride;
    C v[R];
#pragma unroll
    for (int t = 0; t < R; ++t) v[t] = in[lds_idx(j + t * B)];
    const int k = j % NS;
    if (NS > 1) {
      // twiddle exp(SIGN * 2 pi i t k / (NS R)) = tw[t k NTW / (NS R)] (conj for SIGN > 0)
      const int step = NTW / (NS * R);
#pragma unroll
      for (int t = 1; t < R; ++t) {
        C w = tw[t * k * step];
        if (SIGN > 0) w.y = -w.y;
        v[t] = cmul(v[t], w);
      }
    }
    dft<R, SIGN>(v);
    const int base = (j / NS) * NS * R + k;
#pragma unroll
    for (int t = 0; t < R; ++t) out[lds_idx(base + t * NS)] = v[t];
  }
}

template <int L, int SIGN, int NTW, int ST, typename C>
__device__ __forceinline__ C* fft_run(C* a, C* b, int nseq, int stride, int NS, const C* tw,
                                      int tid, int nthr) {
  if constexpr (ST == fft_stages(L)) {
    return a;
  } else {
    constexpr int R = fft_radix(L, ST);
    fft_stage<L, R, SIGN, NTW>(a, b, nseq, stride, NS, tw, tid, nthr);
    __syncthreads();
    return fft_run<L, SIGN, NTW, ST + 1>(b, a, nseq, stride, NS * R, tw, tid, nthr);
  }
}

// Transforms nseq sequences in `a` (b is scratch of the same size); returns
// the buffer holding the result.  Callers must __syncthreads() before.
template <int L, int SIGN, int NTW, typename C>
__device__ __forceinline__ C* fft_lds(C* a, C* b, int nseq, int stride, const C* tw) {
  return fft_run<L, SIGN, NTW, 0>(a, b, nseq, stride, 1, tw, threadIdx.x, blockDim.x);
}

}  // namespace ccpt
