// Correlation stage for 256 x 256 frames in one kernel (Sec. II Eq. 4 / Eq. 7,
// Sec. III first paragraph): prologue, forward 2-D r2c FFT, product with the
// resident conj F[B], inverse 2-D c2r FFT and the integer-lag maximum, with
// the whole half spectrum of a frame held in registers.
//
// One 512-thread block per frame.  The 256 x 129 half spectrum (the DC and
// Nyquist columns packed as one complex column) is 32768 complex values: 64
// per thread, 128 VGPRs.  Each 1-D transform runs as two in-register stages
// (rows: 128 = 16 x 8 after packing pixel pairs as complex values; columns:
// 256 = 16 x 16), and between stages the values move through LDS in two
// rounds of 128 KB (a frame's half spectrum is 256 KB, LDS 160 KB).  Nothing
// but the frame, the reference spectrum (shared, L2-resident) and the
// outputs X (and its split copy) touches memory.
//
// Index conventions (t = thread, all per row y or column kx of the frame):
//   z[y][n] = A[y][2n] + i A[y][2n+1], n < 128; Z = FFT128(z) along n.
//   rows:   n = 8 n1 + n2, k = k1 + 16 k2 (k1 < 16, k2 < 8)
//   unpack: F[k] = E + W256^k O, E = (Z[k] + conj Z[128-k]) / 2,
//           O = (Z[k] - conj Z[128-k]) / 2i; column 0 holds F[0] + i F[128]
//   cols:   y = 16 a + b, ky = c + 16 d (all < 16)
//   inverse columns: ky = c + 16 d -> y = a' + 16 b'
//   c2r pack: Zr[k] = E + i O, E = (G[k] + conj G[128-k]) / 2,
//           O = (G[k] - conj G[128-k]) W256^-k / 2; rows inverse:
//           k = k1 + 16 k2 -> n = a'' + 8 b''
// A thread's two k1 (or c) values are the pair {g, 16 - g} ({0, 8} for
// g = 0), so the partner bin 128 - k (or -ky) of every value it holds is its
// own.  The correlation comes out as half the unnormalised 2-D inverse (the
// scale does not move the maximum).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.h"
#include "fft.h"

namespace ccpt {

namespace {

constexpr int kT = 512;  // threads per block (8 waves)
constexpr int N = 256, H = N / 2 + 1;

// LDS strides (complex values), padded against bank conflicts
// The 16-byte chunks a thread reads with one b128 load are XOR-swizzled by the
// reader's own index, so the 16 lanes served together hit distinct banks.
constexpr int RS2 = 128 + 4;  // first row exchange: [y (128)][k1 (16)][n2 (8)]
constexpr int RS7 = 128 + 8;  // last row exchange: [y (128)][a'' (8)][k1 (16)]
constexpr int CS = 256 + 4;   // transposes: [kx (64)][y (256)]
constexpr int QS = 256 + 2;   // column exchanges: [kx (64)][16][16]
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kLds = cmax(cmax(128 * RS2, 128 * RS7), cmax(64 * CS, 64 * QS));
// element positions within a row or column block
__device__ __forceinline__ int e2pos(int k1, int n2) {  // chunks (n2 pairs) swizzled by bit 2 of k1
  return k1 * 8 + 2 * ((n2 >> 1) ^ ((k1 >> 2) & 1)) + (n2 & 1);
}
__device__ __forceinline__ int e5pos(int a, int c) {  // chunks (c pairs) swizzled by a / 2
  return a * 16 + 2 * ((c >> 1) ^ (a >> 1)) + (c & 1);
}
__device__ __forceinline__ int e7pos(int a, int k1) {  // chunks (k1 pairs) swizzled by a / 2
  return a * 16 + 2 * ((k1 >> 1) ^ (a >> 1)) + (k1 & 1);
}

__device__ __forceinline__ int kap(int g, int s) { return s == 0 ? g : (g == 0 ? 8 : 16 - g); }

// physical register of element m (< 32) of exchange half `half`: the halves
// interleave in groups of four, so that a round's reads land in the registers
// its writes have freed
__host__ __device__ constexpr int pslot(int m, int half) {
  return 8 * (m >> 2) + (m & 3) + 4 * half;
}

// W16^m with exponent sign SIGN, m = n2 k1 in {1, 2, 3, 6, 9}
template <int SIGN>
__device__ __forceinline__ float2 w16mul(float2 a, int m) {
  constexpr float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;
  constexpr float h = 0.70710678118654752440f;
  float c, s;
  switch (m) {
    case 1: c = c1; s = s1; break;
    case 2: c = h; s = h; break;
    case 3: c = s1; s = c1; break;
    case 6: c = -h; s = h; break;
    default: c = -c1; s = -s1; break;  // 9
  }
  s = SIGN * s;  // W = (cos, SIGN sin)
  return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
}

// In-register DFT of 16 values with exponent sign SIGN (16 = 4 x 4).
template <int SIGN>
__device__ __forceinline__ void dft16(float2* v) {
  float2 t[16];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    float2 q[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
    dft<4, SIGN>(q);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) t[n2 * 4 + k1] = q[k1];
  }
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) {
      const int m = n2 * k1;
      t[n2 * 4 + k1] = m == 4 ? mul_i<SIGN>(t[n2 * 4 + k1]) : w16mul<SIGN>(t[n2 * 4 + k1], m);
    }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 q[4] = {t[k1], t[4 + k1], t[8 + k1], t[12 + k1]};
    dft<4, SIGN>(q);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = q[k2];
  }
}

__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

// Pointers read from a descriptor are generic; these say they are global, so
// their loads are global (vector memory only) rather than flat loads, which
// the LDS waits would also have to wait for.
typedef const unsigned long long __attribute__((address_space(1)))* gcf2;  // float2 pairs
typedef const float __attribute__((address_space(1)))* gcf;
typedef const unsigned short __attribute__((address_space(1)))* gcu16;

__device__ __forceinline__ float2 ld2(gcf2 p) {
  const unsigned long long u = *p;
  return make_float2(__uint_as_float((unsigned)u), __uint_as_float((unsigned)(u >> 32)));
}

// F[k] = E + W O from Z[k] (a) and Z[128-k] (b), W = W256^k:
// E = (a + conj b)/2, O = (a - conj b)/2i
__device__ __forceinline__ float2 r2c_bin(float2 a, float2 b, float2 w) {
  const float ex = 0.5f * (a.x + b.x), ey = 0.5f * (a.y - b.y);
  const float ox = 0.5f * (a.y + b.y), oy = -0.5f * (a.x - b.x);
  return make_float2(ex + w.x * ox - w.y * oy, ey + w.x * oy + w.y * ox);
}

// Zr[k] = E + i O from G[k] (a) and G[128-k] (b), W = W256^-k:
// E = (a + conj b)/2, O = (a - conj b) W / 2
__device__ __forceinline__ float2 c2r_bin(float2 a, float2 b, float2 w) {
  const float ex = 0.5f * (a.x + b.x), ey = 0.5f * (a.y - b.y);
  const float dx = 0.5f * (a.x - b.x), dy = 0.5f * (a.y + b.y);
  const float ox = dx * w.x - dy * w.y, oy = dx * w.y + dy * w.x;
  return make_float2(ex - oy, ey + ox);
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

}  // namespace

template <bool SPLIT, bool SN>
__global__ void __launch_bounds__(kT) k_xcorr256(GroupParams g) {
  __shared__ __align__(16) float2 lds[kLds];
  __shared__ float2 tw[N];
  __shared__ float2 stage[2 * N];  // products of the real columns 0 and N/2
  __shared__ float redf[2][kT / 64];
  __shared__ unsigned redu[4][kT / 64];
  __shared__ unsigned xmax_s;  // split precision: largest |Re|, |Im| of X without DC (float bits)
  const int t = threadIdx.x;
  const int f = blockIdx.x;
  if (t == 0) xmax_s = 0u;
  const FrameDesc desc = g.desc[g.first + f];
  for (int i = t; i < N; i += kT) tw[i] = g.tw[i];

  float2 r[64];
  // ---------------------------------------------------------------- load
  // thread (n2 = t % 8, rq = t / 8): rows rq + 64 j, pairs 8 n1 + n2
  unsigned kmin = 0xFFFFFFFFu, kmax = 0u, bad;
  {
    const int n2 = t & 7, rq = t >> 3;
    const float eps = g.eps;
    auto take = [&](float2 a, int e) {
      if (SN) {
        a.x = (a.x + eps) * (a.x + eps);
        a.y = (a.y + eps) * (a.y + eps);
      }
      const unsigned k0 = f2key(a.x), k1 = f2key(a.y);
      kmin = min(kmin, min(k0, k1));
      kmax = max(kmax, max(k0, k1));
      r[e] = a;
    };
    // (the launcher takes this kernel only for uint16 or float32 frames with
    // an even pitch and pairs aligned to their size: one load per pair)
    const size_t p = (size_t)desc.pitch;
    if (desc.dtype == CCPT_U16) {
      const gcu16 b = (gcu16)desc.data + (size_t)rq * p + 2 * n2;
      unsigned raw[64];  // all loads in flight before the first use
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1)
          raw[j * 16 + n1] = *(const unsigned __attribute__((address_space(1)))*)(b + 64 * j * p + 16 * n1);
#pragma unroll
      for (int e = 0; e < 64; ++e) take(make_float2((float)(raw[e] & 0xFFFFu), (float)(raw[e] >> 16)), e);
    } else {
      const gcf b = (gcf)desc.data + (size_t)rq * p + 2 * n2;
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1) r[j * 16 + n1] = ld2((gcf2)(b + 64 * j * p + 16 * n1));
#pragma unroll
      for (int e = 0; e < 64; ++e) take(r[e], e);
    }
  }
  __syncthreads();  // twiddle table
  // ---------------------------------------------------------------- R1
  {
    const int n2 = t & 7;
    float2 w[16];
#pragma unroll
    for (int k1 = 1; k1 < 16; ++k1) w[k1] = tw[(2 * n2 * k1) & 255];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      dft16<-1>(r + 16 * j);
#pragma unroll
      for (int k1 = 1; k1 < 16; ++k1) r[16 * j + k1] = cmul(r[16 * j + k1], w[k1]);
    }
  }
  // ---------------------------------------------------------------- E2: rows
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    {
      const int n2 = t & 7, rq = t >> 3;
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int j = 2 * h + jj, yl = rq + 64 * jj;
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) lds[yl * RS2 + e2pos(k1, n2)] = r[j * 16 + k1];
      }
    }
    __syncthreads();
    {
      const int gg = t & 7, rq = t >> 3;
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int j = 2 * h + jj, yl = rq + 64 * jj;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int k1 = kap(gg, s), sw = (k1 >> 2) & 1;
          const float4* src = (const float4*)&lds[yl * RS2 + k1 * 8];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float4 v = src[q ^ sw];
            r[j * 16 + s * 8 + 2 * q] = make_float2(v.x, v.y);
            r[j * 16 + s * 8 + 2 * q + 1] = make_float2(v.z, v.w);
          }
        }
      }
    }
    __syncthreads();
  }
  // ---------------------------------------------------------------- R2 + unpack
  {
    const int gg = t & 7;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int s = 0; s < 2; ++s) dft<8, -1>(r + j * 16 + s * 8);
    // twiddles W256^k of the thread's 16 bins k = kap(gg, s) + 16 k2
    float2 w[16];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int k2 = 0; k2 < 8; ++k2) w[s * 8 + k2] = tw[kap(gg, s) + 16 * k2];
    const bool g0 = gg == 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float2 z[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) z[e] = r[j * 16 + e];
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) {
          // partner bin 128 - k: slot (1 - s, 7 - k2) for g >= 1; for g = 0,
          // (0, (8 - k2) % 8) or (1, 7 - k2)
          const float2 pa = z[(1 - s) * 8 + 7 - k2];
          const float2 pb = s == 0 ? z[(8 - k2) & 7] : z[8 + 7 - k2];
          const float2 p = g0 ? pb : pa;
          float2 v = r2c_bin(z[s * 8 + k2], p, w[s * 8 + k2]);
          if (s == 0 && k2 == 0) {
            // g = 0: bin 0 carries F[0] + i F[128]
            const float2 z0 = z[0];
            const float2 pk = make_float2(z0.x + z0.y, z0.x - z0.y);
            v = g0 ? pk : v;
          }
          r[j * 16 + s * 8 + k2] = v;
        }
    }
  }
  // ---------------------------------------------------------------- E3: rows -> columns
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    {
      const int gg = t & 7, rq = t >> 3;
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int kxl = kap(gg, s) + 16 * q;  // kx - 64 h, k2 = 4 h + q
            lds[kxl * CS + rq + 64 * j] = r[j * 16 + s * 8 + 4 * h + q];
          }
    }
    __syncthreads();
    {
      const int b = t & 15, cq = t >> 4;
#pragma unroll
      for (int ii = 0; ii < 2; ++ii) {
        const int cl = cq + 32 * ii;
#pragma unroll
        for (int a = 0; a < 16; ++a) r[pslot(ii * 16 + a, h)] = lds[cl * CS + 16 * a + b];
      }
    }
    __syncthreads();
  }
  // ---------------------------------------------------------------- C1
  {
    const int b = t & 15;
    float2 w[16];
#pragma unroll
    for (int c = 1; c < 16; ++c) w[c] = tw[(b * c) & 255];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float2 v[16];
#pragma unroll
      for (int a = 0; a < 16; ++a) v[a] = r[pslot((i & 1) * 16 + a, i >> 1)];
      dft16<-1>(v);
#pragma unroll
      for (int c = 1; c < 16; ++c) v[c] = cmul(v[c], w[c]);
#pragma unroll
      for (int c = 0; c < 16; ++c) r[pslot((i & 1) * 16 + c, i >> 1)] = v[c];
    }
  }
  // ---------------------------------------------------------------- E4: columns
  // C2 thread: hp = t / 64 (c pair, uniform per wave), cp = t % 64 (columns cp, cp + 64)
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    {
      const int b = t & 15, cq = t >> 4;
#pragma unroll
      for (int ii = 0; ii < 2; ++ii) {
        const int cl = cq + 32 * ii;
#pragma unroll
        for (int c = 0; c < 16; ++c) lds[cl * QS + c * 16 + b] = r[pslot(ii * 16 + c, h)];
      }
    }
    __syncthreads();
    {
      const int hp = t >> 6, cp = t & 63;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const float4* src = (const float4*)&lds[cp * QS + kap(hp, s) * 16];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float4 v = src[q];
          r[pslot(s * 16 + 2 * q, h)] = make_float2(v.x, v.y);
          r[pslot(s * 16 + 2 * q + 1, h)] = make_float2(v.z, v.w);
        }
      }
    }
    __syncthreads();
  }
  // ---------------------------------------------------------------- C2, product, X
  // C2 thread: hp = t / 64 (the pair of c values, uniform per wave), cp = t % 64
  // (columns cp and cp + 64).  The reference spectrum is read in batches whose
  // loads are issued before the previous batch's products (no stores come
  // between them, so a batch waits only for its own loads); the products go
  // out after all of a half's loads.  Column 0 (packed) falls to lane 0 of
  // every wave: its two real columns' products go to LDS and out by all
  // threads.
  {
    const int hp = t >> 6, cp = t & 63;
    const gcf2 R = (gcf2)desc.rspec;
    float2* Xf = g.X + (size_t)f * N * H;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        float2 v[16];
#pragma unroll
        for (int d = 0; d < 16; ++d) v[d] = r[pslot(s * 16 + d, i)];
        dft16<-1>(v);
#pragma unroll
        for (int d = 0; d < 16; ++d) r[pslot(s * 16 + d, i)] = v[d];
      }
      const int col = cp + 64 * i;
      const bool packed = i == 0 && cp == 0;
      // split precision: the largest |Re|, |Im| of the X values this thread
      // stores, merged into xmax_s right after the stores (non-negative floats
      // order as their bits), so no register carries it further
      float xmx = 0.f;
      auto merge_xmax = [&]() {
        if constexpr (SPLIT) {
          const unsigned xw = wave_max(__float_as_uint(xmx));
          if ((t & 63) == 0) atomicMax(&xmax_s, xw);
        }
      };
      if (packed) {
        // P = F0 + i F128 with F0, F128 the spectra of the real columns 0 and
        // N/2: F0[ky] = (P[ky] + conj P[-ky]) / 2, F128 = (P[ky] - conj P[-ky]) / 2i;
        // a pair (ky, -ky) gives conjugate values of both.  Pairs by element:
        // hp > 0: (d, 31 - d); hp = 0: (0, 0), (8, 8), (d, 16 - d), (16 + d, 31 - d)
        auto run = [&](auto hz) {
          constexpr bool H0 = decltype(hz)::value;  // hp == 0 (compile-time pair list)
          constexpr int np = H0 ? 17 : 16;
          auto e1_of = [](int q) {
            return !H0 ? q : (q == 0 ? 0 : q == 1 ? 8 : q <= 8 ? q - 1 : 16 + (q - 9));
          };
          auto e2_of = [](int q) {
            return !H0 ? 31 - q : (q == 0 ? 0 : q == 1 ? 8 : q <= 8 ? 16 - (q - 1) : 31 - (q - 9));
          };
          auto ky_of = [&](int e) { return kap(hp, e >> 4) + 16 * (e & 15); };
          // batches of 4 pairs: R*[ky1][0], R*[ky1][N/2], R*[ky2][0], R*[ky2][N/2]
          float2 rb[2][4][4];
          auto load = [&](int b, float2 (*dst)[4]) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int q = 4 * b + k;
              if (q < np) {
                const int k1 = ky_of(e1_of(q)), k2 = ky_of(e2_of(q));
                dst[k][0] = ld2(R + (size_t)k1 * H);
                dst[k][1] = ld2(R + (size_t)k1 * H + N / 2);
                dst[k][2] = ld2(R + (size_t)k2 * H);
                dst[k][3] = ld2(R + (size_t)k2 * H + N / 2);
              }
            }
          };
          load(0, rb[0]);
#pragma unroll
          for (int b = 0; b < 5; ++b) {
            if (b < 4) load(b + 1, rb[(b + 1) & 1]);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int q = 4 * b + k;
              if (q < np) {
                const int e1 = e1_of(q), e2 = e2_of(q);
                const float2 a = r[pslot(e1, 0)], bb = r[pslot(e2, 0)];
                const float2 F0 = make_float2(0.5f * (a.x + bb.x), 0.5f * (a.y - bb.y));
                const float2 F1 = make_float2(0.5f * (a.y + bb.y), -0.5f * (a.x - bb.x));
                const int k1 = ky_of(e1), k2 = ky_of(e2);
                const float2 X0 = cmul(F0, rb[b & 1][k][0]), X1 = cmul(F1, rb[b & 1][k][1]);
                stage[k1] = X0;
                stage[N + k1] = X1;
                r[pslot(e1, 0)] = make_float2(X0.x - X1.y, X0.y + X1.x);  // X0 + i X128
                if (e2 != e1) {
                  const float2 Y0 = cmul(conjf2(F0), rb[b & 1][k][2]);
                  const float2 Y1 = cmul(conjf2(F1), rb[b & 1][k][3]);
                  stage[k2] = Y0;
                  stage[N + k2] = Y1;
                  r[pslot(e2, 0)] = make_float2(Y0.x - Y1.y, Y0.y + Y1.x);
                }
              }
            }
          }
        };
        if (hp == 0)
          run(std::integral_constant<bool, true>());
        else
          run(std::integral_constant<bool, false>());
      } else {
        float2 rb[2][8];
        auto load = [&](int b, float2* dst) {
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int e = 8 * b + k, ky = kap(hp, e >> 4) + 16 * (e & 15);
            dst[k] = ld2(R + (size_t)ky * H + col);
          }
        };
        load(0, rb[0]);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          if (b < 3) load(b + 1, rb[(b + 1) & 1]);
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int e = 8 * b + k;
            r[pslot(e, i)] = cmul(r[pslot(e, i)], rb[b & 1][k]);
          }
        }
#pragma unroll
        for (int e = 0; e < 32; ++e) {
          const int ky = kap(hp, e >> 4) + 16 * (e & 15);
          const float2 x = r[pslot(e, i)];
          Xf[(size_t)ky * H + col] = x;
          if constexpr (SPLIT) xmx = fmaxf(xmx, fmaxf(fabsf(x.x), fabsf(x.y)));
        }
      }
      merge_xmax();
      if (i == 0) {
        // the two real columns' products, staged by the packed lanes; in
        // split precision also Z = X[., 0] + i X[., N/2] without the DC term,
        // the packed column the matrix DFT takes as its kx = 0 operand
        __syncthreads();
        for (int e = t; e < 2 * N; e += kT) {
          const float2 x = stage[e];
          Xf[(size_t)(e & (N - 1)) * H + (e >> 8) * (N / 2)] = x;
          if constexpr (SPLIT)
            if (e) xmx = fmaxf(xmx, fmaxf(fabsf(x.x), fabsf(x.y)));  // (e = 0: the DC term)
        }
        merge_xmax();
        if constexpr (SPLIT) {
          for (int ky = t; ky < N; ky += kT) {
            const float2 x0 = stage[ky], x1 = stage[N + ky];
            g.Zc[(size_t)f * N + ky] = make_float2((ky ? x0.x : 0.f) - x1.y, x0.y + x1.x);
          }
        }
      }
      // I1: inverse DFT over d, twiddle W256^{-c a'}
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int c = kap(hp, s);
        float2 v[16];
#pragma unroll
        for (int d = 0; d < 16; ++d) v[d] = r[pslot(s * 16 + d, i)];
        dft16<+1>(v);
#pragma unroll
        for (int a = 1; a < 16; ++a) v[a] = cmul(v[a], conjf2(tw[(c * a) & 255]));
#pragma unroll
        for (int a = 0; a < 16; ++a) r[pslot(s * 16 + a, i)] = v[a];
      }
    }
  }
  // ---------------------------------------------------------------- E5: columns
  // I2 thread: a' = t % 16, cq = t / 16 (columns cq + 32 i)
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    __syncthreads();
    {
      const int hp = t >> 6, cp = t & 63;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int c = kap(hp, s);
#pragma unroll
        for (int a = 0; a < 16; ++a) lds[cp * QS + e5pos(a, c)] = r[pslot(s * 16 + a, h)];
      }
    }
    __syncthreads();
    {
      const int ap = t & 15, cq = t >> 4;
#pragma unroll
      for (int ii = 0; ii < 2; ++ii) {
        const int cl = cq + 32 * ii;
        const float4* src = (const float4*)&lds[cl * QS + ap * 16];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float4 v = src[q ^ (ap >> 1)];
          r[pslot(ii * 16 + 2 * q, h)] = make_float2(v.x, v.y);
          r[pslot(ii * 16 + 2 * q + 1, h)] = make_float2(v.z, v.w);
        }
      }
    }
  }
  // ---------------------------------------------------------------- I2
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float2 v[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) v[c] = r[pslot((i & 1) * 16 + c, i >> 1)];
    dft16<+1>(v);
#pragma unroll
    for (int c = 0; c < 16; ++c) r[pslot((i & 1) * 16 + c, i >> 1)] = v[c];
  }
  // ---------------------------------------------------------------- E6: columns -> rows
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    __syncthreads();
    {
      const int ap = t & 15, cq = t >> 4;
#pragma unroll
      for (int ii = 0; ii < 2; ++ii) {
        const int cl = cq + 32 * ii;
#pragma unroll
        for (int bp = 0; bp < 16; ++bp) lds[cl * CS + ap + 16 * bp] = r[pslot(ii * 16 + bp, h)];
      }
    }
    __syncthreads();
    {
      const int gg = t & 7, rq = t >> 3;
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int kxl = kap(gg, s) + 16 * q;
            r[j * 16 + s * 8 + 4 * h + q] = lds[kxl * CS + rq + 64 * j];
          }
    }
  }
  // ---------------------------------------------------------------- pack + J1
  {
    const int gg = t & 7;
    float2 w[16];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int k2 = 0; k2 < 8; ++k2) w[s * 8 + k2] = conjf2(tw[kap(gg, s) + 16 * k2]);
    const bool g0 = gg == 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float2 z[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) z[e] = r[j * 16 + e];
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) {
          const float2 pa = z[(1 - s) * 8 + 7 - k2];
          const float2 pb = s == 0 ? z[(8 - k2) & 7] : z[8 + 7 - k2];
          const float2 p = g0 ? pb : pa;
          float2 v = c2r_bin(z[s * 8 + k2], p, w[s * 8 + k2]);
          if (s == 0 && k2 == 0) {
            // g = 0: bin 0 carries g0 + i g128 (both real)
            const float2 z0 = z[0];
            const float2 pk = make_float2(0.5f * (z0.x + z0.y), 0.5f * (z0.x - z0.y));
            v = g0 ? pk : v;
          }
          r[j * 16 + s * 8 + k2] = v;
        }
    }
    float2 wj[2][8];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int a = 1; a < 8; ++a) wj[s][a] = conjf2(tw[(2 * kap(gg, s) * a) & 255]);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        dft<8, +1>(r + j * 16 + s * 8);
#pragma unroll
        for (int a = 1; a < 8; ++a) r[j * 16 + s * 8 + a] = cmul(r[j * 16 + s * 8 + a], wj[s][a]);
      }
  }
  // ---------------------------------------------------------------- E7: rows
  // J2 thread: a'' = t % 8, rq = t / 8
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    __syncthreads();
    {
      const int gg = t & 7, rq = t >> 3;
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int j = 2 * h + jj, yl = rq + 64 * jj;
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int a = 0; a < 8; ++a) lds[yl * RS7 + e7pos(a, kap(gg, s))] = r[j * 16 + s * 8 + a];
      }
    }
    __syncthreads();
    {
      const int a2 = t & 7, rq = t >> 3;
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int j = 2 * h + jj, yl = rq + 64 * jj;
        const float4* src = (const float4*)&lds[yl * RS7 + a2 * 16];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float4 v = src[q ^ (a2 >> 1)];
          r[j * 16 + 2 * q] = make_float2(v.x, v.y);
          r[j * 16 + 2 * q + 1] = make_float2(v.z, v.w);
        }
      }
    }
  }
  // ---------------------------------------------------------------- J2 + maximum
  // the two largest values (equal values count twice) by float max/min, then
  // the lowest row-major index holding the frame's maximum in a second pass
  float t1 = -__builtin_inff(), t2 = -__builtin_inff();
  {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      dft16<+1>(r + 16 * j);
#pragma unroll
      for (int b2 = 0; b2 < 16; ++b2) {
        const float2 v = r[16 * j + b2];
        float lo = fminf(t1, v.x);
        t1 = fmaxf(t1, v.x);
        t2 = fmaxf(t2, lo);
        lo = fminf(t1, v.y);
        t1 = fmaxf(t1, v.y);
        t2 = fmaxf(t2, lo);
      }
    }
  }
  auto merge2 = [](float& a1, float& a2, float b1, float b2) {
    const float lo = fminf(a1, b1);
    a1 = fmaxf(a1, b1);
    a2 = fmaxf(fmaxf(a2, b2), lo);
  };
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) merge2(t1, t2, __shfl_xor(t1, o, 64), __shfl_xor(t2, o, 64));
  // a non-finite value has a key above +inf's (NaN) or below -inf's, or equal
  bad = (kmax >= 0xFF800000u || kmin <= 0x007FFFFFu) ? 1u : 0u;
  kmin = ~wave_max(~kmin);
  kmax = wave_max(kmax);
  bad = wave_max(bad);
  if ((t & 63) == 0) {
    redf[0][t >> 6] = t1;
    redf[1][t >> 6] = t2;
    redu[0][t >> 6] = kmin;
    redu[1][t >> 6] = kmax;
    redu[2][t >> 6] = bad;
  }
  __syncthreads();
  t1 = redf[0][0];
  t2 = redf[1][0];
#pragma unroll
  for (int w = 1; w < kT / 64; ++w) merge2(t1, t2, redf[0][w], redf[1][w]);
  unsigned idx = 0xFFFFFFFFu;
  {
    const int a2 = t & 7, rq = t >> 3;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int b2 = 0; b2 < 16; ++b2) {
        const unsigned flat = (unsigned)((rq + 64 * j) * N + 2 * (a2 + 8 * b2));
        if (r[16 * j + b2].x == t1) idx = min(idx, flat);
        if (r[16 * j + b2].y == t1) idx = min(idx, flat + 1);
      }
  }
  idx = ~wave_max(~idx);
  if ((t & 63) == 0) redu[3][t >> 6] = idx;
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < kT / 64; ++w) {
      idx = min(idx, redu[3][w]);
      kmin = min(kmin, redu[0][w]);
      kmax = max(kmax, redu[1][w]);
      bad |= redu[2][w];
    }
    FrameState& st = g.st[f];
    st.xmax = SPLIT ? xmax_s : 0u;
    st.peak_key = peak_key(t1, idx);
    st.second_key = peak_key(t2, 0u);
    st.amin = kmin;
    st.amax = kmax;
    if (bad) st.flags |= CCPT_ST_NONFINITE;
  }
}

int launch_xcorr256(const GroupParams& g, hipStream_t s) {
  const bool sn = g.mode == CCPT_MODE_CCSN;
  if (g.Zc && sn)
    hipLaunchKernelGGL((k_xcorr256<true, true>), dim3(g.count), dim3(kT), 0, s, g);
  else if (g.Zc)
    hipLaunchKernelGGL((k_xcorr256<true, false>), dim3(g.count), dim3(kT), 0, s, g);
  else if (sn)
    hipLaunchKernelGGL((k_xcorr256<false, true>), dim3(g.count), dim3(kT), 0, s, g);
  else
    hipLaunchKernelGGL((k_xcorr256<false, false>), dim3(g.count), dim3(kT), 0, s, g);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ccpt
