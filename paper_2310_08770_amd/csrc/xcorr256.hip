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

#include "common.h"
#include "fft.h"

namespace ccpt {

namespace {

constexpr int kT = 512;  // threads per block (8 waves)
constexpr int N = 256, H = N / 2 + 1;

// LDS strides (complex values), padded against bank conflicts
constexpr int RS = 128 + 8;   // row exchanges: [y (128)][k1 (16)][n2 (8)]
constexpr int CS = 256 + 4;   // transposes: [kx (64)][y (256)]
constexpr int QS = 256 + 2;   // column exchanges: [kx (64)][16][16]
constexpr int kLds = 128 * RS > 64 * CS ? (128 * RS > 64 * QS ? 128 * RS : 64 * QS)
                                        : (64 * CS > 64 * QS ? 64 * CS : 64 * QS);

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

template <bool SPLIT>
__global__ void __launch_bounds__(kT) k_xcorr256(GroupParams g) {
  __shared__ __align__(16) float2 lds[kLds];
  __shared__ float2 tw[N];
  __shared__ unsigned long long red[2][kT / 64];
  __shared__ unsigned redu[3][kT / 64];
  const int t = threadIdx.x;
  const int f = blockIdx.x;
  const FrameDesc desc = g.desc[g.first + f];
  for (int i = t; i < N; i += kT) tw[i] = g.tw[i];

  float2 r[64];
  // ---------------------------------------------------------------- load
  // thread (n2 = t % 8, rq = t / 8): rows rq + 64 j, pairs 8 n1 + n2
  unsigned kmin = 0xFFFFFFFFu, kmax = 0u, bad;
  {
    const int n2 = t & 7, rq = t >> 3;
    const bool sn = g.mode == CCPT_MODE_CCSN;
    const float eps = g.eps;
    auto take = [&](float2 a, int e) {
      if (sn) {
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
      const unsigned short* b = (const unsigned short*)desc.data + (size_t)rq * p + 2 * n2;
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1) {
          const unsigned w = *(const unsigned*)(b + 64 * j * p + 16 * n1);
          take(make_float2((float)(w & 0xFFFFu), (float)(w >> 16)), j * 16 + n1);
        }
    } else {
      const float* b = (const float*)desc.data + (size_t)rq * p + 2 * n2;
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int n1 = 0; n1 < 16; ++n1) take(*(const float2*)(b + 64 * j * p + 16 * n1), j * 16 + n1);
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
        for (int k1 = 0; k1 < 16; ++k1) lds[yl * RS + k1 * 8 + n2] = r[j * 16 + k1];
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
          const float4* src = (const float4*)&lds[yl * RS + kap(gg, s) * 8];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float4 v = src[q];
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
  {
    const int hp = t >> 6, cp = t & 63;
    const float2* R = (const float2*)desc.rspec;
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
      float2 xb0 = make_float2(0.f, 0.f);
      if (i == 0 && cp == 0) {
        // packed column: P = F0 + i F128 with F0, F128 the spectra of real
        // columns, F0[ky] = (P[ky] + conj P[-ky]) / 2, F128 = (P - conj P[-ky]) / 2i;
        // a pair (ky, -ky) gives conjugate values of both
        auto pair = [&](int e1, int e2) {
          const float2 a = r[pslot(e1, 0)], bb = r[pslot(e2, 0)];
          const float2 F0 = make_float2(0.5f * (a.x + bb.x), 0.5f * (a.y - bb.y));
          const float2 F1 = make_float2(0.5f * (a.y + bb.y), -0.5f * (a.x - bb.x));
          const int ky1 = kap(hp, e1 >> 4) + 16 * (e1 & 15);
          const int ky2 = kap(hp, e2 >> 4) + 16 * (e2 & 15);
          const float2 X0 = cmul(F0, R[(size_t)ky1 * H]);
          const float2 X1 = cmul(F1, R[(size_t)ky1 * H + N / 2]);
          Xf[(size_t)ky1 * H] = X0;
          Xf[(size_t)ky1 * H + N / 2] = X1;
          r[pslot(e1, 0)] = make_float2(X0.x - X1.y, X0.y + X1.x);  // X0 + i X128
          if (ky1 == 0) xb0 = make_float2(-X1.y, X0.y + X1.x);      // the DC term dropped
          if (e2 != e1) {
            const float2 Y0 = cmul(conjf2(F0), R[(size_t)ky2 * H]);
            const float2 Y1 = cmul(conjf2(F1), R[(size_t)ky2 * H + N / 2]);
            Xf[(size_t)ky2 * H] = Y0;
            Xf[(size_t)ky2 * H + N / 2] = Y1;
            r[pslot(e2, 0)] = make_float2(Y0.x - Y1.y, Y0.y + Y1.x);
          }
        };
        if (hp != 0) {
#pragma unroll
          for (int d = 0; d < 16; ++d) pair(d, 16 + 15 - d);
        } else {
          pair(0, 0);
          pair(8, 8);
#pragma unroll
          for (int d = 1; d < 8; ++d) pair(d, 16 - d);
#pragma unroll
          for (int d = 0; d < 8; ++d) pair(16 + d, 16 + 15 - d);
        }
      } else {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int d = 0; d < 16; ++d) {
            const int ky = kap(hp, s) + 16 * d;
            const float2 x = cmul(r[pslot(s * 16 + d, i)], R[(size_t)ky * H + col]);
            Xf[(size_t)ky * H + col] = x;
            r[pslot(s * 16 + d, i)] = x;
          }
      }
      if constexpr (SPLIT) {
        // the split copy for the matrix cores goes out row kx by row kx
        // (ky contiguous) through LDS; row 0 is X[., 0] + i X[., N/2] with
        // the DC term dropped
        uint2* xs = (uint2*)lds;
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int d = 0; d < 16; ++d) {
            const int ky = kap(hp, s) + 16 * d;
            float2 x = r[pslot(s * 16 + d, i)];
            if (i == 0 && s == 0 && d == 0 && cp == 0 && hp == 0) x = xb0;
            unsigned wh, wl;
            split_pair(x, wh, wl);
            xs[cp * QS + ky] = make_uint2(wh, wl);
          }
        __syncthreads();
        constexpr int P = xb_pitch(N);
        unsigned* hi = g.Xb + (size_t)f * 2 * (N / 2) * P;
        unsigned* lo = hi + (size_t)(N / 2) * P;
        for (int e = t; e < 64 * N; e += kT) {
          const int row = e >> 8, ky = e & 255;
          const uint2 wv = xs[row * QS + ky];
          hi[(size_t)(row + 64 * i) * P + ky] = wv.x;
          lo[(size_t)(row + 64 * i) * P + ky] = wv.y;
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
        for (int a = 0; a < 16; ++a) lds[cp * QS + a * 16 + c] = r[pslot(s * 16 + a, h)];
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
          const float4 v = src[q];
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
          for (int a = 0; a < 8; ++a) lds[yl * RS + a * 16 + kap(gg, s)] = r[j * 16 + s * 8 + a];
      }
    }
    __syncthreads();
    {
      const int a2 = t & 7, rq = t >> 3;
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int j = 2 * h + jj, yl = rq + 64 * jj;
        const float4* src = (const float4*)&lds[yl * RS + a2 * 16];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float4 v = src[q];
          r[j * 16 + 2 * q] = make_float2(v.x, v.y);
          r[j * 16 + 2 * q + 1] = make_float2(v.z, v.w);
        }
      }
    }
  }
  // ---------------------------------------------------------------- J2 + maximum
  unsigned long long best = 0, second = 0;
  {
    const int a2 = t & 7, rq = t >> 3;
    auto push = [&](unsigned long long k) {
      const unsigned long long lo = k < best ? k : best;
      best = k < best ? best : k;
      second = second < lo ? lo : second;
    };
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      dft16<+1>(r + 16 * j);
      const int y = rq + 64 * j;
#pragma unroll
      for (int b2 = 0; b2 < 16; ++b2) {
        const int n = a2 + 8 * b2;
        const unsigned flat = (unsigned)(y * N + 2 * n);
        push(peak_key(r[16 * j + b2].x, flat));
        push(peak_key(r[16 * j + b2].y, flat + 1));
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long b1 = __shfl_xor(best, o, 64), b2 = __shfl_xor(second, o, 64);
    const unsigned long long lo = b1 < best ? b1 : best;
    second = second > b2 ? second : b2;
    second = second > lo ? second : lo;
    best = b1 > best ? b1 : best;
  }
  // a non-finite value has a key above +inf's (NaN) or below -inf's, or equal
  bad = (kmax >= 0xFF800000u || kmin <= 0x007FFFFFu) ? 1u : 0u;
  kmin = ~wave_max(~kmin);
  kmax = wave_max(kmax);
  bad = wave_max(bad);
  if ((t & 63) == 0) {
    red[0][t >> 6] = best;
    red[1][t >> 6] = second;
    redu[0][t >> 6] = kmin;
    redu[1][t >> 6] = kmax;
    redu[2][t >> 6] = bad;
  }
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < kT / 64; ++w) {
      const unsigned long long b1 = red[0][w], b2 = red[1][w];
      const unsigned long long lo = b1 < best ? b1 : best;
      second = second > b2 ? second : b2;
      second = second > lo ? second : lo;
      best = b1 > best ? b1 : best;
      kmin = min(kmin, redu[0][w]);
      kmax = max(kmax, redu[1][w]);
      bad |= redu[2][w];
    }
    FrameState& st = g.st[f];
    st.peak_key = best;
    st.second_key = second;
    st.amin = kmin;
    st.amax = kmax;
    if (bad) st.flags |= CCPT_ST_NONFINITE;
  }
}

int launch_xcorr256(const GroupParams& g, hipStream_t s) {
  if (g.Xb)
    hipLaunchKernelGGL((k_xcorr256<true>), dim3(g.count), dim3(kT), 0, s, g);
  else
    hipLaunchKernelGGL((k_xcorr256<false>), dim3(g.count), dim3(kT), 0, s, g);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ccpt
