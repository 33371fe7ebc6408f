// DFT tables of the upsampled matrix DFT, built on the host in FP64 and
// rounded (or split) to the matrix-core operand type.
//
//   K[m][ky] = phi_ky((m - c)/u)                       Stage A, Mp x N complex
//   W[j][mx] = w_kx Re phi_kx((mx - c)/u) / N^2         j = kx <= N/2
//            = -2 Im phi_kx((mx - c)/u) / N^2           j = N/2 + kx, 0 < kx < N/2
//
// phi_k(s) = exp(2 pi i k~ s / N) for the signed frequency k~, and
// cos(pi s) for the Nyquist bin; w = 1 at kx = 0 and N/2, else 2.  Rows
// m >= M and columns mx >= M are zero padding up to Mp (a multiple of 32);
// W rows j >= N are zero padding up to Kb = N rounded up to 32.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/ccpt.h"

namespace ccpt {

// Stage B contraction length, padded for the matrix-core K step.
constexpr int stage_b_k(int n) { return (n + 31) / 32 * 32; }

struct HostTables {
  std::vector<float2> tw;  // exp(-2 pi i m / NY)
  std::vector<char> ky;
  std::vector<char> wb;
  int Mp = 0;
};

inline void phi_host(int k, int n, double s, double& re, double& im) {
  if (2 * k == n) {
    re = std::cos(M_PI * s);
    im = 0.0;
    return;
  }
  const int kt = 2 * k < n ? k : k - n;
  const double a = 2.0 * M_PI * (double)kt * s / (double)n;
  re = std::cos(a);
  im = std::sin(a);
}

// bf16 with round-to-nearest-even, and the hi/lo split x ~ hi + lo
inline uint16_t bf16_rne(float f) {
  uint32_t b;
  memcpy(&b, &f, 4);
  const uint32_t r = 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)((b + r) >> 16);
}
inline float bf16_to_f(uint16_t h) {
  uint32_t b = (uint32_t)h << 16;
  float f;
  memcpy(&f, &b, 4);
  return f;
}
inline void split_bf16(double x, uint16_t& hi, uint16_t& lo) {
  hi = bf16_rne((float)x);
  lo = bf16_rne((float)(x - (double)bf16_to_f(hi)));
}
// fp16 (round to nearest even by the compiler's conversion) and the hi/lo
// split x ~ hi + lo to about 22 significant bits inside the fp16 range
inline void split_f16(double x, uint16_t& hi, uint16_t& lo) {
  const _Float16 h = (_Float16)(float)x;
  const _Float16 l = (_Float16)(float)(x - (double)(float)h);
  memcpy(&hi, &h, 2);
  memcpy(&lo, &l, 2);
}

// Tables of frames of ny rows of nx pixels (nx divides ny): twiddles of
// length ny, K over ky < ny, W over kx <= nx/2 with 1/(ny nx).
inline HostTables build_tables(int ny, int nx, int u, int M, int c, int precision) {
  HostTables t;
  t.Mp = (M + 31) / 32 * 32;
  const int Mp = t.Mp;
  t.tw.resize(ny);
  for (int m = 0; m < ny; ++m) {
    const double a = 2.0 * M_PI * (double)m / (double)ny;
    t.tw[m] = make_float2((float)std::cos(a), (float)-std::sin(a));
  }
  std::vector<double> kr((size_t)Mp * ny, 0.0), ki((size_t)Mp * ny, 0.0);
  for (int m = 0; m < M; ++m)
    for (int ky = 0; ky < ny; ++ky)
      phi_host(ky, ny, (double)(m - c) / u, kr[(size_t)m * ny + ky], ki[(size_t)m * ny + ky]);
  const int Kb = stage_b_k(nx);
  std::vector<double> w((size_t)Kb * Mp, 0.0);
  const double inv = 1.0 / ((double)ny * (double)nx);
  for (int mx = 0; mx < M; ++mx) {
    const double s = (double)(mx - c) / u;
    for (int kx = 0; kx <= nx / 2; ++kx) {
      double re, im;
      phi_host(kx, nx, s, re, im);
      const double wt = (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0;
      w[(size_t)kx * Mp + mx] = wt * re * inv;
      if (kx > 0 && 2 * kx < nx) w[(size_t)(nx / 2 + kx) * Mp + mx] = -2.0 * im * inv;
    }
  }
  // Stage A operand: FP32 complex [Mp][ny] in every precision (the split
  // kernels fold the integer-peak phase into it and split it on the fly)
  t.ky.resize((size_t)Mp * ny * sizeof(float2));
  float2* K = (float2*)t.ky.data();
  for (size_t i = 0; i < (size_t)Mp * ny; ++i) K[i] = make_float2((float)kr[i], (float)ki[i]);
  if (precision == CCPT_PREC_FP32) {
    // Stage B operand, transposed W^T[mx][j] (FP32, [Mp][Kb]): a lane reads its
    // K values as contiguous 16-byte runs
    t.wb.resize((size_t)Kb * Mp * sizeof(float));
    float* W = (float*)t.wb.data();
    for (int mx = 0; mx < Mp; ++mx)
      for (int j = 0; j < Kb; ++j) W[(size_t)mx * Kb + j] = (float)w[(size_t)j * Mp + mx];
  } else if (nx == 256) {
    // (fp16 split: W scaled by 2^16, exact, so its values stay normal fp16)
    const bool f16 = precision == CCPT_PREC_FP16X2;
    // Stage B operand of the 256-column split kernel (k_updft_bf16x2_t256), in
    // the order of its k steps: wave w (kx tile 32 w .. 32 w + 31), k step s
    // (s < 2: the real rows j = kx, s >= 2: the imaginary rows j = N/2 + kx,
    // whose kx = 0 is the Nyquist row), lane l (grid column mx = 32 r + l mod
    // 32 of column tile r, half h = l / 32) holds W[j][mx] for its eight k
    // slots e = 0..7, kx = 32 w + (2 (s mod 2) + e / 4) 8 + 4 h + e mod 4:
    // [2 (hi, lo)][Mp / 32][4][4][64][8] uint16
    const int nr = Mp / 32;
    const size_t plane = (size_t)nr * 4 * 4 * 64 * 8;
    t.wb.resize(2 * plane * 2);
    uint16_t* W = (uint16_t*)t.wb.data();
    for (int r = 0; r < nr; ++r)
      for (int wv = 0; wv < 4; ++wv)
        for (int s4 = 0; s4 < 4; ++s4)
          for (int l = 0; l < 64; ++l)
            for (int e = 0; e < 8; ++e) {
              const int mx = 32 * r + (l & 31), hh = l >> 5;
              const int kx = 32 * wv + (2 * (s4 & 1) + (e >> 2)) * 8 + 4 * hh + (e & 3);
              const int jj = s4 < 2 ? kx : nx / 2 + kx;
              uint16_t hi, lo;
              if (f16)
                split_f16(w[(size_t)jj * Mp + mx] * 65536.0, hi, lo);
              else
                split_bf16(w[(size_t)jj * Mp + mx], hi, lo);
              const size_t o = ((((size_t)r * 4 + wv) * 4 + s4) * 64 + l) * 8 + e;
              W[o] = hi;
              W[plane + o] = lo;
            }
  } else {
    // Stage B operand, transposed W^T[mx][j] as bf16, hi plane then lo plane:
    // [2][Mp][Kb] uint16
    t.wb.resize((size_t)2 * Mp * Kb * 2);
    uint16_t* W = (uint16_t*)t.wb.data();
    for (int mx = 0; mx < Mp; ++mx)
      for (int j = 0; j < Kb; ++j) {
        uint16_t h, l;
        split_bf16(w[(size_t)j * Mp + mx], h, l);
        W[(size_t)mx * Kb + j] = h;
        W[(size_t)Mp * Kb + (size_t)mx * Kb + j] = l;
      }
  }
  return t;
}

// FP64-mode tables: twiddles exp(-2 pi i m / N), K[m][ky] = phi_ky((m - c)/u)
// as [Mp][N] and W[kx][mx] = w_kx phi_kx((mx - c)/u) / N^2 as [N/2+1][Mp],
// complex FP64, zero beyond M.
struct HostTables64 {
  std::vector<double2> tw, ky, wb;
};

inline HostTables64 build_tables64(int n, int u, int M, int c, int Mp) {
  HostTables64 t;
  t.tw.resize(n);
  for (int m = 0; m < n; ++m) {
    const double a = 2.0 * M_PI * (double)m / (double)n;
    t.tw[m] = make_double2(std::cos(a), -std::sin(a));
  }
  const int H = n / 2 + 1;
  t.ky.assign((size_t)Mp * n, make_double2(0.0, 0.0));
  t.wb.assign((size_t)H * Mp, make_double2(0.0, 0.0));
  const double inv = 1.0 / ((double)n * (double)n);
  for (int m = 0; m < M; ++m) {
    const double s = (double)(m - c) / u;
    for (int ky = 0; ky < n; ++ky) {
      double re, im;
      phi_host(ky, n, s, re, im);
      t.ky[(size_t)m * n + ky] = make_double2(re, im);
    }
    for (int kx = 0; kx < H; ++kx) {
      double re, im;
      phi_host(kx, n, s, re, im);
      const double wt = (kx == 0 || 2 * kx == n) ? inv : 2.0 * inv;
      t.wb[(size_t)kx * Mp + m] = make_double2(wt * re, wt * im);
    }
  }
  return t;
}

}  // namespace ccpt
