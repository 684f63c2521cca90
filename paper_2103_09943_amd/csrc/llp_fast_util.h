// Compile-time helpers shared by the specialised kernels (llp_fast.hip, llp_sweep.hip).
#pragma once

#include "llp_device.h"

namespace llp {

constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int cfdiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
constexpr int cpmod(int a, int b) { return a - cfdiv(a, b) * b; }
constexpr int odd(int v) { return v | 1; }
constexpr int al4(int v) { return (v + 3) & ~3; }
constexpr int pad_to(int v, int want) { return v + ((want - v % 64) + 64) % 64; }

// Periodic index for -n <= i < 2n (the host routes a geometry here only when every tile region overhangs the
// image by less than one period; see fast_path_fits).
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// B^T D^T y for output rows [F0, F0+CR) of one LR cell: yv is the cell's y neighbourhood (rows/cols
// I - YL .. I + YR), qd[f][j] accumulates output (F0 + f, j).
template <int C, int R, int YK, int YL, int F0, int CR>
__device__ __forceinline__ void cell_data_term(const float (&yv)[YK][YK], const float* __restrict__ u,
                                               float (&qd)[CR][C]) {
  constexpr int n = 2 * R + 1;
#pragma unroll
  for (int f = 0; f < CR; ++f) {
#pragma unroll
    for (int fj = 0; fj < C; ++fj) {
      const int fi = F0 + f;
      float s = 0.0f;
#pragma unroll
      for (int a = cpmod(R - fi, C); a < n; a += C) {
#pragma unroll
        for (int b = cpmod(R - fj, C); b < n; b += C) {
          const int dy = YL + (fi + a - R) / C, dx = YL + (fj + b - R) / C;
          s = fmaf(u[a * n + b], yv[dy][dx], s);
        }
      }
      qd[f][fj] = s;
    }
  }
}

// (C, R) classes with specialised kernels, for each window radius r.
#define LLP_FAST_R_LIST4(X, r) X(4, 4, r) X(4, 5, r) X(4, 6, r) X(4, 7, r) X(4, 8, r) X(4, 14, r)
#define LLP_FAST_R_LIST2(X, r) X(2, 4, r) X(2, 5, r) X(2, 6, r) X(2, 7, r) X(2, 8, r)

}  // namespace llp
