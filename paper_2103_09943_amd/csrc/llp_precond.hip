// Fourier-domain preconditioner of the conjugate-gradient solve of eq. (Z_ini_matting) (Sec. III-B), and the
// batched mixed-radix FFT it runs on.  Not part of the paper's method: P = B^T D^T D B + lambda mbar L^T L keeps
// the data term of eq. (Z_ini_matting) exactly and replaces the matting matrix of eq. (matting_matrix) by the
// scalar mbar, the mean of its diagonal.
//
// B is circular convolution (Sec. II-A), L circular convolution with the 5-point stencil (eq. reg2) and D
// decimation at phase 0, so in the Fourier domain of an H x W plane P couples only the c^2 frequencies
// (k1 + s h, k2 + t w), s, t < c, that D aliases onto one low-resolution frequency (k1, k2):
//     (P z)^[K] = d_K z^[K] + conj(U_K) / c^2 * sum_{K' in group} U_K' z^[K'],   d_K = lambda mbar Sh_K^2,
// U the DFT of the kernel and Sh the stencil's symbol.  Each group is one c^2 x c^2 block, solved per thread.
//
// Layout.  Two bands go through one complex transform (band a real, band b imaginary: P^{-1} is real, hence
// complex-linear).  The H x W plane is split into its c^2 polyphase components x_{al,be}[m][k] =
// x[c m + al][c k + be], each an h x w plane, so that
//     z^[k1 + s h][k2 + t w] = sum_{al,be} e^{-2 pi i (al k1 / H + be k2 / W)} X_{al,be}[k1][k2] w_c^{al s + be t}
// with X_{al,be} the h x w DFT of x_{al,be} and w_c = e^{-2 pi i / c}: an h x w transform per component, a
// twiddle, and a c x c DFT per low-resolution frequency.  Spectra are stored cell-major, [pair][k1][k2][al c + be]
// (c^2 complex values, 128 bytes at c = 4, per cell), so both passes read and write whole cells:
//   rows    one workgroup per (pair, LR row m): the c HR rows c m .. c m + c - 1 (coalesced) -> c^2 length-w
//           transforms in LDS -> the row of cells;
//   columns one workgroup per (pair, LR column k2): h cells -> c^2 length-h transforms -> per cell the twiddle,
//           c x c DFT, group solve, inverse c x c DFT, conjugate twiddle -> inverse length-h transforms;
//   rows    inverse length-w transforms -> the c HR rows of both bands, scaled by 1/(H W).
//
// FFT.  Stockham autosort passes of radix 8, 4, 2, 7, 5 and 3 on LDS-resident sequences: per pass every thread
// loads its butterflies' inputs into registers, multiplies by twiddles from a table evaluated in FP64 and
// rounded once, transforms, and after a barrier writes its outputs to their sorted positions.  Inverse
// transforms conjugate on the way in and out.
#include "llp_device.h"

#include <math.h>

namespace llp {
using namespace dev;

namespace {

constexpr int T = kPcThreads;
constexpr int kMaxPerThread = kPcMaxElems / T;  // complex values per thread in one pass
constexpr int kPcWaves = T / 64;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }  // -i a

// Forward DFT of R points in registers: X_m = sum_t v_t e^{-2 pi i m t / R}.
template <int R>
struct Dft;

template <>
struct Dft<2> {
  static __device__ __forceinline__ void run(float2 (&v)[2]) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <>
struct Dft<4> {
  static __device__ __forceinline__ void run(float2 (&v)[4]) {
    const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]), t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, mul_mi(t3));
    v[3] = csub(t1, mul_mi(t3));
  }
};

template <>
struct Dft<8> {
  static __device__ __forceinline__ void run(float2 (&v)[8]) {
    float2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4>::run(e);
    Dft<4>::run(o);
    constexpr float h = 0.70710678118654752f;  // cos(pi/4)
    const float2 o1 = make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));    // e^{-i pi/4} o1
    const float2 o2 = mul_mi(o[2]);                                                // e^{-i pi/2} o2
    const float2 o3 = make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));  // e^{-3 i pi/4} o3
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// Odd radices by the definition, with cos and sin of 2 pi k / R as constants.
__constant__ float kCos3[3] = {1.0f, -0.5f, -0.5f};
__constant__ float kSin3[3] = {0.0f, 0.86602540378443865f, -0.86602540378443865f};
__constant__ float kCos5[5] = {1.0f, 0.30901699437494745f, -0.80901699437494742f, -0.80901699437494742f,
                               0.30901699437494745f};
__constant__ float kSin5[5] = {0.0f, 0.95105651629515357f, 0.58778525229247313f, -0.58778525229247313f,
                               -0.95105651629515357f};
__constant__ float kCos7[7] = {1.0f, 0.62348980185873353f, -0.22252093395631440f, -0.90096886790241913f,
                               -0.90096886790241913f, -0.22252093395631440f, 0.62348980185873353f};
__constant__ float kSin7[7] = {0.0f, 0.78183148246802981f, 0.97492791218182361f, 0.43388373911755812f,
                               -0.43388373911755812f, -0.97492791218182361f, -0.78183148246802981f};

template <int R>
__device__ __forceinline__ void dft_odd(float2 (&v)[R], const float* cs, const float* sn) {
  float2 out[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    float2 acc = v[0];
#pragma unroll
    for (int t = 1; t < R; ++t) {
      const int k = (m * t) % R;  // e^{-2 pi i k / R} = cos - i sin
      acc.x += v[t].x * cs[k] + v[t].y * sn[k];
      acc.y += v[t].y * cs[k] - v[t].x * sn[k];
    }
    out[m] = acc;
  }
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = out[m];
}
template <>
struct Dft<3> {
  static __device__ __forceinline__ void run(float2 (&v)[3]) { dft_odd<3>(v, kCos3, kSin3); }
};
template <>
struct Dft<5> {
  static __device__ __forceinline__ void run(float2 (&v)[5]) { dft_odd<5>(v, kCos5, kSin5); }
};
template <>
struct Dft<7> {
  static __device__ __forceinline__ void run(float2 (&v)[7]) { dft_odd<7>(v, kCos7, kSin7); }
};

// One Stockham pass of radix R over nseq sequences of length L stored back to back in buf; Ns is the length of
// the sub-transforms already done.  tw[m] = e^{-2 pi i m / L}.
template <int R>
__device__ __forceinline__ void fft_pass(float2* buf, int L, int nseq, int Ns, const float2* __restrict__ tw) {
  constexpr int NB = (kMaxPerThread + R - 1) / R;
  const int M = L / R, total = nseq * M, stride = L / (Ns * R);
  float2 v[NB][R];
  int ob[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = (int)threadIdx.x + b * T;
    ob[b] = -1;
    if (j < total) {
      const int seq = j / M, jj = j - seq * M;
      const int k = jj % Ns;
      const float2* src = buf + seq * L + jj;
#pragma unroll
      for (int t = 0; t < R; ++t) v[b][t] = src[t * M];
#pragma unroll
      for (int t = 1; t < R; ++t) v[b][t] = cmul(v[b][t], tw[t * k * stride]);
      Dft<R>::run(v[b]);
      ob[b] = seq * L + (jj / Ns) * Ns * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (ob[b] >= 0) {
#pragma unroll
      for (int t = 0; t < R; ++t) buf[ob[b] + t * Ns] = v[b][t];
    }
  }
  __syncthreads();
}

// Forward DFT of nseq sequences of length L in LDS (radices rad[0..nrad), product L).
__device__ void fft_lds(float2* buf, int L, int nseq, const int* rad, int nrad, const float2* __restrict__ tw) {
  int Ns = 1;
  for (int p = 0; p < nrad; ++p) {
    const int R = rad[p];
    switch (R) {
      case 8: fft_pass<8>(buf, L, nseq, Ns, tw); break;
      case 4: fft_pass<4>(buf, L, nseq, Ns, tw); break;
      case 2: fft_pass<2>(buf, L, nseq, Ns, tw); break;
      case 3: fft_pass<3>(buf, L, nseq, Ns, tw); break;
      case 5: fft_pass<5>(buf, L, nseq, Ns, tw); break;
      default: fft_pass<7>(buf, L, nseq, Ns, tw); break;
    }
    Ns *= R;
  }
}

template <typename F>
__device__ __forceinline__ int find_pc(const PcDesc* t, int count, int bid, F first) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first(t[mid]) <= bid) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// w_c^k = e^{-2 pi i k / c} for c <= 4.
__device__ __forceinline__ float2 root_c(int c, int k) {
  k %= c;
  if (c == 2) return make_float2(k ? -1.0f : 1.0f, 0.0f);
  if (c == 4) {
    const float2 r4[4] = {{1.0f, 0.0f}, {0.0f, -1.0f}, {-1.0f, 0.0f}, {0.0f, 1.0f}};
    return r4[k];
  }
  if (c == 3) return make_float2(kCos3[k], -kSin3[k]);
  return make_float2(1.0f, 0.0f);
}

// Solve (diag(d) + conj(U) U^T / c^2) x = F on one group (n = c^2 members).  The member with the smallest d is
// eliminated through the rank-one equation when the rank-one term dominates its row (the frequency nearest
// 0, where d is tiny or, at K = 0, zero): there the Sherman-Morrison form would cancel catastrophically.
__device__ __forceinline__ void group_solve(int c, const float2* F, const float2* U, const float* d, float2* x) {
  const int n = c * c;
  const float c2 = (float)n;
  int js = 0;
  for (int j = 1; j < n; ++j)
    if (d[j] < d[js]) js = j;
  const float u2 = U[js].x * U[js].x + U[js].y * U[js].y;
  if (d[js] * c2 < u2) {
    // S = U^T x / c^2 from the scaled normal equation; x_j = (F_j - conj(U_j) S) / d_j for j != js; x_js from
    // c^2 S = sum_j U_j x_j.
    const float sc = d[js];
    float2 num = make_float2(0.0f, 0.0f);
    float den = c2 * sc;
    for (int k = 0; k < n; ++k) {
      const float wk = k == js ? 1.0f : sc / d[k];
      num = cadd(num, make_float2(wk * (U[k].x * F[k].x - U[k].y * F[k].y), wk * (U[k].x * F[k].y + U[k].y * F[k].x)));
      den += wk * (U[k].x * U[k].x + U[k].y * U[k].y);
    }
    const float2 S = make_float2(num.x / den, num.y / den);
    float2 rest = make_float2(0.0f, 0.0f);
    for (int j = 0; j < n; ++j) {
      if (j == js) continue;
      const float2 xj = csub(F[j], cmul(conjf2(U[j]), S));
      x[j] = make_float2(xj.x / d[j], xj.y / d[j]);
      rest = cadd(rest, cmul(U[j], x[j]));
    }
    const float2 t = csub(make_float2(c2 * S.x, c2 * S.y), rest);  // U_js x_js
    x[js] = make_float2((t.x * U[js].x + t.y * U[js].y) / u2, (t.y * U[js].x - t.x * U[js].y) / u2);
  } else {
    float2 num = make_float2(0.0f, 0.0f);
    float den = c2;
    for (int k = 0; k < n; ++k) {
      const float ek = 1.0f / d[k];
      num = cadd(num, make_float2(ek * (U[k].x * F[k].x - U[k].y * F[k].y), ek * (U[k].x * F[k].y + U[k].y * F[k].x)));
      den += ek * (U[k].x * U[k].x + U[k].y * U[k].y);
    }
    const float2 S = make_float2(num.x / den, num.y / den);
    for (int j = 0; j < n; ++j) {
      const float2 xj = csub(F[j], cmul(conjf2(U[j]), S));
      x[j] = make_float2(xj.x / d[j], xj.y / d[j]);
    }
  }
}

__device__ __forceinline__ bool band_runs(const ChanState* st, int band, int nbands) {
  return band < nbands && st[band].active;
}

}  // namespace

// ------------------------------------------------------------------------------------------- row pass ---
// op kPcRowsStart: the bands' residual r[prev] as it is; kPcRowsUpdate: r[cur] = r[prev] - alpha q and
// z += alpha p[prev] first (the CG update of iteration k); kPcRowsKernel: the blur kernel embedded in an H x W
// plane with its centre tap at (0, 0), in band a of pair 0.  Partial sums of |r|^2 per band go to slot 0 of
// the band's partials (one per LR row).

__global__ __launch_bounds__(T) void k_pc_rows(int op, const PcDesc* __restrict__ t, int count,
                                               const ChanState* __restrict__ st, int prev, int cur) {
  extern __shared__ float2 pcsh[];
  __shared__ double red[2 * kPcWaves];
  const int si = find_pc(t, count, (int)blockIdx.x, [](const PcDesc& d) { return d.row_block0; });
  const PcDesc& d = t[si];
  const Geom& g = d.g;
  const int local = (int)blockIdx.x - d.row_block0;
  const int npair = op == kPcRowsKernel ? 1 : d.npair;
  if (local >= npair * g.h) return;
  const int pair = local / g.h, m = local - pair * g.h;
  const int c = g.c, c2 = c * c, W = g.W, w = g.w;
  const int ba = 2 * pair, bb = 2 * pair + 1;
  const ChanState* sst = st + d.band0;
  const bool ra = op != kPcRowsKernel && band_runs(sst, ba, g.N);
  const bool rb = op != kPcRowsKernel && band_runs(sst, bb, g.N);
  if (op != kPcRowsKernel && !ra && !rb) return;
  const float al_a = ra ? (float)sst[ba].alpha : 0.0f, al_b = rb ? (float)sst[bb].alpha : 0.0f;
  const size_t HW = (size_t)g.H * W;
  double acc_a = 0.0, acc_b = 0.0;
  for (int idx = threadIdx.x; idx < c * W; idx += T) {
    const int al = idx / W, j = idx - al * W;
    const int i = c * m + al;
    const size_t e = (size_t)i * W + j;
    float va = 0.0f, vb = 0.0f;
    if (op == kPcRowsKernel) {
      int a = i + g.R, b = j + g.R;  // plane (i, j) holds u[(i + R) mod H][(j + R) mod W] if inside the kernel
      if (a >= g.H) a -= g.H;
      if (b >= W) b -= W;
      if (a < g.n && b < g.n) va = d.u[a * g.n + b];
    } else {
      if (ra) {
        const size_t o = (size_t)ba * HW + e;
        va = d.r[prev][o];
        if (op == kPcRowsUpdate) {
          va = fmaf(-al_a, d.q[o], va);
          d.r[cur][o] = va;
          d.z[o] = fmaf(al_a, d.p[prev][o], d.z[o]);
        }
        acc_a += (double)va * va;
      }
      if (rb) {
        const size_t o = (size_t)bb * HW + e;
        vb = d.r[prev][o];
        if (op == kPcRowsUpdate) {
          vb = fmaf(-al_b, d.q[o], vb);
          d.r[cur][o] = vb;
          d.z[o] = fmaf(al_b, d.p[prev][o], d.z[o]);
        }
        acc_b += (double)vb * vb;
      }
    }
    const int be = j % c, n = j / c;
    pcsh[(al * c + be) * w + n] = make_float2(va, vb);
  }
  __syncthreads();
  fft_lds(pcsh, w, c2, d.rw, d.nrw, d.tww);
  float2* out = d.spec + ((size_t)pair * g.h + m) * (size_t)w * c2;
  for (int e = threadIdx.x; e < w * c2; e += T) {
    const int k2 = e / c2, ph = e - k2 * c2;
    out[e] = pcsh[ph * w + k2];
  }
  if (op == kPcRowsKernel) return;
  double v[2] = {acc_a, acc_b};
  block_sums<2, kPcWaves>(v, red);
  if (threadIdx.x == 0) {
    if (ra) d.partials[(size_t)ba * d.pstride * 3 + (size_t)m * 3 + 0] = v[0];
    if (rb) d.partials[(size_t)bb * d.pstride * 3 + (size_t)m * 3 + 0] = v[1];
  }
}

// ---------------------------------------------------------------------------------------- column pass ---
// op kPcColsSolve: forward length-h transforms, the group solve of every cell, inverse transforms (unscaled;
// the inverse c x c DFT carries 1/c^2).  op kPcColsData: the same with the data term B^T D^T D B applied to
// every group instead of P^{-1}.  op kPcColsKernel: forward transforms and the c x c DFT of pair 0 (the
// embedded kernel), stored as U in the cell layout.

__global__ __launch_bounds__(T) void k_pc_cols(int op, const PcDesc* __restrict__ t, int count,
                                               const ChanState* __restrict__ st) {
  extern __shared__ float2 pcsh[];
  const int si = find_pc(t, count, (int)blockIdx.x, [](const PcDesc& d) { return d.col_block0; });
  const PcDesc& d = t[si];
  const Geom& g = d.g;
  const int local = (int)blockIdx.x - d.col_block0;
  const int npair = op == kPcColsKernel ? 1 : d.npair;
  if (local >= npair * g.w) return;
  const int pair = local / g.w, k2 = local - pair * g.w;
  const int c = g.c, c2 = c * c, h = g.h, w = g.w, H = g.H, W = g.W;
  if (op != kPcColsKernel) {
    const ChanState* sst = st + d.band0;
    if (!band_runs(sst, 2 * pair, g.N) && !band_runs(sst, 2 * pair + 1, g.N)) return;
  }
  float2* sp = d.spec + (size_t)pair * h * w * c2;
  for (int e = threadIdx.x; e < h * c2; e += T) {
    const int m = e / c2, ph = e - m * c2;
    pcsh[ph * h + m] = sp[((size_t)m * w + k2) * c2 + ph];
  }
  __syncthreads();
  fft_lds(pcsh, h, c2, d.rh, d.nrh, d.twh);
  const float dscale = op == kPcColsSolve ? (float)((double)g.lam * d.mbar[0]) : 0.0f;
  const float inv_c2 = 1.0f / (float)c2;
  for (int k1 = threadIdx.x; k1 < h; k1 += T) {
    float2 Q[16], F[16];
    // twiddle e^{-2 pi i (al k1 / H + be k2 / W)}
    for (int al = 0; al < c; ++al)
      for (int be = 0; be < c; ++be)
        Q[al * c + be] = cmul(pcsh[(al * c + be) * h + k1], cmul(d.twH[al * k1], d.twW[be * k2]));
    // c x c DFT: F[s c + t] = sum_{al, be} Q[al c + be] w_c^{al s + be t}
    for (int s = 0; s < c; ++s)
      for (int tt = 0; tt < c; ++tt) {
        float2 acc = make_float2(0.0f, 0.0f);
        for (int al = 0; al < c; ++al)
          for (int be = 0; be < c; ++be) acc = cadd(acc, cmul(Q[al * c + be], root_c(c, al * s + be * tt)));
        F[s * c + tt] = acc;
      }
    float2* uc = d.uhat + ((size_t)k1 * w + k2) * c2;
    if (op == kPcColsKernel) {
      for (int j = 0; j < c2; ++j) uc[j] = F[j];
      continue;
    }
    float2 U[16], X[16];
    for (int j = 0; j < c2; ++j) U[j] = uc[j];
    if (op == kPcColsData) {  // B^T D^T D B in the Fourier domain: conj(U_j) / c^2 * sum_k U_k F_k
      float2 S = make_float2(0.0f, 0.0f);
      for (int k = 0; k < c2; ++k) S = cadd(S, cmul(U[k], F[k]));
      S = make_float2(S.x * inv_c2, S.y * inv_c2);
      for (int j = 0; j < c2; ++j) X[j] = cmul(conjf2(U[j]), S);
    } else {
      float dd[16];
      for (int s = 0; s < c; ++s)
        for (int tt = 0; tt < c; ++tt) {
          const float sym = 4.0f - 2.0f * d.twH[k1 + s * h].x - 2.0f * d.twW[k2 + tt * w].x;
          dd[s * c + tt] = dscale * sym * sym;
        }
      group_solve(c, F, U, dd, X);
    }
    // inverse c x c DFT (1/c^2), conjugate twiddle; stored conjugated for the inverse length-h transforms
    for (int al = 0; al < c; ++al)
      for (int be = 0; be < c; ++be) {
        float2 acc = make_float2(0.0f, 0.0f);
        for (int s = 0; s < c; ++s)
          for (int tt = 0; tt < c; ++tt) acc = cadd(acc, cmul(X[s * c + tt], conjf2(root_c(c, al * s + be * tt))));
        acc = cmul(acc, conjf2(cmul(d.twH[al * k1], d.twW[be * k2])));
        pcsh[(al * c + be) * h + k1] = make_float2(acc.x * inv_c2, -acc.y * inv_c2);
      }
  }
  if (op == kPcColsKernel) return;
  __syncthreads();
  fft_lds(pcsh, h, c2, d.rh, d.nrh, d.twh);
  for (int e = threadIdx.x; e < h * c2; e += T) {
    const int m = e / c2, ph = e - m * c2;
    sp[((size_t)m * w + k2) * c2 + ph] = conjf2(pcsh[ph * h + m]);
  }
}

// ------------------------------------------------------------------------------------ inverse row pass ---
// s = P^{-1} r for both bands of a pair (inverse length-w transforms, scale 1/(h w)), and the partial sums of
// r[cur]^T s per band into slot 1 of the band's partials.

__global__ __launch_bounds__(T) void k_pc_rows_inv(const PcDesc* __restrict__ t, int count,
                                                   const ChanState* __restrict__ st, int cur) {
  extern __shared__ float2 pcsh[];
  __shared__ double red[2 * kPcWaves];
  const int si = find_pc(t, count, (int)blockIdx.x, [](const PcDesc& d) { return d.row_block0; });
  const PcDesc& d = t[si];
  const Geom& g = d.g;
  const int local = (int)blockIdx.x - d.row_block0;
  if (local >= d.npair * g.h) return;
  const int pair = local / g.h, m = local - pair * g.h;
  const int c = g.c, c2 = c * c, W = g.W, w = g.w;
  const int ba = 2 * pair, bb = 2 * pair + 1;
  const ChanState* sst = st + d.band0;
  const bool ra = band_runs(sst, ba, g.N), rb = band_runs(sst, bb, g.N);
  if (!ra && !rb) return;
  const float2* in = d.spec + ((size_t)pair * g.h + m) * (size_t)w * c2;
  for (int e = threadIdx.x; e < w * c2; e += T) {
    const int k2 = e / c2, ph = e - k2 * c2;
    pcsh[ph * w + k2] = conjf2(in[e]);
  }
  __syncthreads();
  fft_lds(pcsh, w, c2, d.rw, d.nrw, d.tww);
  const float scale = 1.0f / ((float)g.h * (float)w);
  const size_t HW = (size_t)g.H * W;
  double acc_a = 0.0, acc_b = 0.0;
  for (int idx = threadIdx.x; idx < c * W; idx += T) {
    const int al = idx / W, j = idx - al * W;
    const size_t e = (size_t)(c * m + al) * W + j;
    const float2 v = pcsh[(al * c + j % c) * w + j / c];
    if (ra) {
      const size_t o = (size_t)ba * HW + e;
      const float sv = v.x * scale;
      d.s[o] = sv;
      acc_a += (double)d.r[cur][o] * sv;
    }
    if (rb) {
      const size_t o = (size_t)bb * HW + e;
      const float sv = -v.y * scale;
      d.s[o] = sv;
      acc_b += (double)d.r[cur][o] * sv;
    }
  }
  double v[2] = {acc_a, acc_b};
  block_sums<2, kPcWaves>(v, red);
  if (threadIdx.x == 0) {
    if (ra) d.partials[(size_t)ba * d.pstride * 3 + (size_t)m * 3 + 1] = v[0];
    if (rb) d.partials[(size_t)bb * d.pstride * 3 + (size_t)m * 3 + 1] = v[1];
  }
}

// --------------------------------------------------------------------------------------------- mbar ---
// mbar = mean of diag(M_LY).  Summing eq. (matting_matrix)'s diagonal over all pixels window by window gives
// sum_k (|w| - 1 - var_k dinv_k), and var_k dinv_k = 1 - (eps/|w|) dinv_k where dinv_k != 0 (0 otherwise):
// mbar = |w| - 1 - mean_k(var_k dinv_k), one reduction over the dinv plane.

__global__ __launch_bounds__(kBlock) void k_pc_mbar(const PcDesc* __restrict__ t, double* __restrict__ part) {
  __shared__ double red[kWaves];
  const PcDesc& d = t[blockIdx.y];
  const Geom& g = d.g;
  const size_t HW = (size_t)g.H * g.W;
  const double epsw = (double)g.eps / (double)((2 * g.r + 1) * (2 * g.r + 1));
  const float* di = d.DI;
  double acc = 0.0;
  for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < HW; e += (size_t)gridDim.x * kBlock) {
    const double v = di[e];
    acc += v != 0.0 ? 1.0 - epsw * v : 0.0;
  }
  double v[1] = {acc};
  block_partials<1>(v, red, part + (size_t)blockIdx.y * gridDim.x + blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_pc_mbar_fin(const PcDesc* __restrict__ t, int nblk,
                                                        const double* __restrict__ part) {
  __shared__ double red[kWaves];
  const PcDesc& d = t[blockIdx.x];
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kBlock) s += part[(size_t)blockIdx.x * nblk + i];
  double v[1] = {s};
  block_sums<1>(v, red);
  if (threadIdx.x == 0) {
    const Geom& g = d.g;
    const double nw = (double)((2 * g.r + 1) * (2 * g.r + 1));
    d.mbar[0] = nw - 1.0 - v[0] / ((double)g.H * (double)g.W);
  }
}

// ------------------------------------------------------------------------------------------------ host ---

int pc_radices(int L, int* rad) {
  int n = 0;
  for (int r : {8, 4, 2, 7, 5, 3})
    while (L % r == 0 && n < kPcMaxRad) {
      rad[n++] = r;
      L /= r;
    }
  return L == 1 ? n : -1;
}

bool pc_supported(const Geom& g) {
  int rad[kPcMaxRad];
  if (g.c < 1 || g.c > 4 || g.r < 1 || !(g.lam > 0.0f)) return false;
  if ((size_t)g.c * g.W > (size_t)kPcMaxElems || (size_t)g.c * g.H > (size_t)kPcMaxElems) return false;
  return pc_radices(g.w, rad) >= 0 && pc_radices(g.h, rad) >= 0;
}

int pc_row_blocks(const Geom& g) { return ((g.N + 1) / 2) * g.h; }
int pc_col_blocks(const Geom& g) { return ((g.N + 1) / 2) * g.w; }

size_t pc_spec_floats(const Geom& g) { return (size_t)((g.N + 1) / 2) * g.H * g.W * 2; }
size_t pc_uhat_floats(const Geom& g) { return (size_t)g.H * g.W * 2; }
size_t pc_tw_floats(const Geom& g) { return (size_t)2 * (g.h + g.w + g.H + g.W); }

void pc_twiddles(const Geom& g, float* out) {
  const int lens[4] = {g.h, g.w, g.H, g.W};
  for (int L : lens)
    for (int m = 0; m < L; ++m) {
      const double a = -2.0 * M_PI * (double)m / (double)L;
      *out++ = (float)cos(a);
      *out++ = (float)sin(a);
    }
}

void pc_fill(PcDesc& d, const Geom& g, float* tw_dev) {
  d.g = g;
  d.npair = (g.N + 1) / 2;
  float2* tw = (float2*)tw_dev;
  d.twh = tw;
  d.tww = tw + g.h;
  d.twH = tw + g.h + g.w;
  d.twW = tw + g.h + g.w + g.H;
  d.nrw = pc_radices(g.w, d.rw);
  d.nrh = pc_radices(g.h, d.rh);
}

hipError_t pc_prepare() {
  const int bytes = kPcMaxElems * (int)sizeof(float2);
  hipError_t e = hipFuncSetAttribute((const void*)k_pc_rows, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_pc_cols, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_pc_rows_inv, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

static size_t pc_row_lds(const PcDesc* h_tab, int count) {
  size_t m = 0;
  for (int i = 0; i < count; ++i) {
    const size_t b = (size_t)h_tab[i].g.c * h_tab[i].g.W * sizeof(float2);
    if (b > m) m = b;
  }
  return m;
}

static size_t pc_col_lds(const PcDesc* h_tab, int count) {
  size_t m = 0;
  for (int i = 0; i < count; ++i) {
    const size_t b = (size_t)h_tab[i].g.c * h_tab[i].g.H * sizeof(float2);
    if (b > m) m = b;
  }
  return m;
}

void pc_plan(PcDesc* h_tab, int count, PcPlan* plan) {
  PcPlan P;
  P.count = count;
  for (int i = 0; i < count; ++i) {
    h_tab[i].row_block0 = P.row_blocks;
    h_tab[i].col_block0 = P.col_blocks;
    P.row_blocks += pc_row_blocks(h_tab[i].g);
    P.col_blocks += pc_col_blocks(h_tab[i].g);
    P.bands += h_tab[i].g.N;
  }
  P.row_lds = pc_row_lds(h_tab, count);
  P.col_lds = pc_col_lds(h_tab, count);
  *plan = P;
}

hipError_t launch_pc_rows(int op, const PcDesc* t, const PcPlan& P, const ChanState* st, int prev, int cur,
                          hipStream_t s) {
  if (P.row_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pc_rows, dim3(P.row_blocks), dim3(T), P.row_lds, s, op, t, P.count, st, prev, cur);
  return hipGetLastError();
}

hipError_t launch_pc_cols(int op, const PcDesc* t, const PcPlan& P, const ChanState* st, hipStream_t s) {
  if (P.col_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pc_cols, dim3(P.col_blocks), dim3(T), P.col_lds, s, op, t, P.count, st);
  return hipGetLastError();
}

hipError_t launch_pc_rows_inv(const PcDesc* t, const PcPlan& P, const ChanState* st, int cur, hipStream_t s) {
  if (P.row_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pc_rows_inv, dim3(P.row_blocks), dim3(T), P.row_lds, s, t, P.count, st, cur);
  return hipGetLastError();
}

hipError_t launch_pc_mbar(const PcDesc* t, int count, double* part, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pc_mbar, dim3(kPcMbarBlocks, count), dim3(kBlock), 0, s, t, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pc_mbar_fin, dim3(count), dim3(kBlock), 0, s, t, kPcMbarBlocks, part);
  return hipGetLastError();
}

}  // namespace llp
