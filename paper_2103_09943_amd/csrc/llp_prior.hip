// The cross-channel priors of the paper's prior comparison (Sec. IV, Table "cross_channel_prior") as other
// operators in place of LLP: the window penalty of eq. (reg2) applied to F_d Z and F_d Y for one or two
// filters F_d instead of the Laplacian (LGC: the two gradients of eq. (reg2_lgc); LPP: the identity; LPF: the
// blur kernel; HPF: delta minus the blur kernel).  Minimising over the window coefficients gives, as for LLP,
//   (B^T D^T D B + lambda sum_d F_d^T M_{F_d Y} F_d) Z = B^T D^T X,
// solved here by plain conjugate gradients on float32 vectors with FP64 dot products.
//
//   k_prior_taps    the filters' taps (from the blur kernel for LPF and HPF);
//   k_prior_guide   the guide F_d Y (FP64) of each filter;
//   k_prior_wstats  its window means and 1 / (eps/|w| + var) (FP64 window sums);
//   k_prior_apply   q = A p for a tile: stage p with the halo every stage needs, then per filter
//                   l = F_d p, the matting product M l by window sums (as for LLP), F_d^T (M l) accumulated;
//                   finally B^T D^T y (y = D B p from the shared direction kernel) and the dot products the
//                   CG step needs;
//   k_prior_resid / k_prior_verify / k_prior_restart  the true-residual check of a band whose recursive residual
//                   met the tolerance, and its restart from that residual when the check fails.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "llp_ctx.h"
#include "llp_device.h"

namespace llp {

using namespace dev;

namespace {

constexpr int kPriorMaxSide = 31;  // longest filter side
constexpr int kPriorTapStride = kPriorMaxSide * kPriorMaxSide;
constexpr int kPriorTW = 64;
constexpr int kPriorFlat = kBlock * 16;  // elements per workgroup of the flat kernels
constexpr int kStageBatch = 8;           // loads a thread keeps in flight while staging a region
constexpr int kPB = 512, kPW = kPB / 64;  // k_prior_apply: threads and waves per workgroup

__host__ __device__ inline int prior_th(int c) { return c == 3 ? 24 : 16; }  // tile rows (tile count <= the
                                                                             // operator's, for the partials)

struct PriorArgs {
  int mode;  // 0: q = A p;  1: also the partials of p^T q, r^T q, q^T q
  int nf;    // filters, 1 or 2
  int F[2];  // filter sides (odd)
  const float* taps;  // [2][kPriorTapStride], filter d row-major F[d] x F[d] at d * kPriorTapStride
  const float* G[2];
  const float* MU[2];
  const float* DI[2];
  const float* p;
  const float* r;
  const float* y;
  float* q;
  double* partials;
  ChanState* st;
  int TH, tiles_x, ntiles, pstride;
  int E;  // halo of the staged p: 2 max(RF) + 2r
  int offL, offX, offG, offH, offA, offQ, offY, offT, offU, offR, YW;
  int FT, RW;  // kernel instance: compile-time filter side (1, 3) and window radius (1, 2), or 0
};

}  // namespace

// The filters of a prior: LLP the 5-point Laplacian S of eq. (reg2); LGC the forward differences (taps at
// offsets (0, -1) and (-1, 0), true convolution); LPP a single unit tap; LPF the kernel u; HPF delta - u.
__global__ void k_prior_taps(int kind, const float* __restrict__ u, int n, float* __restrict__ taps) {
  for (int i = threadIdx.x; i < 2 * kPriorTapStride; i += blockDim.x) taps[i] = 0.0f;
  __syncthreads();
  if (kind == LLP_PRIOR_LLP) {
    if (threadIdx.x < 9) {
      const int a = threadIdx.x / 3, b = threadIdx.x % 3;
      taps[threadIdx.x] = (a == 1 && b == 1) ? 4.0f : ((a == 1) != (b == 1) ? -1.0f : 0.0f);
    }
  } else if (kind == LLP_PRIOR_LGC) {
    if (threadIdx.x == 0) {
      taps[1 * 3 + 0] = 1.0f;  // horizontal: z[i][j+1] - z[i][j]
      taps[1 * 3 + 1] = -1.0f;
      taps[kPriorTapStride + 0 * 3 + 1] = 1.0f;  // vertical: z[i+1][j] - z[i][j]
      taps[kPriorTapStride + 1 * 3 + 1] = -1.0f;
    }
  } else if (kind == LLP_PRIOR_LPP) {
    if (threadIdx.x == 0) taps[0] = 1.0f;
  } else {
    const int R = (n - 1) / 2;
    for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
      float v = u[i];
      if (kind == LLP_PRIOR_HPF) v = (i == R * n + R) ? 1.0f - v : -v;
      taps[i] = v;
    }
  }
}

// g64 = F Y (true convolution, centre tap at offset 0), in FP64; G its float32 value.
__global__ __launch_bounds__(kBlock) void k_prior_guide(Geom g, const float* __restrict__ Y,
                                                        const float* __restrict__ f, int F,
                                                        double* __restrict__ g64, float* __restrict__ G) {
  const size_t HW = (size_t)g.H * g.W;
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= HW) return;
  const int i = (int)(idx / g.W), j = (int)(idx - (size_t)i * g.W);
  const int RF = (F - 1) / 2;
  double s = 0.0;
  for (int a = 0; a < F; ++a) {
    const size_t row = (size_t)wrapi(i - (a - RF), g.H) * g.W;
    for (int b = 0; b < F; ++b) s += (double)f[a * F + b] * (double)Y[row + wrapi(j - (b - RF), g.W)];
  }
  g64[idx] = s;
  G[idx] = (float)s;
}

// Window mean of the guide and 1 / (eps/|w| + var), 0 where that denominator is 0 (eq. matting_matrix).
__global__ __launch_bounds__(kBlock) void k_prior_wstats(Geom g, const double* __restrict__ g64,
                                                         float* __restrict__ MU, float* __restrict__ DI) {
  const size_t HW = (size_t)g.H * g.W;
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= HW) return;
  const int i = (int)(idx / g.W), j = (int)(idx - (size_t)i * g.W);
  const int r = g.r;
  const double nw = (double)((2 * r + 1) * (2 * r + 1));
  double s1 = 0.0, s2 = 0.0;
  for (int dy = -r; dy <= r; ++dy) {
    const size_t row = (size_t)wrapi(i + dy, g.H) * g.W;
    for (int dx = -r; dx <= r; ++dx) {
      const double v = g64[row + wrapi(j + dx, g.W)];
      s1 += v;
      s2 += v * v;
    }
  }
  const double mu = s1 / nw;
  const double den = (double)g.eps / nw + (s2 / nw - mu * mu);
  MU[idx] = (float)mu;
  DI[idx] = den != 0.0 ? (float)(1.0 / den) : 0.0f;
}

// q = B^T D^T y + lambda sum_d F_d^T M_d F_d p on one tile of one band (and the CG partials in mode 1).
// FT: the filter side at compile time (1 or 3; taps in registers), 0: any side (taps staged in LDS); RW: the
// window radius at compile time (1, 2), 0: any.  Every global
// read is staged into LDS up front (p, then per filter its guide, window means and inverse denominators), so the
// stages run on LDS only; tiles whose halo stays inside the image index without wrapping.
template <int FT, int RW>
__global__ __launch_bounds__(kPB) void k_prior_apply(Geom g, PriorArgs A, const float* __restrict__ u) {
  extern __shared__ float smem[];
  __shared__ double red[3 * kPW];
  int tile, ch;
  tile_and_band(A.ntiles, g.N, blockIdx.x, tile, ch);
  if (A.mode == 1 && !A.st[ch].active) return;
  const int TH = A.TH, TW = kPriorTW;
  const int i0 = (tile / A.tiles_x) * TH, j0 = (tile % A.tiles_x) * TW;
  const int H = g.H, W = g.W, r = RW > 0 ? RW : g.r, C = g.c, R = g.R, n = g.n;
  const size_t HW = (size_t)H * W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int E = A.E, PH = TH + 2 * E, PW = TW + 2 * E;
  const bool wrapped = i0 - E < 0 || j0 - E < 0 || i0 + TH + E > H || j0 + TW + E > W;
  float* P = smem;
  float* Ls = smem + A.offL;
  float* Xs = smem + A.offX;
  float* Gs = smem + A.offG;
  float* Hs = smem + A.offH;
  float* As = smem + A.offA;
  float* Q = smem + A.offQ;
  float* Ys = smem + A.offY;
  float* Ts = smem + A.offT;
  const float* pc = A.p + (size_t)ch * HW;
  // rows*cols region with top-left global pixel (gi0, gj0), periodic, from plane src into dst (row stride cols).
  // Every thread issues kStageBatch loads (clamped, unconditional) before it stores any, so the loads of a batch
  // are in flight together.
  auto stage = [&](float* dst, const float* src, int gi0, int gj0, int rows, int cols) {
    const int total = rows * cols;
    const float inv = 1.0f / (float)cols;
    for (int base = threadIdx.x; base < total; base += kStageBatch * kPB) {
      float v[kStageBatch];
#pragma unroll
      for (int k = 0; k < kStageBatch; ++k) {
        const int e = min(base + k * kPB, total - 1);
        const int row = __float2int_rz(((float)e + 0.5f) * inv), col = e - row * cols;
        const int gi = gi0 + row, gj = gj0 + col;
        v[k] = wrapped ? src[(size_t)wrapi(gi, H) * W + wrapi(gj, W)] : src[(size_t)gi * W + gj];
      }
#pragma unroll
      for (int k = 0; k < kStageBatch; ++k)
        if (base + k * kPB < total) dst[base + k * kPB] = v[k];
    }
  };

  // body(row, col) over a rows x cols region, the elements dealt to the threads in row-major order (regions
  // are a little wider than 64 columns, so row-by-row loops would leave most lanes idle on every second pass).
  auto flat = [&](int rows, int cols, auto&& body) {
    const int total = rows * cols;
    const float inv = 1.0f / (float)cols;
    for (int e = threadIdx.x; e < total; e += kPB) {
      const int row = __float2int_rz(((float)e + 0.5f) * inv);
      body(row, e - row * cols);
    }
  };

  // p on [i0-E, i0+TH+E) x [j0-E, j0+TW+E), the LR y the tile's B^T D^T taps reach, a cleared accumulator.
  stage(P, pc, i0 - E, j0 - E, PH, PW);
  const int mlo = floor_div(i0 - R, C), klo = floor_div(j0 - R, C);
  const int YH = (TH - 1 + 2 * R) / C + 2, YW = A.YW;
  {
    const float* yc = A.y + (size_t)ch * g.h * g.w;
    for (int row = wave; row < YH; row += kPW) {
      const size_t ro = (size_t)wrapi(mlo + row, g.h) * g.w;
      for (int col = lane; col < YW; col += 64) Ys[row * YW + col] = yc[ro + wrapi(klo + col, g.w)];
    }
  }
  for (int e = threadIdx.x; e < TH * TW; e += kPB) Q[e] = 0.0f;
  float* Rs = smem + A.offR;  // r on the tile (mode 1: r^T q)
  if (A.mode == 1) stage(Rs, A.r + (size_t)ch * HW, i0, j0, TH, TW);
  float* Us = smem + A.offU;  // the blur kernel: lanes of a wave sit on different phases and read different taps
  for (int e = threadIdx.x; e < n * n; e += kPB) Us[e] = u[e];

  const float nwf = (float)((2 * r + 1) * (2 * r + 1)), inv_nw = 1.0f / nwf;
  for (int d = 0; d < A.nf; ++d) {
    const int F = FT > 0 ? FT : A.F[d], RF = (F - 1) / 2;
    const float* f = A.taps + d * kPriorTapStride;
    const int LH = TH + 2 * (RF + 2 * r), LW = TW + 2 * (RF + 2 * r);
    const int AH = TH + 2 * (RF + r), AW = TW + 2 * (RF + r);
    const int MH = TH + 2 * RF, W3 = TW + 2 * RF;
    const int off = E - (RF + 2 * r);  // P index of l-space (0, 0) before the tap shift
    float tp[FT > 0 ? FT * FT : 1];
    if (FT > 0) {
#pragma unroll
      for (int t = 0; t < (FT > 0 ? FT * FT : 1); ++t) tp[t] = f[t];
    } else {
      for (int t = threadIdx.x; t < F * F; t += kPB) Ts[t] = f[t];
    }
    // the filter's guide on l-space, its window means and inverse denominators on a-space (into the a, b slots)
    float* Aa = As;
    float* Ab = As + AH * AW;
    stage(Gs, A.G[d], i0 - RF - 2 * r, j0 - RF - 2 * r, LH, LW);
    stage(Aa, A.MU[d], i0 - RF - r, j0 - RF - r, AH, AW);
    stage(Ab, A.DI[d], i0 - RF - r, j0 - RF - r, AH, AW);
    __syncthreads();

    // l = F p and G l on l-space [i0-RF-2r, ..) x [j0-RF-2r, ..): l(x) = sum_{a,b} f[a][b] p(x - (a-RF, b-RF)).
    flat(LH, LW, [&](int row, int col) {
        const float* pb = P + (row + off + RF) * PW + col + off + RF;
        float s = 0.0f;
        if (FT > 0) {
#pragma unroll
          for (int a = 0; a < (FT > 0 ? FT : 1); ++a)
#pragma unroll
            for (int b = 0; b < (FT > 0 ? FT : 1); ++b) s = fmaf(tp[a * FT + b], pb[-a * PW - b], s);
        } else {
          for (int a = 0; a < F; ++a) {
            const float* pr = pb - a * PW;
            const float* fr = Ts + a * F;
            for (int b = 0; b < F; ++b) s = fmaf(fr[b], pr[-b], s);
          }
        }
        Ls[row * LW + col] = s;
        Xs[row * LW + col] = Gs[row * LW + col] * s;
    });
    __syncthreads();
    // Horizontal window sums of l and G l, a-space columns.
    float* Hl = Hs;
    float* Hg = Hs + LH * AW;
    flat(LH, AW, [&](int row, int col) {
        const float* lr = Ls + row * LW + col;
        const float* gr = Xs + row * LW + col;
        float s1 = 0.0f, s2 = 0.0f;
#pragma unroll
        for (int t = 0; t <= 2 * r; ++t) {
          s1 += lr[t];
          s2 += gr[t];
        }
        Hl[row * AW + col] = s1;
        Hg[row * AW + col] = s2;
    });
    __syncthreads();
    // Vertical sums: the window coefficients a = (mean(G l) - mu mean(l)) dinv and b = mean(l) - a mu, written
    // over the staged mu and dinv.
    flat(AH, AW, [&](int row, int col) {
        float s1 = 0.0f, s2 = 0.0f;
#pragma unroll
        for (int t = 0; t <= 2 * r; ++t) {
          s1 += Hl[(row + t) * AW + col];
          s2 += Hg[(row + t) * AW + col];
        }
        const int o = row * AW + col;
        const float mu = Aa[o], di = Ab[o];
        const float m1 = s1 * inv_nw, m2 = s2 * inv_nw;
        const float av = (m2 - mu * m1) * di;
        Aa[o] = av;
        Ab[o] = m1 - av * mu;
    });
    __syncthreads();
    // Horizontal sums of a and b (m-space columns).
    float* Ha = Hs;
    float* Hb = Hs + AH * W3;
    flat(AH, W3, [&](int row, int col) {
        const float* ar = Aa + row * AW + col;
        const float* br = Ab + row * AW + col;
        float s1 = 0.0f, s2 = 0.0f;
#pragma unroll
        for (int t = 0; t <= 2 * r; ++t) {
          s1 += ar[t];
          s2 += br[t];
        }
        Ha[row * W3 + col] = s1;
        Hb[row * W3 + col] = s2;
    });
    __syncthreads();
    // M l = |w| l - G S(a) - S(b) on m-space [i0-RF, i0+TH+RF) x [j0-RF, j0+TW+RF).
    float* Ml = Xs;
    flat(MH, W3, [&](int row, int col) {
        float sa = 0.0f, sb = 0.0f;
#pragma unroll
        for (int t = 0; t <= 2 * r; ++t) {
          sa += Ha[(row + t) * W3 + col];
          sb += Hb[(row + t) * W3 + col];
        }
        const int lo = (row + 2 * r) * LW + col + 2 * r;
        Ml[row * W3 + col] = nwf * Ls[lo] - Gs[lo] * sa - sb;
    });
    __syncthreads();
    // Q += lambda F^T (M l): (F^T m)(x) = sum_{a,b} f[a][b] m(x + (a-RF, b-RF)).
    for (int row = wave; row < TH; row += kPW) {
      for (int col = lane; col < TW; col += 64) {
        const float* mb = Ml + row * W3 + col;
        float s = 0.0f;
        if (FT > 0) {
#pragma unroll
          for (int a = 0; a < (FT > 0 ? FT : 1); ++a)
#pragma unroll
            for (int b = 0; b < (FT > 0 ? FT : 1); ++b) s = fmaf(tp[a * FT + b], mb[a * W3 + b], s);
        } else {
          for (int a = 0; a < F; ++a) {
            const float* mr = mb + a * W3;
            const float* fr = Ts + a * F;
            for (int b = 0; b < F; ++b) s = fmaf(fr[b], mr[b], s);
          }
        }
        Q[row * TW + col] = fmaf(g.lam, s, Q[row * TW + col]);
      }
    }
    __syncthreads();
  }

  // B^T D^T y: q[i][j] += sum over taps (a, b) with i + a - R = C m and j + b - R = C k of u[a][b] y[m][k];
  // then write q and the partials.
  double v[3] = {0.0, 0.0, 0.0};
  float* qc = A.q + (size_t)ch * HW;
  for (int row = wave; row < TH; row += kPW) {
    const int i = i0 + row;
    if (i >= H) break;
    const int a0 = pos_mod(R - i, C), m0 = (i + a0 - R) / C - mlo;
    for (int col = lane; col < TW; col += 64) {
      const int j = j0 + col;
      if (j >= W) break;
      const int b0 = pos_mod(R - j, C), k0 = (j + b0 - R) / C - klo;
      float qd = 0.0f;
      for (int a = a0, m = m0; a < n; a += C, ++m) {
        const float* yrow = Ys + m * YW + k0;
        const float* urow = Us + a * n;
        for (int b = b0, k = 0; b < n; b += C, ++k) qd = fmaf(urow[b], yrow[k], qd);
      }
      const float qv = Q[row * TW + col] + qd;
      const size_t o = (size_t)i * W + j;
      qc[o] = qv;
      if (A.mode == 1) {
        v[0] += (double)P[(row + E) * PW + col + E] * qv;
        v[1] += (double)Rs[row * TW + col] * qv;
        v[2] += (double)qv * qv;
      }
    }
  }
  if (A.mode == 0) return;
  block_partials<3, kPW>(v, red, A.partials + (size_t)ch * A.pstride * 3 + (size_t)tile * 3);
}

// r = b - q (float32) and the partials of |r|^2, for the bands whose check is pending (all bands if !only_pending).
__global__ __launch_bounds__(kBlock) void k_prior_resid(Geom g, const float* __restrict__ b,
                                                        const float* __restrict__ q, float* __restrict__ r,
                                                        const ChanState* __restrict__ st, int only_pending,
                                                        double* __restrict__ partials, int pstride) {
  __shared__ double red[kWaves];
  const int ch = blockIdx.y;
  if (only_pending && !st[ch].pending) return;
  const size_t HW = (size_t)g.H * g.W, base = (size_t)ch * HW;
  const size_t e0 = (size_t)blockIdx.x * kPriorFlat;
  const size_t e1 = e0 + kPriorFlat < HW ? e0 + kPriorFlat : HW;
  double acc = 0.0;
  for (size_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
    const float rv = b[base + e] - q[base + e];
    if (r) r[base + e] = rv;
    acc += (double)rv * rv;
  }
  double v[1] = {acc};
  block_partials<1>(v, red, partials + (size_t)ch * pstride * 3 + blockIdx.x);
}

// The check of a pending band: its true residual |b - A x|^2 (summed partials) against the tolerance.  Passes:
// the band stops (status 0); fails at the iteration cap: stops not converged; fails otherwise: CG restarts from
// that residual (restart[ch] = 1, the caller sets p = r).  rho takes the true residual either way.
__global__ __launch_bounds__(kBlock) void k_prior_verify(const double* __restrict__ partials, int pstride, int nblk,
                                                         ChanState* __restrict__ st, int* __restrict__ restart,
                                                         int max_iters, float tol) {
  __shared__ double red[kWaves];
  const int ch = blockIdx.x;
  ChanState& c = st[ch];
  if (!c.pending) {
    if (threadIdx.x == 0) restart[ch] = 0;
    return;
  }
  double s[1] = {0.0};
  for (int i = threadIdx.x; i < nblk; i += kBlock) s[0] += partials[(size_t)ch * pstride * 3 + i];
  block_sums<1>(s, red);
  if (threadIdx.x != 0) return;
  const double rr = s[0];
  int again = 0;
  c.pending = 0;
  c.rho = rr;
  if (!isfinite(rr)) {
    c.status = -6;
    c.active = 0;
  } else if (sqrt(rr) <= (double)tol * sqrt(c.bnorm2)) {
    c.status = 0;
  } else if (c.iters >= max_iters) {
    c.status = 1;
  } else {
    c.active = 1;
    again = 1;
  }
  restart[ch] = again;
}

__global__ __launch_bounds__(kBlock) void k_prior_restart(Geom g, const float* __restrict__ r, float* __restrict__ p,
                                                          const int* __restrict__ restart) {
  const int ch = blockIdx.y;
  if (!restart[ch]) return;
  const size_t HW = (size_t)g.H * g.W, base = (size_t)ch * HW;
  const size_t e0 = (size_t)blockIdx.x * kPriorFlat;
  const size_t e1 = e0 + kPriorFlat < HW ? e0 + kPriorFlat : HW;
  for (size_t e = e0 + threadIdx.x; e < e1; e += kBlock) p[base + e] = r[base + e];
}

namespace host {

namespace {

int prior_filters(int kind, int n, int F[2]) {
  switch (kind) {
    case LLP_PRIOR_LLP: F[0] = 3; return 1;
    case LLP_PRIOR_LGC: F[0] = F[1] = 3; return 2;
    case LLP_PRIOR_LPP: F[0] = 1; return 1;
    case LLP_PRIOR_LPF:
    case LLP_PRIOR_HPF: F[0] = n; return 1;
    default: return 0;
  }
}

// LDS layout of k_prior_apply for the largest filter half-width RF and window radius r (floats).
size_t prior_layout(const Geom& g, int RF, PriorArgs* A) {
  const int TH = prior_th(g.c), TW = kPriorTW, r = g.r;
  const int E = 2 * RF + 2 * r;
  const size_t PH = TH + 2 * E, PW = TW + 2 * E;
  const size_t LH = TH + 2 * (RF + 2 * r), LW = TW + 2 * (RF + 2 * r);
  const size_t AH = TH + 2 * (RF + r), AW = TW + 2 * (RF + r);
  const size_t YH = (TH - 1 + 2 * g.R) / g.c + 2, YW = (TW - 1 + 2 * g.R) / g.c + 2;
  const size_t F = 2 * RF + 1;
  size_t off = PH * PW;
  A->E = E;
  A->TH = TH;
  A->offL = (int)off;
  off += LH * LW;
  A->offX = (int)off;
  off += LH * LW;
  A->offG = (int)off;
  off += LH * LW;
  A->offH = (int)off;
  off += 2 * LH * AW;
  A->offA = (int)off;
  off += 2 * AH * AW;
  A->offQ = (int)off;
  off += (size_t)TH * TW;
  A->offY = (int)off;
  off += YH * YW;
  A->offT = (int)off;
  off += F * F;
  A->offU = (int)off;
  off += (size_t)g.n * g.n;
  A->offR = (int)off;
  off += (size_t)TH * TW;
  A->YW = (int)YW;
  return off;
}

template <int FT>
const void* prior_kernel_r(int RW) {
  return RW == 1 ? (const void*)k_prior_apply<FT, 1> : RW == 2 ? (const void*)k_prior_apply<FT, 2>
                                                                : (const void*)k_prior_apply<FT, 0>;
}
const void* prior_kernel(int FT, int RW) {
  return FT == 1 ? prior_kernel_r<1>(RW) : FT == 3 ? prior_kernel_r<3>(RW) : prior_kernel_r<0>(RW);
}

struct PriorWs {
  float* stats;   // [2][3][H][W]: G, MU, DI of each filter
  double* g64;    // [H][W]
  float* taps;    // [2][kPriorTapStride]
  int* restart;   // [N]
};

llp_status prior_workspace(llp_ctx* ctx, const Geom& g, PriorWs* w) {
  const size_t HW = (size_t)g.H * g.W;
  size_t off = 0;
  const size_t o_stats = off;
  off = align_up(off + 6 * HW * sizeof(float), 256);
  const size_t o_g64 = off;
  off = align_up(off + HW * sizeof(double), 256);
  const size_t o_taps = off;
  off = align_up(off + 2 * kPriorTapStride * sizeof(float), 256);
  const size_t o_restart = off;
  off = align_up(off + (size_t)g.N * sizeof(int), 256);
  if (off > ctx->prior_bytes) {
    if (ctx->prior_ws) {
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(ctx->prior_ws));
      ctx->prior_ws = nullptr;
      ctx->prior_bytes = 0;
    }
    if (hipMalloc(&ctx->prior_ws, off) != hipSuccess) {
      ctx->prior_ws = nullptr;
      return LLP_E_OOM;
    }
    ctx->prior_bytes = off;
  }
  char* base = (char*)ctx->prior_ws;
  w->stats = (float*)(base + o_stats);
  w->g64 = (double*)(base + o_g64);
  w->taps = (float*)(base + o_taps);
  w->restart = (int*)(base + o_restart);
  return LLP_OK;
}

// Validation and set-up shared by the solve and the operator hook: the filters, the guides and their window
// statistics, and the operator's launch arguments (all but the vectors).
llp_status prior_setup(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, int kind, const float* pan,
                       const float* kernel, Geom* gout, PriorArgs* A, size_t* lds_bytes, hipStream_t s) {
  if (!ctx || !params || !pan || !kernel) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, params, &g);
  if (v != LLP_OK) return v;
  if (kind < LLP_PRIOR_LLP || kind > LLP_PRIOR_HPF) return LLP_E_ARG;
  memset(A, 0, sizeof(*A));
  A->nf = prior_filters(kind, g.n, A->F);
  if (A->F[0] > kPriorMaxSide || A->F[0] > g.H || A->F[0] > g.W) return LLP_E_UNSUPPORTED;
  const int RF = (A->F[0] - 1) / 2;
  const size_t lds = prior_layout(g, RF, A) * sizeof(float);
  if (lds + 512 > (size_t)kMaxLdsFloats * sizeof(float)) return LLP_E_UNSUPPORTED;  // 512 B: static LDS
  A->tiles_x = (g.W + kPriorTW - 1) / kPriorTW;
  A->ntiles = ((g.H + A->TH - 1) / A->TH) * A->tiles_x;
  A->pstride = (int)max_partials_per_band(g);
  if ((size_t)A->ntiles > (size_t)A->pstride) return LLP_E_UNSUPPORTED;
  HIP_TRY(hipSetDevice(ctx->device));
  v = ensure_workspace(ctx, g);
  if (v != LLP_OK) return v;
  PriorWs w;
  v = prior_workspace(ctx, g, &w);
  if (v != LLP_OK) return v;
  const size_t HW = (size_t)g.H * g.W;
  hipLaunchKernelGGL(k_prior_taps, dim3(1), dim3(kBlock), 0, s, kind, kernel, g.n, w.taps);
  HIP_TRY(hipGetLastError());
  const unsigned nb = (unsigned)((HW + kBlock - 1) / kBlock);
  for (int d = 0; d < A->nf; ++d) {
    float* G = w.stats + (size_t)d * 3 * HW;
    hipLaunchKernelGGL(k_prior_guide, dim3(nb), dim3(kBlock), 0, s, g, pan, w.taps + d * kPriorTapStride, A->F[d],
                       w.g64, G);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_prior_wstats, dim3(nb), dim3(kBlock), 0, s, g, w.g64, G + HW, G + 2 * HW);
    HIP_TRY(hipGetLastError());
    A->G[d] = G;
    A->MU[d] = G + HW;
    A->DI[d] = G + 2 * HW;
  }
  A->taps = w.taps;
  A->partials = ctx->partials;
  A->st = ctx->st;
  // the LDS this geometry needs (the attribute may not exceed the CU's LDS less the kernel's static part)
  A->FT = A->F[0] == 1 ? 1 : (A->F[0] == 3 ? 3 : 0);  // every filter of a prior has the same side
  A->RW = (g.r == 1 || g.r == 2) ? g.r : 0;
  HIP_TRY(hipFuncSetAttribute(prior_kernel(A->FT, A->RW), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  *gout = g;
  *lds_bytes = lds;
  return LLP_OK;
}

hipError_t launch_prior_apply(const Geom& g, PriorArgs A, size_t lds, int mode, const float* p, const float* r,
                              const float* y, const float* u, float* q, hipStream_t s) {
  A.mode = mode;
  A.p = p;
  A.r = r;
  A.y = y;
  A.q = q;
  const dim3 grid((unsigned)(A.ntiles * g.N));
  void* args[] = {(void*)&g, (void*)&A, (void*)&u};
  return hipLaunchKernel(prior_kernel(A.FT, A.RW), grid, dim3(kPB), args, lds, s);
}

int flat_blocks(const Geom& g) { return (int)(((size_t)g.H * g.W + kPriorFlat - 1) / kPriorFlat); }

}  // namespace

}  // namespace host
}  // namespace llp

using namespace llp;
using namespace llp::host;

extern "C" {

llp_status llp_apply_prior(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, int prior,
                           const float* pan, const float* kernel, const float* z, float* out, int data_term,
                           hipStream_t stream) {
  if (!z || !out || z == out) return LLP_E_ARG;
  Geom g;
  PriorArgs A;
  size_t lds = 0;
  llp_status v = prior_setup(ctx, shape, params, prior, pan, kernel, &g, &A, &lds, stream);
  if (v != LLP_OK) return v;
  if (data_term) {
    OpConfig cfg;
    if (!ctx_config(ctx, g, &cfg)) return LLP_E_UNSUPPORTED;
    HIP_TRY(launch_dir(g, cfg, 0, 0, 0, z, nullptr, nullptr, nullptr, nullptr, nullptr, ctx->y, kernel,
                       ctx->partials, ctx->st, 0, 0.0f, stream));
  } else {  // y = 0: the B^T D^T y part is then exactly 0
    HIP_TRY(hipMemsetAsync(ctx->y, 0, (size_t)g.N * g.h * g.w * sizeof(float), stream));
  }
  HIP_TRY(launch_prior_apply(g, A, lds, 0, z, nullptr, ctx->y, kernel, out, stream));
  return LLP_OK;
}

llp_status llp_prior_pansharpen(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, int prior,
                                const float* lrms, const float* pan, const float* kernel, const float* init,
                                float* hrms, llp_report* rep, hipStream_t stream) {
  if (!lrms || !hrms || !params) return LLP_E_ARG;
  if (params->precond != 0 || params->init_mode < 0 || params->init_mode > 1) return LLP_E_UNSUPPORTED;
  if (params->init_mode == 1 && !init) return LLP_E_ARG;
  hipStream_t s = stream;
  Geom g;
  PriorArgs A;
  size_t lds = 0;
  llp_status v = prior_setup(ctx, shape, params, prior, pan, kernel, &g, &A, &lds, s);
  if (v != LLP_OK) return v;
  OpConfig cfg;
  if (!ctx_config(ctx, g, &cfg)) return LLP_E_UNSUPPORTED;
  PriorWs w;
  v = prior_workspace(ctx, g, &w);
  if (v != LLP_OK) return v;
  v = check_inputs(ctx, g, lrms, pan, kernel, s);
  if (v != LLP_OK) return v;
  const size_t NHW = (size_t)g.N * g.H * g.W;
  const int max_iters = params->max_iters;
  const float tol = params->tol;
  const int pstride = (int)max_partials_per_band(g);
  const int nflat = flat_blocks(g);
  const dim3 flat_grid((unsigned)nflat, (unsigned)g.N);

  HIP_TRY(launch_rhs(g, lrms, kernel, ctx->b, ctx->partials, ctx->st, s));
  const int from_init = params->init_mode == 1;
  if (from_init) {
    if (init != hrms) HIP_TRY(hipMemcpyAsync(hrms, init, NHW * sizeof(float), hipMemcpyDeviceToDevice, s));
  } else {
    HIP_TRY(hipMemsetAsync(hrms, 0, NHW * sizeof(float), s));
  }
  HIP_TRY(launch_init(g, from_init, ctx->b, ctx->r[0], ctx->st, s));
  if (from_init) {  // r_0 = b - A x_0
    HIP_TRY(launch_dir(g, cfg, 0, 0, 0, hrms, nullptr, nullptr, nullptr, nullptr, nullptr, ctx->y, kernel,
                       ctx->partials, ctx->st, 0, 0.0f, s));
    HIP_TRY(launch_prior_apply(g, A, lds, 0, hrms, nullptr, ctx->y, kernel, ctx->q, s));
    hipLaunchKernelGGL(k_prior_resid, flat_grid, dim3(kBlock), 0, s, g, ctx->b, ctx->q, ctx->r[0], ctx->st, 0,
                       ctx->partials, pstride);
    HIP_TRY(hipGetLastError());
  }
  // p_0 = r_0, y = D B p_0, rho_0 and the stopping rule at x_0
  HIP_TRY(launch_dir(g, cfg, 1, 0, 0, ctx->r[0], nullptr, nullptr, nullptr, ctx->p[0], hrms, ctx->y, kernel,
                     ctx->partials, ctx->st, max_iters, tol, s));
  HIP_TRY(launch_finalize(g, kFinDir, ctx->partials, dir_ntiles(g, cfg), ctx->st, nullptr, 0, 0, max_iters, tol,
                          s));
  const bool tol_mode = tol > 0.0f;
  // The check of bands whose recursive residual met the tolerance: r = b - A x into the buffers of parity `cur`,
  // decision, p = r for the bands that restart, and y = D B p again (the check used y for D B x).
  auto check = [&](int cur) -> llp_status {
    HIP_TRY(launch_dir(g, cfg, 0, 0, 0, hrms, nullptr, nullptr, nullptr, nullptr, nullptr, ctx->y, kernel,
                       ctx->partials, ctx->st, 0, 0.0f, s));
    HIP_TRY(launch_prior_apply(g, A, lds, 0, hrms, nullptr, ctx->y, kernel, ctx->q, s));
    hipLaunchKernelGGL(k_prior_resid, flat_grid, dim3(kBlock), 0, s, g, ctx->b, ctx->q, ctx->r[cur], ctx->st, 1,
                       ctx->partials, pstride);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_prior_verify, dim3(g.N), dim3(kBlock), 0, s, ctx->partials, pstride, nflat, ctx->st,
                       w.restart, max_iters, tol);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_prior_restart, flat_grid, dim3(kBlock), 0, s, g, ctx->r[cur], ctx->p[cur], w.restart);
    HIP_TRY(hipGetLastError());
    HIP_TRY(launch_dir(g, cfg, 0, 0, 0, ctx->p[cur], nullptr, nullptr, nullptr, nullptr, nullptr, ctx->y, kernel,
                       ctx->partials, ctx->st, 0, 0.0f, s));
    return LLP_OK;
  };
  const int nb_dir = dir_ntiles(g, cfg);
  int k = 1;
  if (tol_mode) {
    HIP_TRY(hipMemcpyAsync(ctx->h_st, ctx->st, sizeof(ChanState) * g.N, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    bool pend = false;
    for (int i = 0; i < g.N; ++i) pend |= ctx->h_st[i].pending != 0;
    if (pend) {
      v = check(0);
      if (v != LLP_OK) return v;
    }
  }
  while (k <= max_iters) {
    const int todo = std::min(max_iters - k + 1, 2 * kCheckEvery);
    for (int t = 0; t < todo; ++t, ++k) {
      const int prev = (k - 1) & 1, cur = k & 1;
      int tp = timing_begin(ctx, s);
      HIP_TRY(launch_prior_apply(g, A, lds, 1, ctx->p[prev], ctx->r[prev], ctx->y, kernel, ctx->q, s));
      timing_end(ctx, s, tp, kTApply);
      HIP_TRY(launch_finalize(g, kFinApply, ctx->partials, A.ntiles, ctx->st, nullptr, 0, 0, 0, 0.0f, s));
      tp = timing_begin(ctx, s);
      HIP_TRY(launch_dir(g, cfg, 2, k == max_iters, k, ctx->r[prev], ctx->q, ctx->p[prev], ctx->r[cur],
                         ctx->p[cur], hrms, ctx->y, kernel, ctx->partials, ctx->st, max_iters, tol, s));
      timing_end(ctx, s, tp, kTDir);
      HIP_TRY(launch_finalize(g, kFinDir, ctx->partials, nb_dir, ctx->st, nullptr, 0, -1, max_iters, tol, s));
    }
    if (!tol_mode) continue;
    HIP_TRY(hipMemcpyAsync(ctx->h_st, ctx->st, sizeof(ChanState) * g.N, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    bool any_active = false, pend = false;
    for (int i = 0; i < g.N; ++i) {
      any_active |= ctx->h_st[i].active != 0;
      pend |= ctx->h_st[i].pending != 0;
    }
    if (pend) {
      v = check((k - 1) & 1);
      if (v != LLP_OK) return v;
      HIP_TRY(hipMemcpyAsync(ctx->h_st, ctx->st, sizeof(ChanState) * g.N, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      any_active = false;
      for (int i = 0; i < g.N; ++i) any_active |= ctx->h_st[i].active != 0;
    }
    if (!any_active) break;
  }
  // Report: the true residual of the returned iterate (float32 operator, FP64 sum).
  if (rep) {
    HIP_TRY(launch_dir(g, cfg, 0, 0, 0, hrms, nullptr, nullptr, nullptr, nullptr, nullptr, ctx->y, kernel,
                       ctx->partials, ctx->st, 0, 0.0f, s));
    HIP_TRY(launch_prior_apply(g, A, lds, 0, hrms, nullptr, ctx->y, kernel, ctx->q, s));
    HIP_TRY(launch_residual_norm(g, ctx->b, ctx->q, ctx->partials, ctx->st, ctx->results, s));
    HIP_TRY(hipMemcpyAsync(ctx->h_results, ctx->results, sizeof(double) * kResultSlots * g.N,
                           hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipMemcpyAsync(ctx->h_st, ctx->st, sizeof(ChanState) * g.N, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(ctx->h_flags, ctx->flags, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (ctx->profiling) {
    v = collect_times(ctx);
    if (v != LLP_OK) return v;
  }
  if (ctx->h_flags[0]) return LLP_E_NONFINITE;
  llp_status worst = LLP_OK;
  for (int i = 0; i < g.N; ++i) {
    const ChanState& cs = ctx->h_st[i];
    const int st = (cs.active || cs.pending) ? (tol_mode ? LLP_NOT_CONVERGED : LLP_OK) : cs.status;
    if (st < 0 && (worst >= 0 || st < worst)) worst = (llp_status)st;
    if (st > 0 && worst == LLP_OK) worst = (llp_status)st;
    if (rep) {
      llp_report& R = rep[i];
      R.iters = cs.iters;
      R.init = from_init ? 1 : 0;
      R.status = st;
      const double bn2 = cs.bnorm2;
      R.rel_residual = bn2 > 0 ? sqrt(cs.rho / bn2) : sqrt(cs.rho);
      const double tr = ctx->h_results[i * kResultSlots + kSlotTrueRes];
      R.true_rel_residual = bn2 > 0 ? sqrt(tr / bn2) : sqrt(tr);
      R.out_rel_residual = R.true_rel_residual;
      R.objective = NAN;
    }
  }
  return worst;
}

}  // extern "C"
