// Residual replacement for the conjugate-gradient solve of eq. (Z_ini_matting) (Sec. III-B): the "reliable
// updates" of van der Vorst and Ye applied to the float32 iteration.
//
// The iterate is held in two parts: an FP64 accumulator xacc and a float32 part z that the iteration kernels
// advance (z += alpha p).  Every kRepEvery iterations, and whenever a band's recursive residual meets the
// tolerance, a replacement pass flushes z into xacc (z = 0) and recomputes the band's residual as
// r = b - A xacc with every operation in FP64: D B x on the low-resolution lattice, then per HR tile
// B^T D^T (D B x) + lambda L^T M_LY L x with the PAN statistics of eq. (matting_matrix) recomputed in FP64 from
// the PAN image inside the tile.  The recomputed residual replaces the recursive one (the direction is kept),
// so the recursion's drift from b - A x is reset, and a band stops only when the residual of its FP64 iterate
// meets the tolerance.
//
// The operator is the one the oracle defines; the float32 kernels of the iteration are not used here.  Every
// reduction is two-step and deterministic (per-tile partials, summed in a fixed order by one workgroup per band).
#include "llp_device.h"

#include <math.h>

namespace llp {
using namespace dev;

namespace {

constexpr int kChunkE = kBlock * 16;  // elements per workgroup in the elementwise launch
constexpr int kYRows = 4;             // D B x: LR rows per tile (one wave each), 64 LR columns per tile
constexpr int kResTW = 64;            // residual tile: HR columns
constexpr int kResThreads = 1024;     // residual tile: threads (one workgroup per CU: its LDS; 16 waves hide it)


__device__ __forceinline__ int wrapr(int i, int n) {
  if (i >= -n && i < 2 * n) return i < 0 ? i + n : (i >= n ? i - n : i);
  const int m = i % n;
  return m < 0 ? m + n : m;
}

// force 1: every band; 0: the pending bands and those kRepEvery iterations past their last replacement; 2: the
// bands whose FP64 residual in the results is not that of their current iterate.
__device__ __forceinline__ bool rep_selected(const ChanState& c, int force) {
  if (force == 2) return c.ref_iter != c.iters;
  return force || c.pending || (c.active && c.iters - c.last_rep >= kRepEvery);
}

// Whether any band of the table is selected (every thread of the block gets the answer): a pass that selects
// none returns at once instead of striding over every tile.  One LDS word, so that the tiled launches keep their
// dynamic LDS limit.
__device__ __forceinline__ bool any_selected(const RefDesc* t, int count, const ChanState* st, int force) {
  __shared__ int flag;
  const int nb = t[count - 1].band0 + t[count - 1].g.N;
  if (threadIdx.x == 0) flag = 0;
  __syncthreads();
  bool mine = false;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) mine = mine || rep_selected(st[b], force);
  if (mine) flag = 1;
  __syncthreads();
  return flag != 0;
}

// Scene of workgroup `bid` in a table ordered by block offsets: the last entry whose offset <= bid.
template <typename F>
__device__ __forceinline__ int find_scene(const RefDesc* t, int count, int bid, F first) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first(t[mid]) <= bid) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__host__ __device__ __forceinline__ int res_tiles_x(const Geom& g) { return (g.W + kResTW - 1) / kResTW; }
__host__ __device__ __forceinline__ int y_tiles_x(const Geom& g) { return (g.w + 63) / 64; }
__host__ __device__ __forceinline__ int y_tiles(const Geom& g) { return ((g.h + kYRows - 1) / kYRows) * y_tiles_x(g); }
__host__ __device__ __forceinline__ int lr_span(int t, int R, int c) { return (t - 1 + 2 * R) / c + 2; }

}  // namespace

// ------------------------------------------------------------------------------------------- elementwise ---

__device__ __forceinline__ void ref_elem_block(int op, const RefDesc* __restrict__ t, int count,
                                               const ChanState* __restrict__ st, int force, int vb) {
  const int si = find_scene(t, count, vb, [](const RefDesc& d) { return d.e_block0; });
  const RefDesc& d = t[si];
  const Geom& g = d.g;
  const size_t HW = (size_t)g.H * g.W;
  const int per_band = (int)((HW + kChunkE - 1) / kChunkE);
  const int local = vb - d.e_block0;
  if (local >= per_band * g.N) return;
  const int ch = local / per_band, blk = local - ch * per_band;
  if (op == kRefFlush && !rep_selected(st[d.band0 + ch], force)) return;
  const size_t base = (size_t)ch * HW;
  const size_t e0 = (size_t)blk * kChunkE;
  const size_t e1 = e0 + kChunkE < HW ? e0 + kChunkE : HW;
  float* z = d.z + base;
  double* x = d.xacc + base;
  for (size_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
    switch (op) {
      case kRefFlush: x[e] += (double)z[e]; z[e] = 0.0f; break;
      case kRefStartZero: x[e] = 0.0; z[e] = 0.0f; break;
      case kRefStartFrom: x[e] = (double)z[e]; z[e] = 0.0f; break;
      case kRefOutput: z[e] = (float)(x[e] + (double)z[e]); break;
      default: {  // kRefOutputBack
        const float o = (float)(x[e] + (double)z[e]);
        z[e] = o;
        x[e] = (double)o;
      }
    }
  }
}

// The launches below run a bounded grid that strides over the virtual blocks of every scene and band: a pass
// in which no band is selected costs a few state reads per workgroup, whatever the image sizes.
__global__ __launch_bounds__(kBlock) void k_ref_elem(int op, const RefDesc* __restrict__ t, int count, int total,
                                                     const ChanState* __restrict__ st, int force) {
  if (op == kRefFlush && !any_selected(t, count, st, force)) return;
  for (int vb = blockIdx.x; vb < total; vb += gridDim.x) ref_elem_block(op, t, count, st, force, vb);
}

// ------------------------------------------------------------------------------------------- D B x (FP64) ---
// y[m][k] = sum_{a,b} u[a][b] x[c m + R - a][c k + R - b] (true convolution, then decimation at phase 0).
// One workgroup per band and tile of kYRows x 64 LR points; the x region the taps reach is staged in LDS.

__device__ __forceinline__ void ref_y_block(const RefDesc* __restrict__ t, int count,
                                            const ChanState* __restrict__ st, int force, int vb, double* ysh) {
  const int si = find_scene(t, count, vb, [](const RefDesc& d) { return d.y_block0; });
  const RefDesc& d = t[si];
  const Geom& g = d.g;
  const int nt = y_tiles(g);
  const int local = vb - d.y_block0;
  if (local >= nt * g.N) return;
  const int ch = local / nt, tile = local - ch * nt;
  if (!rep_selected(st[d.band0 + ch], force)) return;
  const int c = g.c, n = g.n, R = g.R, H = g.H, W = g.W;
  const int tx = y_tiles_x(g);
  const int m0 = (tile / tx) * kYRows, k0 = (tile % tx) * 64;
  const int RH = (kYRows - 1) * c + 2 * R + 1, RW = 63 * c + 2 * R + 1;
  double* xs = ysh;
  double* us = ysh + RH * RW;
  const double* xb = d.xacc + (size_t)ch * H * W;
  const int row0 = c * m0 - R, col0 = c * k0 - R;
  for (int idx = threadIdx.x; idx < RH * RW; idx += kBlock) {
    const int li = idx / RW, lj = idx - li * RW;
    xs[idx] = xb[(size_t)wrapr(row0 + li, H) * W + wrapr(col0 + lj, W)];
  }
  for (int idx = threadIdx.x; idx < n * n; idx += kBlock) us[idx] = (double)d.u[idx];
  __syncthreads();
  const int ml = threadIdx.x >> 6, kl = threadIdx.x & 63;
  const int m = m0 + ml, k = k0 + kl;
  if (m >= g.h || k >= g.w) return;
  double s = 0.0;
  for (int a = 0; a < n; ++a) {
    const double* xr = xs + (c * ml + 2 * R - a) * RW + c * kl + 2 * R;  // row c m + R - a, column c k + R
    const double* ur = us + a * n;
    for (int b = 0; b < n; ++b) s = fma(ur[b], xr[-b], s);
  }
  d.y64[((size_t)ch * g.h + m) * g.w + k] = s;
}

__global__ __launch_bounds__(kBlock) void k_ref_y(const RefDesc* __restrict__ t, int count, int total,
                                                  const ChanState* __restrict__ st, int force) {
  extern __shared__ double ysh[];
  if (!any_selected(t, count, st, force)) return;
  for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
    ref_y_block(t, count, st, force, vb, ysh);
    __syncthreads();  // the next block's staging overwrites the region
  }
}

// ------------------------------------------------------------------------------------ residual tile (FP64) ---
// r = b - (B^T D^T y + lambda L M L x) on a tile of TH x kResTW pixels, for every selected band of the scene:
// M l = |w| l - G (.) S(a) - S(b), a = (S(G l)/|w| - mu S(l)/|w|) dinv, b = S(l)/|w| - a mu (S the periodic
// (2r+1)^2 window sum), with G = L Y, mu = S(G)/|w|, var = S(G^2)/|w| - mu^2 and dinv = 1/(eps/|w| + var) (0 where
// that is 0) computed once per tile in FP64 from the float32 PAN image.  Window sums are separable: a
// horizontal pass into row sums, then a vertical pass.  Regions, as offsets from the tile's corner:
//   X (x and Y):    halo E = 2r + 2     L (G, l = L x, G l): halo 2r + 1
//   A (a, b):       halo r + 1          M (M l):             halo 1
// and the LR samples of y the tile's B^T D^T taps reach.

namespace {
struct ResLayout {  // LDS layout of the residual tile (doubles; Ys in floats at the end)
  int TH, E, XH, XW, LH, LW, AH, AW, MH, MW, YH, YW;
  int oG, oMU, oDI, oR0, oL, oR1, oB, oYl, oU, oYs, total_doubles;
  __host__ __device__ ResLayout(const Geom& g, int th) {
    const int r = g.r;
    TH = th;
    E = 2 * r + 2;
    XH = TH + 2 * E, XW = kResTW + 2 * E;
    LH = TH + 2 * (2 * r + 1), LW = kResTW + 2 * (2 * r + 1);
    AH = TH + 2 * (r + 1), AW = kResTW + 2 * (r + 1);
    MH = TH + 2, MW = kResTW + 2;
    YH = lr_span(TH, g.R, g.c), YW = lr_span(kResTW, g.R, g.c);
    const int R1 = 2 * (LH * AW > AH * MW ? LH * AW : AH * MW);
    oG = 0;                       // G (L region), kept for all bands
    oMU = oG + LH * LW;           // mu, dinv (A region), kept for all bands
    oDI = oMU + AH * AW;
    oR0 = oDI + AH * AW;          // x (X region), then a (A region), then M l (M region)
    oL = oR0 + XH * XW;           // l = L x (L region)
    oR1 = oL + LH * LW;           // row sums: (G, G^2) or (l, G l) over L rows x A columns; (a, b) over A rows x M columns
    oB = oR1 + R1;                // b (A region)
    oYl = oB + AH * AW;           // y (LR samples)
    oU = oYl + YH * YW;           // taps
    oYs = oU + g.n * g.n;         // PAN (X region), floats
    total_doubles = oYs + (XH * XW + 1) / 2;
  }
};

// Residual tile height: 16 rows, or 8 or 4 where the FP64 regions of a taller tile do not fit in LDS.
__host__ __device__ __forceinline__ int res_th(const Geom& g) {
  for (int th = 16; th > 4; th /= 2)
    if ((size_t)ResLayout(g, th).total_doubles * sizeof(double) <= kRefMaxLds) return th;
  return 4;
}
__host__ __device__ __forceinline__ ResLayout res_layout(const Geom& g) { return ResLayout(g, res_th(g)); }
__host__ __device__ __forceinline__ int res_tiles(const Geom& g) {
  return ((g.H + res_th(g) - 1) / res_th(g)) * res_tiles_x(g);
}
}  // namespace

__device__ __forceinline__ void ref_res_block(const RefDesc* __restrict__ t, int count,
                                              const ChanState* __restrict__ st, int force, int rpar, int write_r,
                                              int vb, double* rsh, double* red) {
  const int si = find_scene(t, count, vb, [](const RefDesc& d) { return d.r_block0; });
  const RefDesc& d = t[si];
  const Geom& g = d.g;
  const int nt = res_tiles(g);
  const int tile = vb - d.r_block0;
  if (tile >= nt) return;
  bool any = false;
  for (int ch = 0; ch < g.N; ++ch) any |= rep_selected(st[d.band0 + ch], force);
  if (!any) return;
  const ResLayout Lo = res_layout(g);
  const int TH = Lo.TH, XH = Lo.XH, XW = Lo.XW, LH = Lo.LH, LW = Lo.LW, AH = Lo.AH, AW = Lo.AW, MH = Lo.MH,
            MW = Lo.MW, YH = Lo.YH, YW = Lo.YW, E = Lo.E;
  const int H = g.H, W = g.W, r = g.r, c = g.c, n = g.n, R = g.R, K = 2 * r + 1;
  const int tx = res_tiles_x(g);
  const int i0 = (tile / tx) * TH, j0 = (tile % tx) * kResTW;
  const int mlo = floor_div(i0 - R, c), klo = floor_div(j0 - R, c);
  double* Gs = rsh + Lo.oG;
  double* MUs = rsh + Lo.oMU;
  double* DIs = rsh + Lo.oDI;
  double* R0 = rsh + Lo.oR0;
  double* Ls = rsh + Lo.oL;
  double* R1 = rsh + Lo.oR1;
  double* Bs = rsh + Lo.oB;
  double* Yl = rsh + Lo.oYl;
  double* Us = rsh + Lo.oU;
  float* Ys = (float*)(rsh + Lo.oYs);
  const size_t HW = (size_t)H * W;
  const double nw = (double)(K * K), inv_nw = 1.0 / nw;
  const double epsw = (double)g.eps * inv_nw;

  // Once per tile: PAN, taps, G = L Y, and the window statistics mu, dinv.
  for (int idx = threadIdx.x; idx < XH * XW; idx += kResThreads) {
    const int li = idx / XW, lj = idx - li * XW;
    Ys[idx] = d.Y[(size_t)wrapr(i0 - E + li, H) * W + wrapr(j0 - E + lj, W)];
  }
  for (int idx = threadIdx.x; idx < n * n; idx += kResThreads) Us[idx] = (double)d.u[idx];
  __syncthreads();
  for (int idx = threadIdx.x; idx < LH * LW; idx += kResThreads) {
    const int li = idx / LW, lj = idx - li * LW;
    const int o = (li + 1) * XW + lj + 1;
    Gs[idx] = 4.0 * (double)Ys[o] - (double)Ys[o - XW] - (double)Ys[o + XW] - (double)Ys[o - 1] - (double)Ys[o + 1];
  }
  __syncthreads();
  double* hA = R1;
  double* hB = R1 + LH * AW;
  for (int idx = threadIdx.x; idx < LH * AW; idx += kResThreads) {  // row sums of G and G^2
    const int li = idx / AW, aj = idx - li * AW;
    const double* gr = Gs + li * LW + aj;
    double s1 = 0.0, s2 = 0.0;
    for (int dx = 0; dx < K; ++dx) {
      s1 += gr[dx];
      s2 += gr[dx] * gr[dx];
    }
    hA[idx] = s1;
    hB[idx] = s2;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < AH * AW; idx += kResThreads) {
    const int ai = idx / AW, aj = idx - ai * AW;
    double sg = 0.0, sg2 = 0.0;
    for (int dy = 0; dy < K; ++dy) {
      sg += hA[(ai + dy) * AW + aj];
      sg2 += hB[(ai + dy) * AW + aj];
    }
    const double mu = sg * inv_nw;
    const double den = epsw + (sg2 * inv_nw - mu * mu);
    MUs[idx] = mu;
    DIs[idx] = den != 0.0 ? 1.0 / den : 0.0;
  }
  __syncthreads();

  const double lam = (double)g.lam;
  for (int ch = 0; ch < g.N; ++ch) {
    const ChanState& cs = st[d.band0 + ch];
    if (!rep_selected(cs, force)) continue;  // uniform over the workgroup
    double* Xs = R0;
    const double* xb = d.xacc + (size_t)ch * HW;
    for (int idx = threadIdx.x; idx < XH * XW; idx += kResThreads) {
      const int li = idx / XW, lj = idx - li * XW;
      Xs[idx] = xb[(size_t)wrapr(i0 - E + li, H) * W + wrapr(j0 - E + lj, W)];
    }
    const double* yb = d.y64 + (size_t)ch * g.h * g.w;
    for (int idx = threadIdx.x; idx < YH * YW; idx += kResThreads) {
      const int li = idx / YW, lj = idx - li * YW;
      Yl[idx] = yb[(size_t)wrapr(mlo + li, g.h) * g.w + wrapr(klo + lj, g.w)];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < LH * LW; idx += kResThreads) {  // l = L x
      const int li = idx / LW, lj = idx - li * LW;
      const int o = (li + 1) * XW + lj + 1;
      Ls[idx] = 4.0 * Xs[o] - Xs[o - XW] - Xs[o + XW] - Xs[o - 1] - Xs[o + 1];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < LH * AW; idx += kResThreads) {  // row sums of l and G l
      const int li = idx / AW, aj = idx - li * AW;
      const double* lr = Ls + li * LW + aj;
      const double* gr = Gs + li * LW + aj;
      double s1 = 0.0, s2 = 0.0;
      for (int dx = 0; dx < K; ++dx) {
        s1 += lr[dx];
        s2 += gr[dx] * lr[dx];
      }
      hA[idx] = s1;
      hB[idx] = s2;
    }
    __syncthreads();
    double* As = R0;  // x is no longer needed
    for (int idx = threadIdx.x; idx < AH * AW; idx += kResThreads) {  // a, b of every window
      const int ai = idx / AW, aj = idx - ai * AW;
      double sl = 0.0, sgl = 0.0;
      for (int dy = 0; dy < K; ++dy) {
        sl += hA[(ai + dy) * AW + aj];
        sgl += hB[(ai + dy) * AW + aj];
      }
      const double mu = MUs[idx];
      const double m1 = sl * inv_nw, m2 = sgl * inv_nw;
      const double a = (m2 - mu * m1) * DIs[idx];
      As[idx] = a;
      Bs[idx] = m1 - a * mu;
    }
    __syncthreads();
    double* hA2 = R1;
    double* hB2 = R1 + AH * MW;
    for (int idx = threadIdx.x; idx < AH * MW; idx += kResThreads) {  // row sums of a and b
      const int ai = idx / MW, mj = idx - ai * MW;
      const double* ar = As + ai * AW + mj;
      const double* br = Bs + ai * AW + mj;
      double s1 = 0.0, s2 = 0.0;
      for (int dx = 0; dx < K; ++dx) {
        s1 += ar[dx];
        s2 += br[dx];
      }
      hA2[idx] = s1;
      hB2[idx] = s2;
    }
    __syncthreads();
    double* Ms = R0;  // a is no longer needed
    for (int idx = threadIdx.x; idx < MH * MW; idx += kResThreads) {  // M l = |w| l - G S(a) - S(b)
      const int mi = idx / MW, mj = idx - mi * MW;
      double sa = 0.0, sb = 0.0;
      for (int dy = 0; dy < K; ++dy) {
        sa += hA2[(mi + dy) * MW + mj];
        sb += hB2[(mi + dy) * MW + mj];
      }
      const int lo = (mi + 2 * r) * LW + mj + 2 * r;
      Ms[idx] = nw * Ls[lo] - Gs[lo] * sa - sb;
    }
    __syncthreads();
    // Tile: r = b - (B^T D^T y + lambda L (M l)).
    const float* bb = d.b + (size_t)ch * HW;
    const int bpar = cs.iters & 1;  // the buffers holding this band's r_k and p_k
    float* rout = d.r[rpar] + (size_t)ch * HW;
    const float* pin = d.p[bpar] + (size_t)ch * HW;
    float* pout = d.p[rpar] + (size_t)ch * HW;
    double acc = 0.0;
    for (int idx = threadIdx.x; idx < TH * kResTW; idx += kResThreads) {
      const int pi = idx / kResTW, pj = idx - pi * kResTW;
      const int i = i0 + pi, j = j0 + pj;
      if (i >= H || j >= W) continue;
      const int o = (pi + 1) * MW + pj + 1;
      const double llp = 4.0 * Ms[o] - Ms[o - MW] - Ms[o + MW] - Ms[o - 1] - Ms[o + 1];
      // B^T D^T y: taps (a, b) with i + a - R = c m and j + b - R = c k.
      const int a0 = pos_mod(R - i, c), b0 = pos_mod(R - j, c);
      const int mr = (i + a0 - R) / c - mlo, kr = (j + b0 - R) / c - klo;
      double dat = 0.0;
      for (int a = a0, m = mr; a < n; a += c, ++m) {
        const double* yr = Yl + m * YW;
        const double* ur = Us + a * n;
        for (int b = b0, k = kr; b < n; b += c, ++k) dat = fma(ur[b], yr[k], dat);
      }
      const size_t e = (size_t)i * W + j;
      const double res = (double)bb[e] - (dat + lam * llp);
      acc += res * res;
      if (write_r) {
        rout[e] = (float)res;
        if (bpar != rpar) pout[e] = pin[e];
      }
    }
    double v[1] = {acc};
    block_partials<1, kResThreads / 64>(v, red, d.partials + (size_t)ch * d.pstride * 3 + tile);
    __syncthreads();  // the next band's staging overwrites the regions
  }
}

__global__ __launch_bounds__(kResThreads) void k_ref_res(const RefDesc* __restrict__ t, int count, int total,
                                                         const ChanState* __restrict__ st, int force, int rpar,
                                                         int write_r) {
  extern __shared__ double rsh[];
  __shared__ double red[kResThreads / 64];
  if (!any_selected(t, count, st, force)) return;
  for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
    ref_res_block(t, count, st, force, rpar, write_r, vb, rsh, red);
    __syncthreads();  // the next tile's staging overwrites the regions
  }
}

// ---------------------------------------------------------------------------------------------- finalise ---

__global__ __launch_bounds__(kBlock) void k_ref_fin(int op, const RefDesc* __restrict__ t, int count,
                                                    ChanState* __restrict__ st, double* __restrict__ results,
                                                    int force, int plain_cg, int max_iters, float tol) {
  __shared__ double red[kWaves];
  const int band = blockIdx.x;
  int lo = 0, hi = count - 1;  // scene of the band: the last entry whose band0 <= band
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (t[mid].band0 <= band) lo = mid;
    else hi = mid - 1;
  }
  const RefDesc& d = t[lo];
  ChanState& cs = st[band];
  if (!rep_selected(cs, force)) return;
  const int ch = band - d.band0;
  const int nt = res_tiles(d.g);
  const double* part = d.partials + (size_t)ch * d.pstride * 3;
  double s = 0.0;
  for (int i = threadIdx.x; i < nt; i += kBlock) s += part[i];
  double v[1] = {s};
  block_sums<1>(v, red);
  if (threadIdx.x != 0) return;
  s = v[0];
  double* res = results + (size_t)band * kResultSlots;
  if (op == kRefOut) {
    res[kSlotOutRes] = s;
    return;
  }
  res[kSlotTrueRes] = s;
  cs.ref_iter = cs.iters;
  if (op != kRefStep) return;
  cs.last_rep = cs.iters;
  if (plain_cg) cs.rho = s;  // the recursion continues from the replaced residual
  const bool conv = tol > 0.0f && (s == 0.0 || sqrt(s) <= (double)tol * sqrt(cs.bnorm2));
  if (!isfinite(s)) {
    cs.status = -6;
    cs.active = 0;
    cs.pending = 0;
  } else if (cs.pending) {
    cs.pending = 0;
    if (conv) {
      cs.active = 0;
      cs.status = 0;
    } else if (cs.iters < max_iters) {
      cs.active = 1;  // the recursion had drifted: go on from the replaced residual
    } else {
      cs.active = 0;
      cs.status = 1;
    }
  } else if (cs.active && conv) {
    cs.active = 0;
    cs.status = 0;
  }
}

// ------------------------------------------------------------------------------------------------ host ---

int ref_elem_blocks(const Geom& g) {
  const size_t HW = (size_t)g.H * g.W;
  return (int)((HW + kChunkE - 1) / kChunkE) * g.N;
}
int ref_y_blocks(const Geom& g) { return y_tiles(g) * g.N; }
int ref_res_blocks(const Geom& g) { return res_tiles(g); }  // one workgroup per tile, for all bands

size_t ref_y_lds(const Geom& g) {
  const size_t RH = (size_t)(kYRows - 1) * g.c + 2 * g.R + 1, RW = (size_t)63 * g.c + 2 * g.R + 1;
  return (RH * RW + (size_t)g.n * g.n) * sizeof(double);
}

size_t ref_res_lds(const Geom& g) { return (size_t)res_layout(g).total_doubles * sizeof(double); }

hipError_t ref_prepare() {
  hipError_t e = hipFuncSetAttribute((const void*)k_ref_y, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)kRefMaxLds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_ref_res, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRefMaxLds);
}

constexpr int kRefGrid = 2048;  // workgroups of a replacement launch (they stride over the virtual blocks)

hipError_t launch_ref_elem(int op, const RefDesc* t, int count, int blocks, const ChanState* st, int force,
                           hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ref_elem, dim3(blocks < kRefGrid ? blocks : kRefGrid), dim3(kBlock), 0, s, op, t, count,
                     blocks, st, force);
  return hipGetLastError();
}

hipError_t launch_ref_y(const RefDesc* t, int count, int blocks, size_t lds, const ChanState* st, int force,
                        hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ref_y, dim3(blocks < kRefGrid ? blocks : kRefGrid), dim3(kBlock), lds, s, t, count, blocks,
                     st, force);
  return hipGetLastError();
}

hipError_t launch_ref_res(const RefDesc* t, int count, int blocks, size_t lds, const ChanState* st, int force,
                          int rpar, int write_r, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ref_res, dim3(blocks < kRefGrid ? blocks : kRefGrid), dim3(kResThreads), lds, s, t, count,
                     blocks, st, force, rpar, write_r);
  return hipGetLastError();
}

hipError_t launch_ref_fin(int op, const RefDesc* t, int count, int bands, ChanState* st, double* results,
                          int force, int plain_cg, int max_iters, float tol, hipStream_t s) {
  if (bands <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ref_fin, dim3(bands), dim3(kBlock), 0, s, op, t, count, st, results, force, plain_cg,
                     max_iters, tol);
  return hipGetLastError();
}

}  // namespace llp
