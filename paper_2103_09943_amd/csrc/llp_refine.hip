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
constexpr int kResTH = 8;             // residual tile: HR rows
constexpr int kResTW = 64;            // residual tile: HR columns

__device__ __forceinline__ int wrapr(int i, int n) {
  if (i >= -n && i < 2 * n) return i < 0 ? i + n : (i >= n ? i - n : i);
  const int m = i % n;
  return m < 0 ? m + n : m;
}

__device__ __forceinline__ bool rep_selected(const ChanState& c, int force) {
  return force || c.pending || (c.active && c.iters - c.last_rep >= kRepEvery);
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
__host__ __device__ __forceinline__ int res_tiles(const Geom& g) {
  return ((g.H + kResTH - 1) / kResTH) * res_tiles_x(g);
}
__host__ __device__ __forceinline__ int y_tiles_x(const Geom& g) { return (g.w + 63) / 64; }
__host__ __device__ __forceinline__ int y_tiles(const Geom& g) { return ((g.h + kYRows - 1) / kYRows) * y_tiles_x(g); }
__host__ __device__ __forceinline__ int lr_span(int t, int R, int c) { return (t - 1 + 2 * R) / c + 2; }

}  // namespace

// ------------------------------------------------------------------------------------------- elementwise ---

__global__ __launch_bounds__(kBlock) void k_ref_elem(int op, const RefDesc* __restrict__ t, int count,
                                                     const ChanState* __restrict__ st, int force) {
  const int si = find_scene(t, count, (int)blockIdx.x, [](const RefDesc& d) { return d.e_block0; });
  const RefDesc& d = t[si];
  const Geom& g = d.g;
  const size_t HW = (size_t)g.H * g.W;
  const int per_band = (int)((HW + kChunkE - 1) / kChunkE);
  const int local = (int)blockIdx.x - d.e_block0;
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

// ------------------------------------------------------------------------------------------- D B x (FP64) ---
// y[m][k] = sum_{a,b} u[a][b] x[c m + R - a][c k + R - b] (true convolution, then decimation at phase 0).
// One workgroup per band and tile of kYRows x 64 LR points; the x region the taps reach is staged in LDS.

__global__ __launch_bounds__(kBlock) void k_ref_y(const RefDesc* __restrict__ t, int count,
                                                  const ChanState* __restrict__ st, int force) {
  extern __shared__ double ysh[];
  const int si = find_scene(t, count, (int)blockIdx.x, [](const RefDesc& d) { return d.y_block0; });
  const RefDesc& d = t[si];
  const Geom& g = d.g;
  const int nt = y_tiles(g);
  const int local = (int)blockIdx.x - d.y_block0;
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

// ------------------------------------------------------------------------------------ residual tile (FP64) ---
// r = b - (B^T D^T y + lambda L M L x) on a kResTH x kResTW tile, with M l = |w| l - G (.) S(a) - S(b),
// a = (S(G l)/|w| - mu S(l)/|w|) dinv, b = S(l)/|w| - a mu (S the periodic (2r+1)^2 window sum), and G = L Y,
// mu = S(G)/|w|, var = S(G^2)/|w| - mu^2, dinv = 1/(eps/|w| + var) (0 where that is 0), all in FP64 from the
// float32 PAN image.  Regions, as offsets from the tile's corner:
//   X (x and Y):    halo E = 2r + 2     L (G, l = L x, G l): halo 2r + 1
//   A (a, b):       halo r + 1          M (M l):             halo 1
// and the LR samples of y the tile's B^T D^T taps reach.

__global__ __launch_bounds__(kBlock) void k_ref_res(const RefDesc* __restrict__ t, int count,
                                                    const ChanState* __restrict__ st, int force, int rpar,
                                                    int write_r) {
  extern __shared__ double rsh[];
  __shared__ double red[kWaves];
  const int si = find_scene(t, count, (int)blockIdx.x, [](const RefDesc& d) { return d.r_block0; });
  const RefDesc& d = t[si];
  const Geom& g = d.g;
  const int nt = res_tiles(g);
  const int local = (int)blockIdx.x - d.r_block0;
  if (local >= nt * g.N) return;
  const int ch = local / nt, tile = local - ch * nt;
  const ChanState& cs = st[d.band0 + ch];
  if (!rep_selected(cs, force)) return;
  const int H = g.H, W = g.W, r = g.r, c = g.c, n = g.n, R = g.R;
  const int tx = res_tiles_x(g);
  const int i0 = (tile / tx) * kResTH, j0 = (tile % tx) * kResTW;
  const int E = 2 * r + 2, h1 = 2 * r + 1, h2 = r + 1;
  const int XH = kResTH + 2 * E, XW = kResTW + 2 * E;
  const int LH = kResTH + 2 * h1, LW = kResTW + 2 * h1;
  const int AH = kResTH + 2 * h2, AW = kResTW + 2 * h2;
  const int MH = kResTH + 2, MW = kResTW + 2;
  const int mlo = floor_div(i0 - R, c), klo = floor_div(j0 - R, c);
  const int YH = lr_span(kResTH, R, c), YW = lr_span(kResTW, R, c);
  double* Xs = rsh;               // x, later M l
  double* Gs = Xs + XH * XW;      // G = L Y
  double* Ls = Gs + LH * LW;      // l = L x
  double* GLs = Ls + LH * LW;     // G l
  double* As = GLs + LH * LW;     // a
  double* Bs = As + AH * AW;      // b
  double* Yl = Bs + AH * AW;      // y (LR)
  double* Us = Yl + YH * YW;      // taps
  float* Ys = (float*)(Us + n * n);  // PAN

  const size_t HW = (size_t)H * W;
  const double* xb = d.xacc + (size_t)ch * HW;
  for (int idx = threadIdx.x; idx < XH * XW; idx += kBlock) {
    const int li = idx / XW, lj = idx - li * XW;
    const size_t e = (size_t)wrapr(i0 - E + li, H) * W + wrapr(j0 - E + lj, W);
    Xs[idx] = xb[e];
    Ys[idx] = d.Y[e];
  }
  const double* yb = d.y64 + (size_t)ch * g.h * g.w;
  for (int idx = threadIdx.x; idx < YH * YW; idx += kBlock) {
    const int li = idx / YW, lj = idx - li * YW;
    Yl[idx] = yb[(size_t)wrapr(mlo + li, g.h) * g.w + wrapr(klo + lj, g.w)];
  }
  for (int idx = threadIdx.x; idx < n * n; idx += kBlock) Us[idx] = (double)d.u[idx];
  __syncthreads();

  // L region: G = L Y, l = L x, G l (5-point stencil of eq. reg2).
  for (int idx = threadIdx.x; idx < LH * LW; idx += kBlock) {
    const int li = idx / LW, lj = idx - li * LW;
    const int o = (li + 1) * XW + lj + 1;
    const double gv = 4.0 * (double)Ys[o] - (double)Ys[o - XW] - (double)Ys[o + XW] - (double)Ys[o - 1] -
                      (double)Ys[o + 1];
    const double lv = 4.0 * Xs[o] - Xs[o - XW] - Xs[o + XW] - Xs[o - 1] - Xs[o + 1];
    Gs[idx] = gv;
    Ls[idx] = lv;
    GLs[idx] = gv * lv;
  }
  __syncthreads();

  // A region: window statistics of G and the local linear coefficients (a, b) of l on G.
  const double nw = (double)((2 * r + 1) * (2 * r + 1));
  const double epsw = (double)g.eps / nw;
  for (int idx = threadIdx.x; idx < AH * AW; idx += kBlock) {
    const int ai = idx / AW, aj = idx - ai * AW;
    double sg = 0.0, sg2 = 0.0, sl = 0.0, sgl = 0.0;
    for (int dy = 0; dy <= 2 * r; ++dy) {
      const int o = (ai + dy) * LW + aj;
      for (int dx = 0; dx <= 2 * r; ++dx) {
        const double gv = Gs[o + dx];
        sg += gv;
        sg2 += gv * gv;
        sl += Ls[o + dx];
        sgl += GLs[o + dx];
      }
    }
    const double mu = sg / nw;
    const double var = sg2 / nw - mu * mu;
    const double den = epsw + var;
    const double di = den != 0.0 ? 1.0 / den : 0.0;
    const double m1 = sl / nw, m2 = sgl / nw;
    const double a = (m2 - mu * m1) * di;
    As[idx] = a;
    Bs[idx] = m1 - a * mu;
  }
  __syncthreads();

  // M region: M l = |w| l - G S(a) - S(b)  (into the x buffer, no longer needed).
  double* Ms = Xs;
  for (int idx = threadIdx.x; idx < MH * MW; idx += kBlock) {
    const int mi = idx / MW, mj = idx - mi * MW;
    double sa = 0.0, sb = 0.0;
    for (int dy = 0; dy <= 2 * r; ++dy) {
      const int o = (mi + dy) * AW + mj;
      for (int dx = 0; dx <= 2 * r; ++dx) {
        sa += As[o + dx];
        sb += Bs[o + dx];
      }
    }
    const int lo = (mi + 2 * r) * LW + mj + 2 * r;
    Ms[idx] = nw * Ls[lo] - Gs[lo] * sa - sb;
  }
  __syncthreads();

  // Tile: r = b - (B^T D^T y + lambda L (M l)).
  const double lam = (double)g.lam;
  const float* bb = d.b + (size_t)ch * HW;
  const int bpar = cs.iters & 1;  // the buffers holding this band's r_k and p_k
  float* rout = d.r[rpar] + (size_t)ch * HW;
  const float* pin = d.p[bpar] + (size_t)ch * HW;
  float* pout = d.p[rpar] + (size_t)ch * HW;
  double acc = 0.0;
  for (int idx = threadIdx.x; idx < kResTH * kResTW; idx += kBlock) {
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
  block_partials<1>(v, red, d.partials + (size_t)ch * d.pstride * 3 + tile);
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
int ref_res_blocks(const Geom& g) { return res_tiles(g) * g.N; }

size_t ref_y_lds(const Geom& g) {
  const size_t RH = (size_t)(kYRows - 1) * g.c + 2 * g.R + 1, RW = (size_t)63 * g.c + 2 * g.R + 1;
  return (RH * RW + (size_t)g.n * g.n) * sizeof(double);
}

size_t ref_res_lds(const Geom& g) {
  const int r = g.r, E = 2 * r + 2, h1 = 2 * r + 1, h2 = r + 1;
  const size_t X = (size_t)(kResTH + 2 * E) * (kResTW + 2 * E);
  const size_t L = (size_t)(kResTH + 2 * h1) * (kResTW + 2 * h1);
  const size_t A = (size_t)(kResTH + 2 * h2) * (kResTW + 2 * h2);
  const size_t Y = (size_t)lr_span(kResTH, g.R, g.c) * lr_span(kResTW, g.R, g.c);
  return (X + 3 * L + 2 * A + Y + (size_t)g.n * g.n) * sizeof(double) + X * sizeof(float);
}

hipError_t ref_prepare() {
  hipError_t e = hipFuncSetAttribute((const void*)k_ref_y, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)kRefMaxLds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_ref_res, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRefMaxLds);
}

hipError_t launch_ref_elem(int op, const RefDesc* t, int count, int blocks, const ChanState* st, int force,
                           hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ref_elem, dim3(blocks), dim3(kBlock), 0, s, op, t, count, st, force);
  return hipGetLastError();
}

hipError_t launch_ref_y(const RefDesc* t, int count, int blocks, size_t lds, const ChanState* st, int force,
                        hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ref_y, dim3(blocks), dim3(kBlock), lds, s, t, count, st, force);
  return hipGetLastError();
}

hipError_t launch_ref_res(const RefDesc* t, int count, int blocks, size_t lds, const ChanState* st, int force,
                          int rpar, int write_r, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ref_res, dim3(blocks), dim3(kBlock), lds, s, t, count, st, force, rpar, write_r);
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
