// HIP kernels (gfx950) for the LLP HRMS solve of Sec. III-B: the system of eq. (Z_ini_matting),
//   (B^T D^T D B + lambda L^T M_LY L) Z_i = B^T D^T X_i,
// solved per band by conjugate gradients.
//
// Layout: planar float32, row-major, band-major ([N][H][W]); all convolutions and windows are periodic.
// The data term is applied in the spatial domain on the low-resolution lattice: D B p is evaluated only at
// the h x w kept pixels (n^2 taps each), and B^T D^T spreads those values back (about (n/c)^2 taps per
// high-resolution pixel).  The LLP term is applied matrix-free from the window form of eq. (matting_matrix):
//   M l = |w| l - G (.) S_r(a) - S_r(b),  a_k = (mean_k(G l) - mu_k mean_k(l)) dinv_k,  b_k = mean_k(l) - a_k mu_k,
// with G = L Y, S_r the (2r+1)^2 window sum, and (mu, dinv) the PAN window statistics computed once per scene.
// Reductions (dot products, norms, objective) accumulate in FP64 in a fixed order (deterministic).
#include "llp_internal.h"

#include <math.h>

namespace llp {

constexpr int kBlock = 256;
constexpr int kChunk = kBlock * 16;  // elements per block in the flat kernels

const TileShape kTileVariants[kNumTileVariants] = {{32, 64}, {16, 64}, {32, 32}, {64, 64}, {16, 128}};

__device__ __forceinline__ int wrapi(int i, int n) {
  int m = i % n;
  return m < 0 ? m + n : m;
}
__host__ __device__ __forceinline__ int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
__host__ __device__ __forceinline__ int ceil_div(int a, int b) { return -floor_div(-a, b); }

// ------------------------------------------------------------------------------------- reductions ---

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the block; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / 64; ++i) t += red[i];
  return t;
}

// Store this block's partial and count it in; returns true (uniformly) in the block that arrives last.
__device__ __forceinline__ bool publish_partial(double total, double* slot, unsigned* counter, int nblk,
                                                int* sflag) {
  if (threadIdx.x == 0) {
    *slot = total;
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    *sflag = (prev == (unsigned)(nblk - 1));
  }
  __syncthreads();
  const bool last = *sflag != 0;
  if (last) __threadfence();
  return last;
}

// In the last block: sum of nblk partials in a fixed order; result valid in thread 0.
__device__ __forceinline__ double gather_partials(const double* partials, int nblk, double* red) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kBlock) v += __builtin_nontemporal_load(partials + i);
  __syncthreads();  // red may still be read by thread 0 of the first block_sum
  return block_sum(v, red);
}

// ---------------------------------------------------------------------------------- input checks ---

__global__ __launch_bounds__(kBlock) void k_check_finite(const float* __restrict__ a, size_t count,
                                                         int* __restrict__ flag) {
  int bad = 0;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (size_t)gridDim.x * kBlock)
    bad |= !isfinite(a[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

hipError_t launch_check_finite(const float* a, size_t count, int* flag, hipStream_t s) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + kBlock * 8 - 1) / (kBlock * 8);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)blocks), dim3(kBlock), 0, s, a, count, flag);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------ PAN statistics (a2) ---
// G = L Y, and for every window centre k: mu_k = mean of G over w_k, var_k its population variance,
// dinv_k = 1/(eps/|w| + var_k) (0 where that vanishes).  eq. (matting_matrix) with I = L Y.

__device__ __forceinline__ double lap64(const float* __restrict__ Y, int i, int j, int H, int W) {
  const int im = i == 0 ? H - 1 : i - 1, ip = i == H - 1 ? 0 : i + 1;
  const int jm = j == 0 ? W - 1 : j - 1, jp = j == W - 1 ? 0 : j + 1;
  return 4.0 * (double)Y[(size_t)i * W + j] - (double)Y[(size_t)im * W + j] - (double)Y[(size_t)ip * W + j] -
         (double)Y[(size_t)i * W + jm] - (double)Y[(size_t)i * W + jp];
}

__global__ __launch_bounds__(kBlock) void k_pan_stats(Geom g, const float* __restrict__ Y, float* __restrict__ G,
                                                      float* __restrict__ MU, float* __restrict__ DI) {
  const size_t HW = (size_t)g.H * g.W;
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= HW) return;
  const int ki = (int)(idx / g.W), kj = (int)(idx % g.W);
  const int r = g.r;
  const double nw = (double)((2 * r + 1) * (2 * r + 1));
  double s1 = 0.0, s2 = 0.0;
  for (int dy = -r; dy <= r; ++dy) {
    const int i = wrapi(ki + dy, g.H);
    for (int dx = -r; dx <= r; ++dx) {
      const double v = lap64(Y, i, wrapi(kj + dx, g.W), g.H, g.W);
      s1 += v;
      s2 += v * v;
    }
  }
  const double mu = s1 / nw;
  const double var = s2 / nw - mu * mu;
  const double den = (double)g.eps / nw + var;
  G[idx] = (float)lap64(Y, ki, kj, g.H, g.W);
  MU[idx] = (float)mu;
  DI[idx] = den != 0.0 ? (float)(1.0 / den) : 0.0f;
}

hipError_t launch_pan_stats(const Geom& g, const float* Y, float* G, float* mu, float* dinv, int* flag,
                            hipStream_t s) {
  (void)flag;
  const size_t HW = (size_t)g.H * g.W;
  hipLaunchKernelGGL(k_pan_stats, dim3((unsigned)((HW + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, g, Y, G, mu,
                     dinv);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------ RHS (a3) ---
// b = B^T D^T X: the low-resolution sample X[m][k] sits at (c m, c k); B^T correlates with u, so
// b[i][j] = sum over taps (a, b') with (i + a - R) = c m and (j + b' - R) = c k of u[a][b'] X[m][k].

__global__ __launch_bounds__(kBlock) void k_rhs(Geom g, const float* __restrict__ X, const float* __restrict__ u,
                                                float* __restrict__ b, double* __restrict__ partials,
                                                unsigned* __restrict__ counters, ChanState* __restrict__ st,
                                                int pstride, int nblk) {
  __shared__ double red[kBlock / 64];
  __shared__ int sflag;
  const int ch = blockIdx.y;
  const size_t HW = (size_t)g.H * g.W;
  const float* Xc = X + (size_t)ch * g.h * g.w;
  float* bc = b + (size_t)ch * HW;
  double acc = 0.0;
  const size_t e0 = (size_t)blockIdx.x * kChunk;
  const size_t e1 = e0 + kChunk < HW ? e0 + kChunk : HW;
  for (size_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
    const int i = (int)(e / g.W), j = (int)(e % g.W);
    const int a0 = wrapi(g.R - i, g.c), b0 = wrapi(g.R - j, g.c);
    double v = 0.0;
    for (int a = a0; a < g.n; a += g.c) {
      const int m = wrapi((i + a - g.R) / g.c, g.h);
      for (int bb = b0; bb < g.n; bb += g.c) {
        const int k = wrapi((j + bb - g.R) / g.c, g.w);
        v += (double)u[a * g.n + bb] * (double)Xc[(size_t)m * g.w + k];
      }
    }
    const float vf = (float)v;
    bc[e] = vf;
    acc += (double)vf * (double)vf;
  }
  const double tot = block_sum(acc, red);
  if (publish_partial(tot, partials + (size_t)ch * pstride + blockIdx.x, counters + ch, nblk, &sflag)) {
    const double s = gather_partials(partials + (size_t)ch * pstride, nblk, red);
    if (threadIdx.x == 0) {
      st[ch].bnorm2 = s;
      counters[ch] = 0;
    }
  }
}

hipError_t launch_rhs(const Geom& g, const float* X, const float* u, float* b, double* partials,
                      unsigned* counters, ChanState* st, hipStream_t s) {
  const size_t HW = (size_t)g.H * g.W;
  const int nblk = (int)((HW + kChunk - 1) / kChunk);
  const int pstride = (int)max_partials_per_band(g);
  hipLaunchKernelGGL(k_rhs, dim3(nblk, g.N), dim3(kBlock), 0, s, g, X, u, b, partials, counters, st, pstride,
                     nblk);
  return hipGetLastError();
}

// ------------------------------------------------------------------- operator A (a5 + a6, fused) ---

ApplyLayout apply_layout(int TH, int TW, int R, int r, int c, int n) {
  ApplyLayout L;
  L.TH = TH;
  L.TW = TW;
  const int hl = 2 * r + 2;
  L.E = 2 * R > hl ? 2 * R : hl;
  L.PH = TH + 2 * L.E;
  L.PW = TW + 2 * L.E;
  L.YHm = (TH - 1 + 2 * R) / c + 2;
  L.YWm = (TW - 1 + 2 * R) / c + 2;
  const int h1 = 2 * r + 1, h2 = r + 1;
  L.LH = TH + 2 * h1;
  L.LW = TW + 2 * h1;
  L.AH = TH + 2 * h2;
  L.AW = TW + 2 * h2;
  auto mx = [](int a, int b) { return a > b ? a : b; };
  const int szP = mx(L.PH * L.PW, mx(2 * L.LH * L.AW, 2 * L.AH * (TW + 2)));
  const int szL = L.LH * L.LW;
  const int szX = mx(L.LH * L.LW, mx(2 * L.AH * L.AW, (TH + 2) * (TW + 2)));
  const int szY = L.YHm * L.YWm;
  const int szU = n * n;
  auto al = [](int v) { return (v + 3) & ~3; };
  L.offP = 0;
  L.offL = L.offP + al(szP);
  L.offX = L.offL + al(szL);
  L.offY = L.offX + al(szX);
  L.offU = L.offY + al(szY);
  L.total = L.offU + al(szU);
  return L;
}

// One workgroup computes q = A p on a TH x TW tile of one band.  The input (with a halo of E pixels) is
// staged in LDS; the low-resolution intermediate D B p of the tile, l = L p, the window sums and the window
// coefficients (a, b) are formed in LDS stage by stage; buffers whose stage has passed are reused.
// mode 1 fuses the CG direction update p_new = r + beta p_old (written for the tile interior) and the
// partial p_new^T q; the last workgroup of a band turns the sum into gamma and alpha = rho / gamma.
template <int TH, int TW>
__global__ __launch_bounds__(kBlock) void k_apply(Geom g, ApplyLayout lay, int mode, const float* __restrict__ zr,
                                                  const float* __restrict__ p_old, float* __restrict__ p_new,
                                                  const float* __restrict__ u, const float* __restrict__ Gp,
                                                  const float* __restrict__ MU, const float* __restrict__ DI,
                                                  float* __restrict__ q, double* __restrict__ partials,
                                                  unsigned* __restrict__ counters, ChanState* __restrict__ st,
                                                  int tiles_x, int ntiles, int pstride) {
  constexpr int NPT = TH * TW / kBlock;
  static_assert(TH * TW % kBlock == 0, "tile must be a multiple of the block");
  extern __shared__ float smem[];
  __shared__ double red[kBlock / 64];
  __shared__ int sflag;

  // Block -> (tile, band): consecutive workgroups are dealt round-robin to the 8 XCDs; remap so that each XCD
  // walks a contiguous run of (tile, band) pairs with the bands of a tile adjacent (shared halos and PAN
  // statistics stay in that XCD's L2).
  const int nb = ntiles * g.N;
  const int b8 = (nb / 8) * 8;
  const int bid = blockIdx.x;
  const int lin = bid < b8 ? (bid % 8) * (b8 / 8) + bid / 8 : bid;
  const int tile = lin / g.N, ch = lin % g.N;
  const int i0 = (tile / tiles_x) * TH, j0 = (tile % tiles_x) * TW;

  const int H = g.H, W = g.W, n = g.n, R = g.R, r = g.r, c = g.c;
  const size_t HW = (size_t)H * W;
  float beta = 0.0f;
  bool first = true;
  if (mode == 1) {
    if (!st[ch].active) return;
    first = st[ch].iters == 0;
    beta = (float)st[ch].beta;
  }

  float* P = smem + lay.offP;
  float* Ls = smem + lay.offL;
  float* Xs = smem + lay.offX;
  float* Ys = smem + lay.offY;
  float* Us = smem + lay.offU;
  const int E = lay.E, PH = lay.PH, PW = lay.PW;

  // S1: stage the input region [i0-E, i0+TH+E) x [j0-E, j0+TW+E) (periodic) and the kernel.
  for (int idx = threadIdx.x; idx < n * n; idx += kBlock) Us[idx] = u[idx];
  {
    const float* zin = zr + (size_t)ch * HW;
    const float* pin = p_old + (size_t)ch * HW;
    float* pout = p_new + (size_t)ch * HW;
    for (int idx = threadIdx.x; idx < PH * PW; idx += kBlock) {
      const int py = idx / PW, px = idx - py * PW;
      const int ui = i0 - E + py, uj = j0 - E + px;
      const size_t off = (size_t)wrapi(ui, H) * W + wrapi(uj, W);
      float v = zin[off];
      if (mode == 1) {
        if (!first) v = fmaf(beta, pin[off], v);
        if (py >= E && py < E + TH && px >= E && px < E + TW && ui < H && uj < W) pout[off] = v;
      }
      P[idx] = v;
    }
  }
  __syncthreads();

  // S2a: y = D B p on the low-resolution points whose taps reach the tile.
  const int mlo = ceil_div(i0 - R, c), klo = ceil_div(j0 - R, c);
  const int YH = floor_div(i0 + TH - 1 + R, c) - mlo + 1;
  const int YW = floor_div(j0 + TW - 1 + R, c) - klo + 1;
  for (int idx = threadIdx.x; idx < YH * YW; idx += kBlock) {
    const int ym = idx / YW, yk = idx - ym * YW;
    const int prow0 = c * (mlo + ym) + R - (i0 - E);
    const int pcol0 = c * (klo + yk) + R - (j0 - E);
    float acc = 0.0f;
    for (int a = 0; a < n; ++a) {
      const float* prow = P + (prow0 - a) * PW + pcol0;
      const float* urow = Us + a * n;
      for (int b = 0; b < n; ++b) acc = fmaf(urow[b], prow[-b], acc);
    }
    Ys[idx] = acc;
  }
  // S2b: l = L p and G l on [i0-h1, i0+TH+h1) x [j0-h1, j0+TW+h1).
  const int h1 = 2 * r + 1, h2 = r + 1;
  const int LH = lay.LH, LW = lay.LW;
  for (int idx = threadIdx.x; idx < LH * LW; idx += kBlock) {
    const int ly = idx / LW, lx = idx - ly * LW;
    const float* pc = P + (ly - h1 + E) * PW + (lx - h1 + E);
    const float lv = 4.0f * pc[0] - pc[-PW] - pc[PW] - pc[-1] - pc[1];
    const float gv = Gp[(size_t)wrapi(i0 - h1 + ly, H) * W + wrapi(j0 - h1 + lx, W)];
    Ls[idx] = lv;
    Xs[idx] = gv * lv;
  }
  float pv[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int idx = threadIdx.x + k * kBlock;
    pv[k] = P[(idx / TW + E) * PW + (idx % TW) + E];
  }
  __syncthreads();

  // S3: horizontal window sums of l and G l (columns [j0-h2, j0+TW+h2)).
  const int AW = lay.AW, AH = lay.AH;
  float* HBl = P;
  float* HBg = P + LH * AW;
  for (int idx = threadIdx.x; idx < LH * AW; idx += kBlock) {
    const int y = idx / AW, x = idx - y * AW;
    const float* lr = Ls + y * LW + x;
    const float* gr = Xs + y * LW + x;
    float s1 = 0.0f, s2 = 0.0f;
    for (int d = 0; d <= 2 * r; ++d) {
      s1 += lr[d];
      s2 += gr[d];
    }
    HBl[idx] = s1;
    HBg[idx] = s2;
  }
  __syncthreads();

  // S4: vertical window sums -> window coefficients a, b on [i0-h2, i0+TH+h2) x [j0-h2, j0+TW+h2).
  const float inv_nw = 1.0f / (float)((2 * r + 1) * (2 * r + 1));
  float* As = Xs;
  float* Bs = Xs + AH * AW;
  for (int idx = threadIdx.x; idx < AH * AW; idx += kBlock) {
    const int y = idx / AW, x = idx - y * AW;
    float s1 = 0.0f, s2 = 0.0f;
    for (int d = 0; d <= 2 * r; ++d) {
      s1 += HBl[(y + d) * AW + x];
      s2 += HBg[(y + d) * AW + x];
    }
    const size_t goff = (size_t)wrapi(i0 - h2 + y, H) * W + wrapi(j0 - h2 + x, W);
    const float mu = MU[goff], di = DI[goff];
    const float m1 = s1 * inv_nw, m2 = s2 * inv_nw;
    const float a = (m2 - mu * m1) * di;
    As[idx] = a;
    Bs[idx] = m1 - a * mu;
  }
  __syncthreads();

  // S5: horizontal window sums of a, b (columns [j0-1, j0+TW+1)).
  const int W3 = TW + 2;
  float* HAa = P;
  float* HAb = P + AH * W3;
  for (int idx = threadIdx.x; idx < AH * W3; idx += kBlock) {
    const int y = idx / W3, x = idx - y * W3;
    const float* ar = As + y * AW + x;
    const float* br = Bs + y * AW + x;
    float s1 = 0.0f, s2 = 0.0f;
    for (int d = 0; d <= 2 * r; ++d) {
      s1 += ar[d];
      s2 += br[d];
    }
    HAa[idx] = s1;
    HAb[idx] = s2;
  }
  __syncthreads();

  // S6: M l = |w| l - G S(a) - S(b) on [i0-1, i0+TH+1) x [j0-1, j0+TW+1).
  const float nwf = (float)((2 * r + 1) * (2 * r + 1));
  float* Ml = Xs;
  for (int idx = threadIdx.x; idx < (TH + 2) * W3; idx += kBlock) {
    const int y = idx / W3, x = idx - y * W3;
    float sa = 0.0f, sb = 0.0f;
    for (int d = 0; d <= 2 * r; ++d) {
      sa += HAa[(y + d) * W3 + x];
      sb += HAb[(y + d) * W3 + x];
    }
    const float lv = Ls[(y - 1 + h1) * LW + (x - 1 + h1)];
    const float gv = Gp[(size_t)wrapi(i0 - 1 + y, H) * W + wrapi(j0 - 1 + x, W)];
    Ml[idx] = nwf * lv - gv * sa - sb;
  }
  __syncthreads();

  // S7: q = B^T D^T y + lambda L (M l) on the tile.
  double acc = 0.0;
  float* qc = q + (size_t)ch * HW;
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int idx = threadIdx.x + k * kBlock;
    const int y = idx / TW, x = idx % TW;
    const int i = i0 + y, j = j0 + x;
    if (i < H && j < W) {
      const float* mc = Ml + (y + 1) * W3 + (x + 1);
      const float ql = g.lam * (4.0f * mc[0] - mc[-W3] - mc[W3] - mc[-1] - mc[1]);
      const int a0 = wrapi(R - i, c), b0 = wrapi(R - j, c);
      float qd = 0.0f;
      for (int a = a0; a < n; a += c) {
        const int ym = (i + a - R) / c - mlo;
        const float* yrow = Ys + ym * YW - klo;
        const float* urow = Us + a * n;
        for (int b = b0; b < n; b += c) qd = fmaf(urow[b], yrow[(j + b - R) / c], qd);
      }
      const float qv = qd + ql;
      qc[(size_t)i * W + j] = qv;
      acc += (double)pv[k] * (double)qv;
    }
  }
  if (mode == 1) {
    const double tot = block_sum(acc, red);
    if (publish_partial(tot, partials + (size_t)ch * pstride + tile, counters + ch, ntiles, &sflag)) {
      const double gam = gather_partials(partials + (size_t)ch * pstride, ntiles, red);
      if (threadIdx.x == 0) {
        ChanState& s = st[ch];
        s.gamma = gam;
        if (!(gam > 0.0) || !isfinite(gam)) {
          s.status = -6;  // LLP_E_BREAKDOWN
          s.active = 0;
        } else {
          s.alpha = s.rho / gam;
        }
        counters[ch] = 0;
      }
    }
  }
}

template <int TH, int TW>
static hipError_t launch_apply_t(const Geom& g, int mode, const float* zr, const float* p_old, float* p_new,
                                 const float* u, const float* G, const float* mu, const float* dinv, float* q,
                                 double* partials, unsigned* counters, ChanState* st, hipStream_t s) {
  const ApplyLayout lay = apply_layout(TH, TW, g.R, g.r, g.c, g.n);
  const size_t bytes = (size_t)lay.total * sizeof(float);
  static size_t configured = 0;
  if (bytes > 65536 && bytes > configured) {
    hipError_t e = hipFuncSetAttribute((const void*)k_apply<TH, TW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)bytes);
    if (e != hipSuccess) return e;
    configured = bytes;
  }
  const int tiles_x = (g.W + TW - 1) / TW, tiles_y = (g.H + TH - 1) / TH;
  const int ntiles = tiles_x * tiles_y;
  const int pstride = (int)max_partials_per_band(g);
  hipLaunchKernelGGL((k_apply<TH, TW>), dim3(ntiles * g.N), dim3(kBlock), bytes, s, g, lay, mode, zr,
                     p_old ? p_old : zr, p_new, u, G, mu, dinv, q, partials, counters, st, tiles_x, ntiles,
                     pstride);
  return hipGetLastError();
}

hipError_t launch_apply(const Geom& g, int variant, int mode, const float* zr, const float* p_old, float* p_new,
                        const float* u, const float* G, const float* mu, const float* dinv, float* q,
                        double* partials, unsigned* counters, ChanState* st, hipStream_t s) {
  switch (variant) {
    case 0: return launch_apply_t<32, 64>(g, mode, zr, p_old, p_new, u, G, mu, dinv, q, partials, counters, st, s);
    case 1: return launch_apply_t<16, 64>(g, mode, zr, p_old, p_new, u, G, mu, dinv, q, partials, counters, st, s);
    case 2: return launch_apply_t<32, 32>(g, mode, zr, p_old, p_new, u, G, mu, dinv, q, partials, counters, st, s);
    case 3: return launch_apply_t<64, 64>(g, mode, zr, p_old, p_new, u, G, mu, dinv, q, partials, counters, st, s);
    case 4: return launch_apply_t<16, 128>(g, mode, zr, p_old, p_new, u, G, mu, dinv, q, partials, counters, st, s);
    default: return hipErrorInvalidValue;
  }
}

size_t max_partials_per_band(const Geom& g) {
  const size_t HW = (size_t)g.H * g.W;
  size_t m = (HW + kChunk - 1) / kChunk;
  for (int v = 0; v < kNumTileVariants; ++v) {
    const size_t t = (size_t)((g.H + kTileVariants[v].TH - 1) / kTileVariants[v].TH) *
                     (size_t)((g.W + kTileVariants[v].TW - 1) / kTileVariants[v].TW);
    if (t > m) m = t;
  }
  return m;
}

// ------------------------------------------------------------------------------ CG vector steps (a7) ---

// Start of the recursion: r = b (Z = 0) or r = b - A Z (caller's start, q = A Z); rho = r^T r.
__global__ __launch_bounds__(kBlock) void k_init_residual(Geom g, int from_init, const float* __restrict__ b,
                                                          const float* __restrict__ q, float* __restrict__ r,
                                                          float* __restrict__ x, double* __restrict__ partials,
                                                          unsigned* __restrict__ counters,
                                                          ChanState* __restrict__ st, int pstride, int nblk,
                                                          int max_iters, float tol) {
  __shared__ double red[kBlock / 64];
  __shared__ int sflag;
  const int ch = blockIdx.y;
  const size_t HW = (size_t)g.H * g.W;
  const size_t base = (size_t)ch * HW;
  double acc = 0.0;
  const size_t e0 = (size_t)blockIdx.x * kChunk;
  const size_t e1 = e0 + kChunk < HW ? e0 + kChunk : HW;
  for (size_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
    float v = b[base + e];
    if (from_init) v -= q[base + e];
    else x[base + e] = 0.0f;
    r[base + e] = v;
    acc += (double)v * (double)v;
  }
  const double tot = block_sum(acc, red);
  if (publish_partial(tot, partials + (size_t)ch * pstride + blockIdx.x, counters + ch, nblk, &sflag)) {
    const double rho = gather_partials(partials + (size_t)ch * pstride, nblk, red);
    if (threadIdx.x == 0) {
      ChanState& s = st[ch];
      s.rho = rho;
      s.iters = 0;
      s.alpha = 0.0;
      s.beta = 0.0;
      s.gamma = 0.0;
      const bool exact = (!from_init && s.bnorm2 == 0.0) || rho == 0.0;
      const bool conv = exact || (tol > 0.0f && sqrt(rho) <= (double)tol * sqrt(s.bnorm2));
      s.active = (!conv && max_iters > 0) ? 1 : 0;
      s.status = (conv || tol <= 0.0f) ? 0 : 1;
      if (!isfinite(rho)) {
        s.status = -7;
        s.active = 0;
      }
      counters[ch] = 0;
    }
  }
}

hipError_t launch_init_residual(const Geom& g, int from_init, const float* b, const float* q, float* r, float* x,
                                double* partials, unsigned* counters, ChanState* st, int max_iters, float tol,
                                hipStream_t s) {
  const size_t HW = (size_t)g.H * g.W;
  const int nblk = (int)((HW + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_init_residual, dim3(nblk, g.N), dim3(kBlock), 0, s, g, from_init, b, q, r, x, partials,
                     counters, st, (int)max_partials_per_band(g), nblk, max_iters, tol);
  return hipGetLastError();
}

// x += alpha p, r -= alpha q, rho' = r^T r; the last block sets beta = rho'/rho and the stopping state.
__global__ __launch_bounds__(kBlock) void k_cg_update(Geom g, float* __restrict__ x, float* __restrict__ r,
                                                      const float* __restrict__ p, const float* __restrict__ q,
                                                      double* __restrict__ partials, unsigned* __restrict__ counters,
                                                      ChanState* __restrict__ st, int pstride, int nblk,
                                                      int max_iters, float tol) {
  __shared__ double red[kBlock / 64];
  __shared__ int sflag;
  const int ch = blockIdx.y;
  if (!st[ch].active) return;
  const float alpha = (float)st[ch].alpha;
  const size_t HW = (size_t)g.H * g.W;
  const size_t base = (size_t)ch * HW;
  double acc = 0.0;
  const size_t e0 = (size_t)blockIdx.x * kChunk;
  const size_t e1 = e0 + kChunk < HW ? e0 + kChunk : HW;
  if ((HW & 3) == 0) {
    float4* x4 = reinterpret_cast<float4*>(x + base);
    float4* r4 = reinterpret_cast<float4*>(r + base);
    const float4* p4 = reinterpret_cast<const float4*>(p + base);
    const float4* q4 = reinterpret_cast<const float4*>(q + base);
    for (size_t e = e0 / 4 + threadIdx.x; e < e1 / 4; e += kBlock) {
      float4 xv = x4[e], rv = r4[e];
      const float4 pv = p4[e], qv = q4[e];
      xv.x = fmaf(alpha, pv.x, xv.x);
      xv.y = fmaf(alpha, pv.y, xv.y);
      xv.z = fmaf(alpha, pv.z, xv.z);
      xv.w = fmaf(alpha, pv.w, xv.w);
      rv.x = fmaf(-alpha, qv.x, rv.x);
      rv.y = fmaf(-alpha, qv.y, rv.y);
      rv.z = fmaf(-alpha, qv.z, rv.z);
      rv.w = fmaf(-alpha, qv.w, rv.w);
      x4[e] = xv;
      r4[e] = rv;
      acc += (double)rv.x * rv.x + (double)rv.y * rv.y + (double)rv.z * rv.z + (double)rv.w * rv.w;
    }
  } else {
    for (size_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
      x[base + e] = fmaf(alpha, p[base + e], x[base + e]);
      const float rv = fmaf(-alpha, q[base + e], r[base + e]);
      r[base + e] = rv;
      acc += (double)rv * rv;
    }
  }
  const double tot = block_sum(acc, red);
  if (publish_partial(tot, partials + (size_t)ch * pstride + blockIdx.x, counters + ch, nblk, &sflag)) {
    const double rho = gather_partials(partials + (size_t)ch * pstride, nblk, red);
    if (threadIdx.x == 0) {
      ChanState& s = st[ch];
      s.beta = rho / s.rho;
      s.rho = rho;
      s.iters += 1;
      if (!isfinite(rho)) {
        s.status = -6;
        s.active = 0;
      } else if (tol > 0.0f && sqrt(rho) <= (double)tol * sqrt(s.bnorm2)) {
        s.status = 0;
        s.active = 0;
      } else if (s.iters >= max_iters) {
        s.status = tol > 0.0f ? 1 : 0;
        s.active = 0;
      }
      counters[ch] = 0;
    }
  }
}

hipError_t launch_cg_update(const Geom& g, float* x, float* r, const float* p, const float* q, double* partials,
                            unsigned* counters, ChanState* st, int max_iters, float tol, hipStream_t s) {
  const size_t HW = (size_t)g.H * g.W;
  const int nblk = (int)((HW + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_cg_update, dim3(nblk, g.N), dim3(kBlock), 0, s, g, x, r, p, q, partials, counters, st,
                     (int)max_partials_per_band(g), nblk, max_iters, tol);
  return hipGetLastError();
}

// ||b - q||^2 per band (q = A Z): the true residual of the returned iterate.
__global__ __launch_bounds__(kBlock) void k_residual_norm(Geom g, const float* __restrict__ b,
                                                          const float* __restrict__ q, double* __restrict__ partials,
                                                          unsigned* __restrict__ counters,
                                                          double* __restrict__ results, int pstride, int nblk) {
  __shared__ double red[kBlock / 64];
  __shared__ int sflag;
  const int ch = blockIdx.y;
  const size_t HW = (size_t)g.H * g.W;
  const size_t base = (size_t)ch * HW;
  double acc = 0.0;
  const size_t e0 = (size_t)blockIdx.x * kChunk;
  const size_t e1 = e0 + kChunk < HW ? e0 + kChunk : HW;
  for (size_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
    const double d = (double)b[base + e] - (double)q[base + e];
    acc += d * d;
  }
  const double tot = block_sum(acc, red);
  if (publish_partial(tot, partials + (size_t)ch * pstride + blockIdx.x, counters + ch, nblk, &sflag)) {
    const double s = gather_partials(partials + (size_t)ch * pstride, nblk, red);
    if (threadIdx.x == 0) {
      results[ch * kResultSlots + kSlotTrueRes] = s;
      counters[ch] = 0;
    }
  }
}

hipError_t launch_residual_norm(const Geom& g, const float* b, const float* q, double* partials,
                                unsigned* counters, double* results, hipStream_t s) {
  const size_t HW = (size_t)g.H * g.W;
  const int nblk = (int)((HW + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_residual_norm, dim3(nblk, g.N), dim3(kBlock), 0, s, g, b, q, partials, counters, results,
                     (int)max_partials_per_band(g), nblk);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------------- objective (a8) ---
// 1/2 ||D B z - X||^2 (on the low-resolution lattice) + lambda/2 sum_k min_{a,c} [sum_{i in w_k}
// (l_i - a G_i - c)^2 + eps a^2] with l = L z (eq. pansharp with the per-window optimum; equal to
// (L z)^T M_LY (L z) of eq. initialize_z_fast).  Every term is a sum of squares accumulated in FP64.

__global__ __launch_bounds__(kBlock) void k_obj_data(Geom g, const float* __restrict__ z, const float* __restrict__ X,
                                                     const float* __restrict__ u, double* __restrict__ partials,
                                                     unsigned* __restrict__ counters, double* __restrict__ results,
                                                     int pstride, int nblk) {
  __shared__ double red[kBlock / 64];
  __shared__ int sflag;
  const int ch = blockIdx.y;
  const size_t hw = (size_t)g.h * g.w;
  const float* zc = z + (size_t)ch * g.H * g.W;
  double acc = 0.0;
  const size_t e0 = (size_t)blockIdx.x * kChunk;
  const size_t e1 = e0 + kChunk < hw ? e0 + kChunk : hw;
  for (size_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
    const int m = (int)(e / g.w), k = (int)(e % g.w);
    double v = 0.0;
    for (int a = 0; a < g.n; ++a) {
      const size_t row = (size_t)wrapi(g.c * m + g.R - a, g.H) * g.W;
      for (int b = 0; b < g.n; ++b)
        v += (double)u[a * g.n + b] * (double)zc[row + wrapi(g.c * k + g.R - b, g.W)];
    }
    const double d = v - (double)X[(size_t)ch * hw + e];
    acc += d * d;
  }
  const double tot = block_sum(acc, red);
  if (publish_partial(tot, partials + (size_t)ch * pstride + blockIdx.x, counters + ch, nblk, &sflag)) {
    const double s = gather_partials(partials + (size_t)ch * pstride, nblk, red);
    if (threadIdx.x == 0) {
      results[ch * kResultSlots + kSlotObjData] = s;
      counters[ch] = 0;
    }
  }
}

__device__ __forceinline__ double lapz(const float* __restrict__ z, int i, int j, int H, int W) {
  const int im = i == 0 ? H - 1 : i - 1, ip = i == H - 1 ? 0 : i + 1;
  const int jm = j == 0 ? W - 1 : j - 1, jp = j == W - 1 ? 0 : j + 1;
  return 4.0 * (double)z[(size_t)i * W + j] - (double)z[(size_t)im * W + j] - (double)z[(size_t)ip * W + j] -
         (double)z[(size_t)i * W + jm] - (double)z[(size_t)i * W + jp];
}

__global__ __launch_bounds__(kBlock) void k_obj_llp(Geom g, const float* __restrict__ z, const float* __restrict__ G,
                                                    const float* __restrict__ MU, const float* __restrict__ DI,
                                                    double* __restrict__ partials, unsigned* __restrict__ counters,
                                                    double* __restrict__ results, int pstride, int nblk) {
  __shared__ double red[kBlock / 64];
  __shared__ int sflag;
  const int ch = blockIdx.y;
  const size_t HW = (size_t)g.H * g.W;
  const float* zc = z + (size_t)ch * HW;
  const int r = g.r;
  const double nw = (double)((2 * r + 1) * (2 * r + 1));
  double acc = 0.0;
  const size_t e0 = (size_t)blockIdx.x * kChunk;
  const size_t e1 = e0 + kChunk < HW ? e0 + kChunk : HW;
  for (size_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
    const int ki = (int)(e / g.W), kj = (int)(e % g.W);
    double sl = 0.0, sgl = 0.0;
    for (int dy = -r; dy <= r; ++dy) {
      const int i = wrapi(ki + dy, g.H);
      for (int dx = -r; dx <= r; ++dx) {
        const int j = wrapi(kj + dx, g.W);
        const double l = lapz(zc, i, j, g.H, g.W);
        sl += l;
        sgl += (double)G[(size_t)i * g.W + j] * l;
      }
    }
    const double mu = MU[e], di = DI[e];
    const double m1 = sl / nw, m2 = sgl / nw;
    const double a = (m2 - mu * m1) * di;
    const double cc = m1 - a * mu;
    double pen = (double)g.eps * a * a;
    for (int dy = -r; dy <= r; ++dy) {
      const int i = wrapi(ki + dy, g.H);
      for (int dx = -r; dx <= r; ++dx) {
        const int j = wrapi(kj + dx, g.W);
        const double res = lapz(zc, i, j, g.H, g.W) - a * (double)G[(size_t)i * g.W + j] - cc;
        pen += res * res;
      }
    }
    acc += pen;
  }
  const double tot = block_sum(acc, red);
  if (publish_partial(tot, partials + (size_t)ch * pstride + blockIdx.x, counters + ch, nblk, &sflag)) {
    const double s = gather_partials(partials + (size_t)ch * pstride, nblk, red);
    if (threadIdx.x == 0) {
      results[ch * kResultSlots + kSlotObjLlp] = s;
      counters[ch] = 0;
    }
  }
}

hipError_t launch_objective(const Geom& g, const float* z, const float* X, const float* u, const float* G,
                            const float* mu, const float* dinv, double* partials, unsigned* counters,
                            double* results, hipStream_t s) {
  const int pstride = (int)max_partials_per_band(g);
  const size_t hw = (size_t)g.h * g.w, HW = (size_t)g.H * g.W;
  const int nb1 = (int)((hw + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_obj_data, dim3(nb1, g.N), dim3(kBlock), 0, s, g, z, X, u, partials, counters, results,
                     pstride, nb1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nb2 = (int)((HW + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_obj_llp, dim3(nb2, g.N), dim3(kBlock), 0, s, g, z, G, mu, dinv, partials, counters, results,
                     pstride, nb2);
  return hipGetLastError();
}

}  // namespace llp
