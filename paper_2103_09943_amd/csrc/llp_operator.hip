// The two kernels of one conjugate-gradient iteration on eq. (Z_ini_matting) (Sec. III-B):
//
//   k_dir   (per LR tile):  r_k = r_{k-1} - alpha q_{k-1},  x_k = x_{k-1} + alpha p_{k-1},  p_k = r_k + beta p_{k-1},
//                           y = D B p_k on the low-resolution lattice,  rho_k = r_k^T r_k.
//   k_apply (per HR tile):  q_k = B^T D^T y + lambda L^T M_LY L p_k,  gamma = p_k^T q_k, sigma = r_k^T q_k, tau = q^T q;
//                           alpha_k = rho_k / gamma,  beta_k = (rho_k - 2 alpha sigma + alpha^2 tau) / rho_k.
//
// beta_k is ||r_k - alpha q_k||^2 / rho_k expanded, so both reductions of an iteration close at a kernel
// boundary and no separate vector-update pass is needed; alpha uses the directly summed rho_k.  In exact
// arithmetic the iterates are those of textbook CG.
//
// Data term, spatially: D B p is n^2 taps per kept pixel; B^T D^T y is about (n/c)^2 taps per HR pixel.
// k_dir stages p_k in LDS as c x c polyphase planes so that lanes on consecutive LR columns read consecutive
// words for every tap.  k_apply evaluates B^T D^T y with every wave on one output phase (identical taps across
// lanes, kernel taps read as scalars) and consecutive lanes on consecutive LR columns.
// LLP term: M l = |w| l - G (.) S(a) - S(b) with a = (S(G l) - mu S(l)) dinv / |w|, b = S(l)/|w| - a mu and
// S the (2r+1)^2 window sum; l = L p and the final L are 5-point stencils.  All stages stay in LDS.
#include "llp_device.h"

#include <math.h>

namespace llp {

using namespace dev;


// ======================================================================================== k_dir ===



template <int C, int TYL>
__global__ __launch_bounds__(kBlock) void k_dir(Geom g, DirArgs A, const float* __restrict__ u) {
  constexpr int TXL = 64;
  extern __shared__ float smem[];
  __shared__ double red[kWaves];
  int tile, ch;
  tile_and_band(A.ntiles, g.N, blockIdx.x, tile, ch);
  const int m0 = (tile / A.tiles_x) * TYL, k0 = (tile % A.tiles_x) * TXL;
  const int H = g.H, W = g.W, n = g.n, R = g.R;
  const size_t HW = (size_t)H * W;
  float alpha = 0.0f, beta = 0.0f;
  if (A.mode != 0) {
    if (!A.st[ch].active) return;
    alpha = (float)A.st[ch].alpha;
    beta = (float)A.st[ch].beta;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int HYR = (R + C - 1) / C;
  const int PC = TXL + 2 * HYR;
  const int RH = C * (TYL + 2 * HYR), RW = C * PC;
  const int row0 = C * (m0 - HYR), col0 = C * (k0 - HYR);
  const int in_r0 = C * HYR, in_r1 = C * (HYR + TYL), in_c0 = C * HYR, in_c1 = C * (HYR + TXL);
  const bool wrapped = row0 < 0 || col0 < 0 || row0 + RH > H || col0 + RW > W;
  const size_t base = (size_t)ch * HW;

  // Phase 1: stage the direction over the tile's footprint plus halo R (periodic), as polyphase planes;
  // update x, r and write p on the tile's own pixels.
  double acc = 0.0;
  for (int row = wave; row < RH; row += kWaves) {
    const int gr = row0 + row;
    const size_t roff = base + (size_t)(wrapped ? wrapi(gr, H) : gr) * W;
    const bool own_row = row >= in_r0 && row < in_r1 && gr < H;
    float* prow = smem + (row % C) * C * A.PS + (row / C) * PC;
    for (int col = lane; col < RW; col += 64) {
      const int gc = col0 + col;
      const size_t off = roff + (wrapped ? wrapi(gc, W) : gc);
      const bool own = own_row && col >= in_c0 && col < in_c1 && gc < W;
      float v;
      if (A.mode == 0) {
        v = A.rin[off];
      } else if (A.mode == 1) {
        v = A.rin[off];
        if (own) {
          A.pout[off] = v;
          acc += (double)v * v;
        }
      } else if (A.mode == 3) {
        const float pv = A.pin[off];
        v = fmaf(beta, pv, A.rin[off]);
        if (own) {
          A.pout[off] = v;
          A.x[off] = fmaf(alpha, pv, A.x[off]);
        }
      } else {
        const float pv = A.pin[off];
        const float rn = fmaf(-alpha, A.qin[off], A.rin[off]);
        v = fmaf(beta, pv, rn);
        if (own) {
          A.rout[off] = rn;
          if (!A.final_step) A.pout[off] = v;
          A.x[off] = fmaf(alpha, pv, A.x[off]);
          acc += (double)rn * rn;
        }
      }
      prow[(col % C) * A.PS + col / C] = v;
    }
  }
  __syncthreads();

  // Phase 2: y = D B p at the tile's LR points: y[m][k] = sum_{a,b} u[a][b] p[c m + R - a][c k + R - b].
  if (!(A.mode == 2 && A.final_step)) {
    const int k = k0 + lane;
    for (int ml = wave; ml < TYL; ml += kWaves) {
      const int m = m0 + ml;
      float s = 0.0f;
      for (int a = 0; a < n; ++a) {
        const int da = R - a;
        const float* rowp = smem + pos_mod(da, C) * C * A.PS + (ml + HYR + floor_div(da, C)) * PC + HYR + lane;
        const float* urow = u + a * n;
        for (int b = 0; b < n; ++b) {
          const int db = R - b;
          s = fmaf(urow[b], rowp[pos_mod(db, C) * A.PS + floor_div(db, C)], s);
        }
      }
      if (m < g.h && k < g.w) A.y[(size_t)ch * g.h * g.w + (size_t)m * g.w + k] = s;
    }
  }

  if (A.mode == 0 || A.mode == 3) return;
  double v[1] = {acc};
  block_partials<1>(v, red, A.partials + (size_t)ch * A.pstride * 3 + tile);
}

// ====================================================================================== k_apply ===



template <int C, int TH, int TW>
__global__ __launch_bounds__(kBlock) void k_apply(Geom g, ApplyArgs A, const float* __restrict__ u) {
  static_assert(TH % C == 0 && TW % C == 0, "tile must hold whole LR cells");
  constexpr int NI = TH / C, NJ = TW / C;
  extern __shared__ float smem[];
  __shared__ double red[3 * kWaves];
  int tile, ch;
  tile_and_band(A.ntiles, g.N, blockIdx.x, tile, ch);
  const int i0 = (tile / A.tiles_x) * TH, j0 = (tile % A.tiles_x) * TW;
  const int H = g.H, W = g.W, n = g.n, R = g.R, r = g.r;
  const size_t HW = (size_t)H * W;
  if (A.mode == 1 && !A.st[ch].active) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h1 = 2 * r + 1, h2 = r + 1, E = 2 * r + 2;
  const int PW = TW + 2 * E, PH = TH + 2 * E;
  const int LW = TW + 2 * h1, LH = TH + 2 * h1;
  const int AW = TW + 2 * h2, AH = TH + 2 * h2;
  const int W3 = TW + 2;
  const int HY = (R + C - 1) / C;
  const int YW = NJ + 2 * HY, YH = NI + 2 * HY;
  const int hs = g.h, ws = g.w;
  const bool wrapped = i0 - E < 0 || j0 - E < 0 || i0 + TH + E > H || j0 + TW + E > W;
  auto goff = [&](int gi, int gj) -> size_t {
    return wrapped ? (size_t)wrapi(gi, H) * W + wrapi(gj, W) : (size_t)gi * W + gj;
  };
  float* P = smem;               // p region, later the horizontal sums, later q in phase-major order
  float* Ls = smem + A.offL;     // l = L p
  float* Xs = smem + A.offX;     // G l, later a and b, later M l
  float* Ys = smem + A.offY;     // y = D B p with halo HY

  // S1: stage p on [i0-E, i0+TH+E) x [j0-E, j0+TW+E) and y on the LR cells the tile's taps reach.
  const float* pc = A.p + (size_t)ch * HW;
  for (int row = wave; row < PH; row += kWaves) {
    for (int col = lane; col < PW; col += 64) P[row * PW + col] = pc[goff(i0 - E + row, j0 - E + col)];
  }
  {
    const float* yc = A.y + (size_t)ch * hs * ws;
    const int I0 = i0 / C - HY, J0 = j0 / C - HY;
    for (int row = wave; row < YH; row += kWaves) {
      const size_t yro = (size_t)wrapi(I0 + row, hs) * ws;
      for (int col = lane; col < YW; col += 64) Ys[row * YW + col] = yc[yro + wrapi(J0 + col, ws)];
    }
  }
  __syncthreads();

  // S2: l = L p and G l on [i0-h1, i0+TH+h1) x [j0-h1, j0+TW+h1).
  for (int row = wave; row < LH; row += kWaves) {
    for (int col = lane; col < LW; col += 64) {
      const float* c0 = P + (row + 1) * PW + col + 1;
      const float lv = 4.0f * c0[0] - c0[-PW] - c0[PW] - c0[-1] - c0[1];
      Ls[row * LW + col] = lv;
      Xs[row * LW + col] = A.G[goff(i0 - h1 + row, j0 - h1 + col)] * lv;
    }
  }
  __syncthreads();

  // S3: horizontal window sums of l and G l, columns [j0-h2, j0+TW+h2).
  float* HBl = P;
  float* HBg = P + LH * AW;
  for (int row = wave; row < LH; row += kWaves) {
    for (int col = lane; col < AW; col += 64) {
      const float* lr = Ls + row * LW + col;
      const float* gr = Xs + row * LW + col;
      float s1 = 0.0f, s2 = 0.0f;
      for (int d = 0; d <= 2 * r; ++d) {
        s1 += lr[d];
        s2 += gr[d];
      }
      HBl[row * AW + col] = s1;
      HBg[row * AW + col] = s2;
    }
  }
  __syncthreads();

  // S4: vertical window sums -> a, b on [i0-h2, i0+TH+h2) x [j0-h2, j0+TW+h2).
  const float inv_nw = 1.0f / (float)((2 * r + 1) * (2 * r + 1));
  float* As = Xs;
  float* Bs = Xs + AH * AW;
  for (int row = wave; row < AH; row += kWaves) {
    for (int col = lane; col < AW; col += 64) {
      float s1 = 0.0f, s2 = 0.0f;
      for (int d = 0; d <= 2 * r; ++d) {
        s1 += HBl[(row + d) * AW + col];
        s2 += HBg[(row + d) * AW + col];
      }
      const size_t o = goff(i0 - h2 + row, j0 - h2 + col);
      const float mu = A.MU[o], di = A.DI[o];
      const float m1 = s1 * inv_nw, m2 = s2 * inv_nw;
      const float av = (m2 - mu * m1) * di;
      As[row * AW + col] = av;
      Bs[row * AW + col] = m1 - av * mu;
    }
  }
  __syncthreads();

  // S5: horizontal window sums of a, b, columns [j0-1, j0+TW+1).
  float* HAa = P;
  float* HAb = P + AH * W3;
  for (int row = wave; row < AH; row += kWaves) {
    for (int col = lane; col < W3; col += 64) {
      const float* ar = As + row * AW + col;
      const float* br = Bs + row * AW + col;
      float s1 = 0.0f, s2 = 0.0f;
      for (int d = 0; d <= 2 * r; ++d) {
        s1 += ar[d];
        s2 += br[d];
      }
      HAa[row * W3 + col] = s1;
      HAb[row * W3 + col] = s2;
    }
  }
  __syncthreads();

  // S6: M l = |w| l - G S(a) - S(b) on [i0-1, i0+TH+1) x [j0-1, j0+TW+1).
  const float nwf = (float)((2 * r + 1) * (2 * r + 1));
  float* Ml = Xs;
  for (int row = wave; row < TH + 2; row += kWaves) {
    for (int col = lane; col < W3; col += 64) {
      float sa = 0.0f, sb = 0.0f;
      for (int d = 0; d <= 2 * r; ++d) {
        sa += HAa[(row + d) * W3 + col];
        sb += HAb[(row + d) * W3 + col];
      }
      const float lv = Ls[(row + h1 - 1) * LW + col + h1 - 1];
      const float gv = A.G[goff(i0 - 1 + row, j0 - 1 + col)];
      Ml[row * W3 + col] = nwf * lv - gv * sa - sb;
    }
  }
  __syncthreads();

  // S7: lambda L (M l) on the tile, stored in phase-major order (phase planes padded to spread banks).
  float* Q = P;
  const float lam = g.lam;
  for (int row = wave; row < TH; row += kWaves) {
    for (int col = lane; col < TW; col += 64) {
      const float* mc = Ml + (row + 1) * W3 + col + 1;
      const float ql = lam * (4.0f * mc[0] - mc[-W3] - mc[W3] - mc[-1] - mc[1]);
      Q[((row % C) * C + col % C) * A.QPS + (row / C) * NJ + col / C] = ql;
    }
  }
  __syncthreads();

  // S8: B^T D^T y, one output phase per wave: q[i][j] += sum over taps a = a0 + C t, b = b0 + C s of
  // u[a][b] y[(i + a - R)/C][(j + b - R)/C].
  for (int task = threadIdx.x; task < TH * TW; task += kBlock) {
    const int ph = task / (NI * NJ), rem = task % (NI * NJ);
    const int I = rem / NJ, J = rem % NJ;
    const int fi = ph / C, fj = ph % C;
    const int a0 = pos_mod(R - fi, C), b0 = pos_mod(R - fj, C);
    const int di = (fi + a0 - R) / C, dj = (fj + b0 - R) / C;
    float qd = 0.0f;
    const float* ybase = Ys + (I + HY + di) * YW + (J + HY + dj);
    for (int a = a0, t = 0; a < n; a += C, ++t) {
      const float* yrow = ybase + t * YW;
      const float* urow = u + a * n;
      for (int b = b0, s = 0; b < n; b += C, ++s) qd = fmaf(urow[b], yrow[s], qd);
    }
    Q[ph * A.QPS + rem] += qd;
  }
  __syncthreads();

  // S9: write q (row-major) and the partial dot products p^T q, r^T q, q^T q (p re-read from L2: the staged
  // copy was overwritten by the window sums).
  double v[3] = {0.0, 0.0, 0.0};
  float* qc = A.q + (size_t)ch * HW;
  const float* rc = A.r + (size_t)ch * HW;
  for (int row = wave; row < TH; row += kWaves) {
    const int i = i0 + row;
    if (i >= H) break;
    for (int col = lane; col < TW; col += 64) {
      const int j = j0 + col;
      if (j >= W) break;
      const float qv = Q[((row % C) * C + col % C) * A.QPS + (row / C) * NJ + col / C];
      const size_t o = (size_t)i * W + j;
      qc[o] = qv;
      if (A.mode == 1) {
        v[0] += (double)pc[o] * qv;
        v[1] += (double)rc[o] * qv;
        v[2] += (double)qv * qv;
      }
    }
  }
  if (A.mode == 0) return;
  block_partials<3>(v, red, A.partials + (size_t)ch * A.pstride * 3 + (size_t)tile * 3);
}

// ==================================================================================== launchers ===

namespace {

template <int C>
struct ApplyTiles;
template <> struct ApplyTiles<1> { static constexpr int TH[3] = {16, 32, 16}, TW[3] = {64, 64, 128}; };
template <> struct ApplyTiles<2> { static constexpr int TH[3] = {16, 32, 16}, TW[3] = {64, 64, 128}; };
template <> struct ApplyTiles<3> { static constexpr int TH[3] = {12, 24, 24}, TW[3] = {96, 48, 96}; };
template <> struct ApplyTiles<4> { static constexpr int TH[3] = {16, 32, 16}, TW[3] = {64, 64, 128}; };

size_t align4(size_t v) { return (v + 3) & ~(size_t)3; }

}  // namespace

int dir_lds_floats(int C, int TYL, int R, int* PS_out) {
  const int HYR = (R + C - 1) / C;
  const int plane = (TYL + 2 * HYR) * (64 + 2 * HYR);
  // pad each plane so that consecutive planes start 64/C banks apart (the phase-interleaved stores of a row
  // then hit distinct banks)
  const int want = (64 / C) % 64;
  int PS = plane;
  while (PS % 64 != want) ++PS;
  if (PS_out) *PS_out = PS;
  return C * C * PS;
}

int apply_lds_floats(int C, int TH, int TW, int R, int r, int* offL, int* offX, int* offY, int* QPS_out) {
  const int h1 = 2 * r + 1, h2 = r + 1, E = 2 * r + 2;
  const int PW = TW + 2 * E, PH = TH + 2 * E;
  const int LW = TW + 2 * h1, LH = TH + 2 * h1;
  const int AW = TW + 2 * h2, AH = TH + 2 * h2;
  const int HY = (R + C - 1) / C;
  const int NI = TH / C, NJ = TW / C;
  int QPS = NI * NJ;
  const int want = (64 / C) % 64;
  while (QPS % 64 != want) ++QPS;
  size_t szP = (size_t)PH * PW;
  szP = szP > (size_t)2 * LH * AW ? szP : (size_t)2 * LH * AW;
  szP = szP > (size_t)2 * AH * (TW + 2) ? szP : (size_t)2 * AH * (TW + 2);
  szP = szP > (size_t)C * C * QPS ? szP : (size_t)C * C * QPS;
  const size_t szL = (size_t)LH * LW;
  size_t szX = (size_t)LH * LW;
  szX = szX > (size_t)2 * AH * AW ? szX : (size_t)2 * AH * AW;
  szX = szX > (size_t)(TH + 2) * (TW + 2) ? szX : (size_t)(TH + 2) * (TW + 2);
  const size_t szY = (size_t)(NI + 2 * HY) * (NJ + 2 * HY);
  const size_t oL = align4(szP), oX = oL + align4(szL), oY = oX + align4(szX), tot = oY + align4(szY);
  if (offL) *offL = (int)oL;
  if (offX) *offX = (int)oX;
  if (offY) *offY = (int)oY;
  if (QPS_out) *QPS_out = QPS;
  return (int)tot;
}

int apply_tile(int C, int variant, int* TH, int* TW) {
  if (variant < 0 || variant >= kApplyVariants) return -1;
  switch (C) {
    case 1: *TH = ApplyTiles<1>::TH[variant]; *TW = ApplyTiles<1>::TW[variant]; return 0;
    case 2: *TH = ApplyTiles<2>::TH[variant]; *TW = ApplyTiles<2>::TW[variant]; return 0;
    case 3: *TH = ApplyTiles<3>::TH[variant]; *TW = ApplyTiles<3>::TW[variant]; return 0;
    case 4: *TH = ApplyTiles<4>::TH[variant]; *TW = ApplyTiles<4>::TW[variant]; return 0;
    default: return -1;
  }
}

namespace {

template <typename K>
hipError_t set_lds(K kern, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int C, int TYL>
hipError_t launch_dir_t(const Geom& g, DirArgs A, const float* u, hipStream_t s) {
  const size_t bytes = (size_t)dir_lds_floats(C, TYL, g.R, &A.PS) * sizeof(float);
  hipError_t e = set_lds(k_dir<C, TYL>, bytes);
  if (e != hipSuccess) return e;
  A.tiles_x = (g.w + 63) / 64;
  A.ntiles = A.tiles_x * ((g.h + TYL - 1) / TYL);
  hipLaunchKernelGGL((k_dir<C, TYL>), dim3(A.ntiles * g.N), dim3(kBlock), bytes, s, g, A, u);
  return hipGetLastError();
}

template <int C, int V>
hipError_t launch_apply_v(const Geom& g, ApplyArgs A, const float* u, hipStream_t s) {
  constexpr int TH = ApplyTiles<C>::TH[V], TW = ApplyTiles<C>::TW[V];
  const size_t bytes =
      (size_t)apply_lds_floats(C, TH, TW, g.R, g.r, &A.offL, &A.offX, &A.offY, &A.QPS) * sizeof(float);
  hipError_t e = set_lds(k_apply<C, TH, TW>, bytes);
  if (e != hipSuccess) return e;
  A.tiles_x = (g.W + TW - 1) / TW;
  A.ntiles = A.tiles_x * ((g.H + TH - 1) / TH);
  hipLaunchKernelGGL((k_apply<C, TH, TW>), dim3(A.ntiles * g.N), dim3(kBlock), bytes, s, g, A, u);
  return hipGetLastError();
}

template <int C>
hipError_t launch_apply_c(const Geom& g, int variant, ApplyArgs A, const float* u, hipStream_t s) {
  switch (variant) {
    case 0: return launch_apply_v<C, 0>(g, A, u, s);
    case 1: return launch_apply_v<C, 1>(g, A, u, s);
    case 2: return launch_apply_v<C, 2>(g, A, u, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

static hipError_t launch_dir_kernel(const Geom& g, const OpConfig& cfg, DirArgs A, const float* u, hipStream_t s);

hipError_t launch_dir(const Geom& g, const OpConfig& cfg, int mode, int final_step, int k_iter, const float* rin,
                      const float* qin, const float* pin, float* rout, float* pout, float* x, float* y,
                      const float* u, double* partials, ChanState* st, int max_iters, float tol, hipStream_t s) {
  DirArgs A{};
  A.mode = mode;
  A.final_step = final_step;
  A.k_iter = k_iter;
  A.rin = rin;
  A.qin = qin;
  A.pin = pin;
  A.rout = rout;
  A.pout = pout;
  A.x = x;
  A.y = y;
  A.partials = partials;
  A.st = st;
  A.pstride = (int)max_partials_per_band(g);
  (void)max_iters;
  (void)tol;
  return launch_dir_kernel(g, cfg, A, u, s);
}

int dir_ntiles(const Geom& g, const OpConfig& cfg) {
  return ((g.w + 63) / 64) * ((g.h + cfg.dir_rows - 1) / cfg.dir_rows);
}

int apply_ntiles(const Geom& g, const OpConfig& cfg) {
  if (cfg.fast && cfg.apply_variant == kSweepVariant) return sweep_ntiles(g, cfg.seg_rows);
  int TH = 16, TW = 64;
  if (cfg.fast) TH = cfg.apply_variant == 0 ? 32 : 16;
  else if (apply_tile(g.c, cfg.apply_variant, &TH, &TW) != 0) return 0;
  return ((g.W + TW - 1) / TW) * ((g.H + TH - 1) / TH);
}

static hipError_t launch_dir_kernel(const Geom& g, const OpConfig& cfg, DirArgs A, const float* u, hipStream_t s) {
  if (cfg.fast) return launch_dir_fast(g, A, cfg.dir_rows, u, s);
  const int tyl = cfg.dir_rows;
  switch (g.c * 16 + tyl) {
    case 1 * 16 + 4: return launch_dir_t<1, 4>(g, A, u, s);
    case 1 * 16 + 8: return launch_dir_t<1, 8>(g, A, u, s);
    case 2 * 16 + 4: return launch_dir_t<2, 4>(g, A, u, s);
    case 2 * 16 + 8: return launch_dir_t<2, 8>(g, A, u, s);
    case 3 * 16 + 4: return launch_dir_t<3, 4>(g, A, u, s);
    case 3 * 16 + 8: return launch_dir_t<3, 8>(g, A, u, s);
    case 4 * 16 + 4: return launch_dir_t<4, 4>(g, A, u, s);
    case 4 * 16 + 8: return launch_dir_t<4, 8>(g, A, u, s);
    default: return hipErrorInvalidValue;
  }
}

static hipError_t launch_apply_kernel(const Geom& g, const OpConfig& cfg, ApplyArgs A, const float* u,
                                      hipStream_t s);

hipError_t launch_apply(const Geom& g, const OpConfig& cfg, int mode, const float* p, const float* r,
                        const float* y, const float* u, const float* G, const float* mu, const float* dinv,
                        float* q, double* partials, ChanState* st, hipStream_t s) {
  ApplyArgs A{};
  A.mode = mode;
  A.p = p;
  A.r = r;
  A.y = y;
  A.G = G;
  A.MU = mu;
  A.DI = dinv;
  A.q = q;
  A.partials = partials;
  A.st = st;
  A.pstride = (int)max_partials_per_band(g);
  if (cfg.fast && cfg.apply_variant == kSweepVariant)
    return launch_apply_sweep(g, cfg.seg_rows, mode, p, r, y, u, G, mu, dinv, q, partials, st, s);
  return launch_apply_kernel(g, cfg, A, u, s);
}

static hipError_t launch_apply_kernel(const Geom& g, const OpConfig& cfg, ApplyArgs A, const float* u,
                                      hipStream_t s) {
  if (cfg.fast) return launch_apply_fast(g, cfg.apply_variant, A, u, s);
  switch (g.c) {
    case 1: return launch_apply_c<1>(g, cfg.apply_variant, A, u, s);
    case 2: return launch_apply_c<2>(g, cfg.apply_variant, A, u, s);
    case 3: return launch_apply_c<3>(g, cfg.apply_variant, A, u, s);
    case 4: return launch_apply_c<4>(g, cfg.apply_variant, A, u, s);
    default: return hipErrorInvalidValue;
  }
}

size_t max_partials_per_band(const Geom& g) {
  // flat kernels: one partial per 4096 pixels; k_dir: one per LR tile (>= 4 x 64 LR points);
  // k_apply: one per HR tile (>= 12 x 96 or 16 x 64 pixels)
  const size_t HW = (size_t)g.H * g.W;
  size_t m = (HW + 4095) / 4096;
  const size_t d = (size_t)((g.h + 3) / 4) * ((g.w + 63) / 64);
  if (d > m) m = d;
  for (int v = 0; v < kApplyVariants; ++v) {
    int TH = 0, TW = 0;
    if (apply_tile(g.c, v, &TH, &TW) != 0) continue;
    const size_t t = (size_t)((g.H + TH - 1) / TH) * ((g.W + TW - 1) / TW);
    if (t > m) m = t;
  }
  // column sweep: strips of at least 52 columns, segments of at least kMinSegRows rows
  const size_t sw = (size_t)((g.W + 51) / 52) * ((g.H + kMinSegRows - 1) / kMinSegRows);
  if (sw > m) m = sw;
  // preconditioner: one per LR row
  if ((size_t)g.h > m) m = g.h;
  // FP64 residual replacement: one per tile of 8 (or 16) x 64 pixels
  const size_t rt = (size_t)ref_res_blocks(g);
  if (rt > m) m = rt;
  return m;
}

}  // namespace llp
