// Fast path of the two iteration kernels (see llp_operator.hip for what they compute), specialised at compile
// time on the resolution gap C, the blur-kernel radius R = (n-1)/2 and the LLP window radius r.
//
// k_dir_fast: the n^2 taps of D B p are fully unrolled: each tap is one LDS read at an immediate offset (the
// direction is staged as C x C polyphase planes, so lanes on consecutive LR columns read consecutive words)
// and one FMA with the tap held in a scalar register.  Each lane computes two LR points.
//
// k_apply_fast: the LLP window sums run as register strips of K outputs over layouts that alternate between
// row-major and transposed, so every strip reads consecutive words across lanes and each input word is read
// about (K + 2r)/K times instead of 2r+1 times.  B^T D^T y is evaluated per LR cell: a thread holds the
// (2 floor(R/C) + 1)^2 neighbourhood of y in registers and forms the C x C outputs of its cell from it; the
// cell's q is then written with one vector store per row.
#include "llp_fast_util.h"

#include <math.h>

namespace llp {
using namespace dev;


// ==================================================================================== k_dir_fast ===

// Words per polyphase plane: the C planes a row of the region is dealt to must start an odd multiple of 64/C
// banks apart, so that the 64 lanes of one LDS store hit distinct banks.
constexpr int phase_stride(int v, int C) {
  return ((v % 64) % (64 / C) == 0 && ((v % 64) / (64 / C)) % 2 == 1) ? v : pad_to(v, (64 / C) % 64);
}

// One LR row of the tile per wave: TYL = 4 runs 4 waves (256 threads), TYL = 8 runs 8 waves (512 threads).
template <int C, int R, int TYL_ = 4>
struct DirShape {
  static constexpr int TYL = TYL_, TXL = 64, NW = TYL_;
  static constexpr int HYR = (R + C - 1) / C;
  static constexpr int PR = TYL + 2 * HYR, PC = TXL + 2 * HYR;
  static constexpr int PS = phase_stride(PR * PC, C);
  static constexpr int RH = C * PR, RW = C * PC;
  static constexpr int LDS = C * C * PS;
  static constexpr int LDS_ALLOC = LDS + 64;  // plus one slot per lane for the stores of lanes past the region
  static_assert(NW == 4 || NW == 8, "4 or 8 LR rows per tile");
};

// Byte offset past every plane: buffer loads from it return 0 and stores to it are dropped (the planes of the
// fast path hold fewer than 2^29 floats).
constexpr unsigned kNoAccess = 0x80000000u;

template <int C, int R, int TYL, int MODE>
__device__ __forceinline__ void dir_fast_body(const Geom& g, const DirArgs& A, const float* __restrict__ u, int bid) {
  using S = DirShape<C, R, TYL>;
  constexpr int n = 2 * R + 1, NW = S::NW;
  extern __shared__ float smem[];
  __shared__ double red[NW];
  int tile, ch;
  tile_and_band(A.ntiles, g.N, bid, tile, ch);
  const int m0 = (tile / A.tiles_x) * S::TYL, k0 = (tile % A.tiles_x) * S::TXL;
  const int H = g.H, W = g.W;
  const size_t HW = (size_t)H * W;
  float alpha = 0.0f, beta = 0.0f;
  if (MODE != 0) {
    if (!A.st[ch].active) return;
    alpha = (float)A.st[ch].alpha;
    beta = (float)A.st[ch].beta;
  }
  // the wave index is uniform: rows, and the row offsets of every access, stay in scalar registers
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int row0 = C * (m0 - S::HYR), col0 = C * (k0 - S::HYR);
  constexpr int in_r0 = C * S::HYR, in_r1 = C * (S::HYR + S::TYL), in_c0 = C * S::HYR, in_c1 = C * (S::HYR + S::TXL);
  // Per-band planes through buffer resources: the row is a scalar byte offset, the lane's column a vector one;
  // lanes past the region or outside the tile's own pixels use kNoAccess instead of branching.
  const unsigned plane = (unsigned)(HW * 4);
  auto rsrc = [&](const float* base) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)(base + (size_t)ch * HW), (short)0, (int)plane, 0x00020000);
  };
  auto ld = [](__amdgpu_buffer_rsrc_t rs, unsigned vo, unsigned so) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, 0));
  };
  auto st = [](float v, __amdgpu_buffer_rsrc_t rs, unsigned vo, unsigned so) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rs, vo, so, 0);
  };
  const __amdgpu_buffer_rsrc_t Rr = rsrc(A.rin);
  const __amdgpu_buffer_rsrc_t Rq = rsrc(MODE == 2 ? A.qin : A.rin), Rp = rsrc(MODE >= 2 ? A.pin : A.rin);
  const __amdgpu_buffer_rsrc_t Rro = rsrc(MODE == 2 ? A.rout : A.rin), Rx = rsrc(MODE >= 2 ? A.x : A.rin);
  const __amdgpu_buffer_rsrc_t Rpo = rsrc(MODE != 0 ? A.pout : A.rin);

  // Column offsets of this lane (the same for every row of the region).
  constexpr int NCI = (S::RW + 63) / 64;
  unsigned vld[NCI], vown[NCI];
  int lcol[NCI];
#pragma unroll
  for (int ci = 0; ci < NCI; ++ci) {
    const int col = ci * 64 + lane;
    const int gc = col0 + col;
    const bool valid = col < S::RW;
    const bool own = valid && col >= in_c0 && col < in_c1 && gc < W;
    const unsigned cb = (unsigned)wrap1(gc, W) * 4u;
    vld[ci] = valid ? cb : kNoAccess;
    vown[ci] = own ? cb : kNoAccess;
    lcol[ci] = valid ? (col % C) * S::PS + col / C : -1;
  }
  double acc = 0.0;
  constexpr int RPI = 2;  // region rows per wave per iteration (their loads are in flight together)
  for (int row_b = wave; row_b < S::RH; row_b += NW * RPI) {
    float rv[RPI][NCI], qv[RPI][NCI], pv[RPI][NCI], xv[RPI][NCI];
    unsigned so[RPI];
#pragma unroll
    for (int j = 0; j < RPI; ++j) {
      const int row = row_b + j * NW;
      const int gr = row0 + row;
      so[j] = (unsigned)(wrap1(gr, H) * W) * 4u;
      const bool own_row = row >= in_r0 && row < in_r1 && gr < H;
      if (row < S::RH) {
#pragma unroll
        for (int ci = 0; ci < NCI; ++ci) {
          rv[j][ci] = ld(Rr, vld[ci], so[j]);
          if (MODE == 2) qv[j][ci] = ld(Rq, vld[ci], so[j]);
          if (MODE >= 2) pv[j][ci] = ld(Rp, vld[ci], so[j]);
        }
        if (MODE >= 2 && own_row) {
#pragma unroll
          for (int ci = 0; ci < NCI; ++ci) xv[j][ci] = ld(Rx, vown[ci], so[j]);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < RPI; ++j) {
      const int row = row_b + j * NW;
      if (row >= S::RH) continue;
      const int gr = row0 + row;
      const bool own_row = row >= in_r0 && row < in_r1 && gr < H;
      float* prow = smem + (row % C) * C * S::PS + (row / C) * S::PC;
      float vv[NCI];
#pragma unroll
      for (int ci = 0; ci < NCI; ++ci)
        vv[ci] = MODE == 2   ? fmaf(beta, pv[j][ci], fmaf(-alpha, qv[j][ci], rv[j][ci]))
                 : MODE == 3 ? fmaf(beta, pv[j][ci], rv[j][ci])
                             : rv[j][ci];
      if (MODE != 0 && own_row) {
#pragma unroll
        for (int ci = 0; ci < NCI; ++ci) {
          if (MODE == 1) {
            st(vv[ci], Rpo, vown[ci], so[j]);
            acc += (double)(vown[ci] != kNoAccess ? vv[ci] * vv[ci] : 0.0f);
          } else if (MODE == 3) {
            st(vv[ci], Rpo, vown[ci], so[j]);
            st(fmaf(alpha, pv[j][ci], xv[j][ci]), Rx, vown[ci], so[j]);
          } else {
            const float rn = fmaf(-alpha, qv[j][ci], rv[j][ci]);
            st(rn, Rro, vown[ci], so[j]);
            if (!A.final_step) st(vv[ci], Rpo, vown[ci], so[j]);
            st(fmaf(alpha, pv[j][ci], xv[j][ci]), Rx, vown[ci], so[j]);
            acc += (double)(vown[ci] != kNoAccess ? rn * rn : 0.0f);
          }
        }
      }
#pragma unroll
      for (int ci = 0; ci < NCI; ++ci) {
        float* dst = lcol[ci] >= 0 ? prow + lcol[ci] : smem + S::LDS + lane;
        *dst = vv[ci];
      }
    }
  }
  __syncthreads();

  if (!(MODE == 2 && A.final_step)) {
    // y[m][k] = sum_{a,b} u[a][b] p[C m + R - a][C k + R - b] on LR row m0 + wave, column k0 + lane.
    // Every tap is one LDS read at an immediate offset from the lane's base and one FMA with the tap in a
    // scalar register.
    constexpr int MPW = TYL / NW;
    const float* b0 = smem + (S::HYR + wave) * S::PC + S::HYR + lane;
    float sacc[MPW];
#pragma unroll
    for (int m = 0; m < MPW; ++m) sacc[m] = 0.0f;
#pragma unroll
    for (int a = 0; a < n; ++a) {
      const float* rowp = b0 + cpmod(R - a, C) * C * S::PS + cfdiv(R - a, C) * S::PC;
      const float* urow = u + a * n;
#pragma unroll
      for (int b = 0; b < n; ++b) {
        const int off = cpmod(R - b, C) * S::PS + cfdiv(R - b, C);
        const float w = urow[b];
#pragma unroll
        for (int m = 0; m < MPW; ++m) sacc[m] = fmaf(w, rowp[off + m * NW * S::PC], sacc[m]);
      }
    }
    const int k = k0 + lane;
    const __amdgpu_buffer_rsrc_t Ry = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(A.y + (size_t)ch * g.h * g.w), (short)0, (int)((size_t)g.h * g.w * 4), 0x00020000);
    const unsigned ko = k < g.w ? (unsigned)k * 4u : kNoAccess;
#pragma unroll
    for (int m = 0; m < MPW; ++m) {
      const int mm = m0 + wave + m * NW;
      if (mm < g.h) st(sacc[m], Ry, ko, (unsigned)(mm * g.w) * 4u);
    }
  }

  if (MODE == 0 || MODE == 3) return;
  double v[1] = {acc};
  block_partials<1, NW>(v, red, A.partials + (size_t)ch * A.pstride * 3 + tile);
}

// ================================================================================== k_apply_fast ===

template <int C, int R, int r, int TH, int TW>
struct ApplyShape {
  static constexpr int K = 8;  // strip length
  static constexpr int E = 2 * r + 2, h1 = 2 * r + 1, h2 = r + 1, WN = 2 * r + 1;
  static constexpr int PH = TH + 2 * E, PW = TW + 2 * E;
  static constexpr int LH = TH + 2 * h1, LW = TW + 2 * h1, LHs = odd(LH);
  static constexpr int AH = TH + 2 * h2, AW = TW + 2 * h2, AHs = odd(AH), AWs = odd(AW);
  static constexpr int H3 = TH + 2, W3 = TW + 2, W3s = odd(W3);
  static constexpr int NI = TH / C, NJ = TW / C;
  static constexpr int YL = R / C, YR = (C - 1 + R) / C, YK = YL + YR + 1;
  static constexpr int YH = NI + YL + YR, YW = NJ + YL + YR, YWs = odd(YW);
  static constexpr int CS = C == 4 ? 20 : C * C;  // floats per LR cell in the phase-blocked q layout
  // strip counts of the five window stages
  static constexpr int NS2 = (LH + K - 1) / K, NS3 = (AW + K - 1) / K, NS4 = (AH + K - 1) / K,
                       NS5 = (W3 + K - 1) / K, NS6 = (H3 + K - 1) / K;
  // allocated extents (the last strip of each stage may read past the valid extent)
  static constexpr int PHa = cmax(PH, NS2 * K + 2);
  static constexpr int LWa = cmax(LW, NS3 * K + 2 * r);
  static constexpr int LHa = cmax(LH, NS4 * K + 2 * r);
  static constexpr int AWa = cmax(AW, NS5 * K + 2 * r);
  static constexpr int AHa = cmax(AH, NS6 * K + 2 * r);
  static constexpr int szR1 = cmax(PHa * PW, cmax(2 * LHa * AWs, 2 * AHa * W3s));
  static constexpr int szL = LWa * LHs;
  static constexpr int szR2 = cmax(LWa * LHs, cmax(2 * AWa * AHs, cmax(H3 * W3s, NI * NJ * CS)));
  static constexpr int szY = YH * YWs;
  static constexpr int oL = al4(szR1), oR2 = oL + al4(szL), oY = oR2 + al4(szR2), total = oY + al4(szY);
  static constexpr int SPLIT = (NI * NJ >= kBlock) ? 1 : (kBlock / (NI * NJ) >= C ? C : kBlock / (NI * NJ));
  static constexpr int CR = C / SPLIT;  // output rows of a cell per thread in the final stage
};

// Sliding window sums of width WN over v[0 .. K+WN-1): out[t] = sum_{d < WN} v[t+d].
template <int K, int WN>
__device__ __forceinline__ void window_sums(const float (&v)[K + WN - 1], float (&out)[K]) {
  float s = 0.0f;
#pragma unroll
  for (int d = 0; d < WN; ++d) s += v[d];
  out[0] = s;
#pragma unroll
  for (int t = 1; t < K; ++t) {
    s += v[t + WN - 1] - v[t - 1];
    out[t] = s;
  }
}

template <int C, int R, int r, int TH, int TW, int MODE>
__device__ __forceinline__ void apply_fast_body(const Geom& g, const ApplyArgs& A, const float* __restrict__ u,
                                                int bid) {
  using S = ApplyShape<C, R, r, TH, TW>;
  constexpr int K = S::K, WN = S::WN;
  extern __shared__ float smem[];
  __shared__ double red[3 * kWaves];
  int tile, ch;
  tile_and_band(A.ntiles, g.N, bid, tile, ch);
  const int i0 = (tile / A.tiles_x) * TH, j0 = (tile % A.tiles_x) * TW;
  const int H = g.H, W = g.W;
  const size_t HW = (size_t)H * W;
  if (MODE == 1 && !A.st[ch].active) return;
  // 32-bit unsigned element offsets within a plane (H W <= 2^31), so loads take a scalar base plus a vector
  // offset.
  auto goff = [&](int gi, int gj) -> unsigned { return (unsigned)(wrap1(gi, H) * W + wrap1(gj, W)); };
  const float* __restrict__ Gp = A.G;
  const float* __restrict__ MUp = A.MU;
  const float* __restrict__ DIp = A.DI;
  float* R1 = smem;              // p region -> horizontal sums of (l, G l) -> horizontal sums of (a, b)
  float* LT = smem + S::oL;      // l = L p, transposed
  float* R2 = smem + S::oR2;     // G l (transposed) -> a, b (transposed) -> M l -> lambda L M l (cell-blocked)
  float* Ys = smem + S::oY;      // y on the LR cells the tile's taps reach
  const float* pc = A.p + (size_t)ch * HW;

  // Prefetch: every global value this thread will need in the later stages is requested now, so that the
  // workgroup waits for global memory once instead of once per stage (barriers do not wait for these loads).
  constexpr int T2 = S::LW * S::NS2, T4 = S::AW * S::NS4, T6 = S::W3 * S::NS6, T8 = S::NI * S::NJ * S::SPLIT;
  constexpr int NT2 = (T2 + kBlock - 1) / kBlock, NT4 = (T4 + kBlock - 1) / kBlock, NT6 = (T6 + kBlock - 1) / kBlock,
                NT8 = (T8 + kBlock - 1) / kBlock;
  float g2[NT2][K], mu4[NT4][K], di4[NT4][K], g6[NT6][K];
#pragma unroll
  for (int k = 0; k < NT2; ++k) {
    const int task = min((int)threadIdx.x + k * kBlock, T2 - 1);
    const int col = task % S::LW, y0 = (task / S::LW) * K;
    const int gcj = wrap1(j0 - S::h1 + col, W);
#pragma unroll
    for (int t = 0; t < K; ++t) g2[k][t] = Gp[(unsigned)(wrap1(i0 - S::h1 + min(y0 + t, S::LH - 1), H) * W + gcj)];
  }
#pragma unroll
  for (int k = 0; k < NT4; ++k) {
    const int task = min((int)threadIdx.x + k * kBlock, T4 - 1);
    const int col = task % S::AW, y0 = (task / S::AW) * K;
    const int gcj = wrap1(j0 - S::h2 + col, W);
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const unsigned o = (unsigned)(wrap1(i0 - S::h2 + min(y0 + t, S::AH - 1), H) * W + gcj);
      mu4[k][t] = MUp[o];
      di4[k][t] = DIp[o];
    }
  }
#pragma unroll
  for (int k = 0; k < NT6; ++k) {
    const int task = min((int)threadIdx.x + k * kBlock, T6 - 1);
    const int col = task % S::W3, y0 = (task / S::W3) * K;
    const int gcj = wrap1(j0 - 1 + col, W);
#pragma unroll
    for (int t = 0; t < K; ++t) g6[k][t] = Gp[(unsigned)(wrap1(i0 - 1 + min(y0 + t, S::H3 - 1), H) * W + gcj)];
  }
  float p8[NT8][S::CR][C], r8[NT8][S::CR][C];
  if (MODE == 1) {
    const float* rc0 = A.r + (size_t)ch * HW;
#pragma unroll
    for (int k = 0; k < NT8; ++k) {
      const int task = min((int)threadIdx.x + k * kBlock, T8 - 1);
      const int J = task % S::NJ, I = (task / S::NJ) % S::NI, part = task / (S::NI * S::NJ);
      const int j = min(j0 + C * J, W - C);
#pragma unroll
      for (int f = 0; f < S::CR; ++f) {
        const int i = min(i0 + C * I + part * S::CR + f, H - 1);
        const unsigned o = (unsigned)(i * W + j);
#pragma unroll
        for (int fj = 0; fj < C; ++fj) {
          p8[k][f][fj] = pc[o + fj];
          r8[k][f][fj] = rc0[o + fj];
        }
      }
    }
  }

  // S1: stage p on [i0-E, i0+TH+E) x [j0-E, j0+TW+E) (rows by wave, columns by lane; the row offset is a
  // scalar, the lane's column indices are computed once) and y on LR [i0/C-YL, i0/C+NI+YR) x [...].
  {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NCI = (S::PW + 63) / 64;
    int pcol[NCI];
#pragma unroll
    for (int ci = 0; ci < NCI; ++ci) pcol[ci] = wrap1(j0 - S::E + min(ci * 64 + lane, S::PW - 1), W);
    constexpr int RPW = (S::PH + kWaves - 1) / kWaves;
    float pv[RPW][NCI];
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int row = wave + k * kWaves;
      const unsigned ro = (unsigned)(wrap1(i0 - S::E + min(row, S::PH - 1), H) * W);
#pragma unroll
      for (int ci = 0; ci < NCI; ++ci) pv[k][ci] = pc[ro + (unsigned)pcol[ci]];
    }
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int row = wave + k * kWaves;
#pragma unroll
      for (int ci = 0; ci < NCI; ++ci) {
        const int col = ci * 64 + lane;
        if (row < S::PH && col < S::PW) R1[row * S::PW + col] = pv[k][ci];
      }
    }
  }
  {
    const float* yc = A.y + (size_t)ch * g.h * g.w;
    const int I0 = i0 / C - S::YL, J0 = j0 / C - S::YL;
    for (int idx = threadIdx.x; idx < S::YH * S::YW; idx += kBlock) {
      const int row = idx / S::YW, col = idx % S::YW;
      Ys[row * S::YWs + col] = yc[(unsigned)(wrap1(I0 + row, g.h) * g.w + wrap1(J0 + col, g.w))];
    }
  }
  __syncthreads();

  // S2: l = L p (and G l) on rows [-h1, TH+h1), cols [-h1, TW+h1); column strips of K rows, stored transposed.
#pragma unroll
  for (int kt = 0; kt < NT2; ++kt) {
    const int task = threadIdx.x + kt * kBlock;
    if (task >= T2) break;
    const int col = task % S::LW, y0 = (task / S::LW) * K;
    float cv[K + 2], lv[K], rv[K];
#pragma unroll
    for (int t = 0; t < K + 2; ++t) cv[t] = R1[(y0 + t) * S::PW + col + 1];
#pragma unroll
    for (int t = 0; t < K; ++t) {
      lv[t] = R1[(y0 + t + 1) * S::PW + col];
      rv[t] = R1[(y0 + t + 1) * S::PW + col + 2];
    }
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int y = y0 + t;
      if (y < S::LH) {
        const float l = 4.0f * cv[t + 1] - cv[t] - cv[t + 2] - lv[t] - rv[t];
        LT[col * S::LHs + y] = l;
        R2[col * S::LHs + y] = g2[kt][t] * l;
      }
    }
  }
  __syncthreads();

  // S3: horizontal window sums of l and G l: cols [-h2, TW+h2), row strips of K columns; row-major out.
  float* HB1 = R1;
  float* HB2 = R1 + S::LHa * S::AWs;
  for (int task = threadIdx.x; task < S::LH * S::NS3; task += kBlock) {
    const int row = task % S::LH, x0 = (task / S::LH) * K;
    float v1[K + WN - 1], v2[K + WN - 1], o1[K], o2[K];
#pragma unroll
    for (int t = 0; t < K + WN - 1; ++t) {
      v1[t] = LT[(x0 + t) * S::LHs + row];
      v2[t] = R2[(x0 + t) * S::LHs + row];
    }
    window_sums<K, WN>(v1, o1);
    window_sums<K, WN>(v2, o2);
#pragma unroll
    for (int t = 0; t < K; ++t) {
      if (x0 + t < S::AW) {
        HB1[row * S::AWs + x0 + t] = o1[t];
        HB2[row * S::AWs + x0 + t] = o2[t];
      }
    }
  }
  __syncthreads();

  // S4: vertical window sums -> a, b on rows [-h2, TH+h2), cols [-h2, TW+h2); column strips, transposed out.
  constexpr float inv_nw = 1.0f / (float)(WN * WN);
  float* AT = R2;
  float* BT = R2 + S::AWa * S::AHs;
#pragma unroll
  for (int kt = 0; kt < NT4; ++kt) {
    const int task = threadIdx.x + kt * kBlock;
    if (task >= T4) break;
    const int col = task % S::AW, y0 = (task / S::AW) * K;
    float v1[K + WN - 1], v2[K + WN - 1], o1[K], o2[K];
#pragma unroll
    for (int t = 0; t < K + WN - 1; ++t) {
      v1[t] = HB1[(y0 + t) * S::AWs + col];
      v2[t] = HB2[(y0 + t) * S::AWs + col];
    }
    window_sums<K, WN>(v1, o1);
    window_sums<K, WN>(v2, o2);
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int y = y0 + t;
      if (y < S::AH) {
        const float mu = mu4[kt][t], di = di4[kt][t];
        const float m1 = o1[t] * inv_nw, m2 = o2[t] * inv_nw;
        const float av = (m2 - mu * m1) * di;
        AT[col * S::AHs + y] = av;
        BT[col * S::AHs + y] = m1 - av * mu;
      }
    }
  }
  __syncthreads();

  // S5: horizontal window sums of a, b: cols [-1, TW+1); row strips, row-major out.
  float* HA1 = R1;
  float* HA2 = R1 + S::AHa * S::W3s;
  for (int task = threadIdx.x; task < S::AH * S::NS5; task += kBlock) {
    const int row = task % S::AH, x0 = (task / S::AH) * K;
    float v1[K + WN - 1], v2[K + WN - 1], o1[K], o2[K];
#pragma unroll
    for (int t = 0; t < K + WN - 1; ++t) {
      v1[t] = AT[(x0 + t) * S::AHs + row];
      v2[t] = BT[(x0 + t) * S::AHs + row];
    }
    window_sums<K, WN>(v1, o1);
    window_sums<K, WN>(v2, o2);
#pragma unroll
    for (int t = 0; t < K; ++t) {
      if (x0 + t < S::W3) {
        HA1[row * S::W3s + x0 + t] = o1[t];
        HA2[row * S::W3s + x0 + t] = o2[t];
      }
    }
  }
  __syncthreads();

  // S6: M l = |w| l - G S(a) - S(b) on rows [-1, TH+1), cols [-1, TW+1); column strips, row-major out.
  constexpr float nwf = (float)(WN * WN);
  float* Ml = R2;
#pragma unroll
  for (int kt = 0; kt < NT6; ++kt) {
    const int task = threadIdx.x + kt * kBlock;
    if (task >= T6) break;
    const int col = task % S::W3, y0 = (task / S::W3) * K;
    float v1[K + WN - 1], v2[K + WN - 1], o1[K], o2[K];
#pragma unroll
    for (int t = 0; t < K + WN - 1; ++t) {
      v1[t] = HA1[(y0 + t) * S::W3s + col];
      v2[t] = HA2[(y0 + t) * S::W3s + col];
    }
    window_sums<K, WN>(v1, o1);
    window_sums<K, WN>(v2, o2);
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int y = y0 + t;
      if (y < S::H3) {
        const float l = LT[(col - 1 + S::h1) * S::LHs + (y - 1 + S::h1)];
        Ml[y * S::W3s + col] = nwf * l - g6[kt][t] * o1[t] - o2[t];
      }
    }
  }
  __syncthreads();

  // S7: lambda L (M l) on the tile, row-major in, stored cell-blocked (cell (I, J) at (I NJ + J) CS).
  constexpr int NQ = (TH * TW + kBlock - 1) / kBlock;
  float ql_reg[NQ];
  const float lam = g.lam;
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int idx = threadIdx.x + k * kBlock;
    if (idx < TH * TW) {
      const int row = idx / TW, col = idx % TW;
      const float* mc = Ml + (row + 1) * S::W3s + col + 1;
      ql_reg[k] = lam * (4.0f * mc[0] - mc[-S::W3s] - mc[S::W3s] - mc[-1] - mc[1]);
    }
  }
  __syncthreads();  // Ml and the cell-blocked buffer share R2
  float* QL = R2;
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int idx = threadIdx.x + k * kBlock;
    if (idx < TH * TW) {
      const int row = idx / TW, col = idx % TW;
      QL[((row / C) * S::NJ + col / C) * S::CS + (row % C) * C + (col % C)] = ql_reg[k];
    }
  }
  __syncthreads();

  // S8: per LR cell: q = B^T D^T y + lambda L M l, written row by row; partial p^T q, r^T q, q^T q.
  double v[3] = {0.0, 0.0, 0.0};
  float* qc = A.q + (size_t)ch * HW;
#pragma unroll
  for (int kt = 0; kt < NT8; ++kt) {
    const int task = threadIdx.x + kt * kBlock;
    if (task >= T8) break;
    const int J = task % S::NJ, I = (task / S::NJ) % S::NI, part = task / (S::NI * S::NJ);
    float yv[S::YK][S::YK];
#pragma unroll
    for (int dy = 0; dy < S::YK; ++dy)
#pragma unroll
      for (int dx = 0; dx < S::YK; ++dx) yv[dy][dx] = Ys[(I + dy) * S::YWs + J + dx];
    float qd[S::CR][C];
    if constexpr (S::SPLIT == 1) {
      cell_data_term<C, R, S::YK, S::YL, 0, S::CR>(yv, u, qd);
    } else if constexpr (S::SPLIT == 2) {
      if (part == 0) cell_data_term<C, R, S::YK, S::YL, 0, S::CR>(yv, u, qd);
      else cell_data_term<C, R, S::YK, S::YL, S::CR, S::CR>(yv, u, qd);
    } else {
      static_assert(S::SPLIT == C, "cells split by single rows");
      switch (part) {
        case 0: cell_data_term<C, R, S::YK, S::YL, 0, 1>(yv, u, qd); break;
        case 1: cell_data_term<C, R, S::YK, S::YL, 1 % C, 1>(yv, u, qd); break;
        case 2: cell_data_term<C, R, S::YK, S::YL, 2 % C, 1>(yv, u, qd); break;
        default: cell_data_term<C, R, S::YK, S::YL, 3 % C, 1>(yv, u, qd); break;
      }
    }
    const float* qlc = QL + (I * S::NJ + J) * S::CS;
    const int j = j0 + C * J;
#pragma unroll
    for (int f = 0; f < S::CR; ++f) {
      const int fi = part * S::CR + f;
      const int i = i0 + C * I + fi;
      float qv[C];
#pragma unroll
      for (int fj = 0; fj < C; ++fj) qv[fj] = qd[f][fj] + qlc[fi * C + fj];
      if (i < H && j < W) {
        const unsigned o = (unsigned)(i * W + j);
        if constexpr (C == 4) {
          *reinterpret_cast<float4*>(qc + o) = make_float4(qv[0], qv[1], qv[2], qv[3]);
        } else if constexpr (C == 2) {
          *reinterpret_cast<float2*>(qc + o) = make_float2(qv[0], qv[1]);
        } else {
#pragma unroll
          for (int fj = 0; fj < C; ++fj) qc[o + fj] = qv[fj];
        }
        if (MODE == 1) {
#pragma unroll
          for (int fj = 0; fj < C; ++fj) {
            v[0] += (double)p8[kt][f][fj] * qv[fj];
            v[1] += (double)r8[kt][f][fj] * qv[fj];
          }
        }
        if (MODE == 1) {
#pragma unroll
          for (int fj = 0; fj < C; ++fj) v[2] += (double)qv[fj] * qv[fj];
        }
      }
    }
  }
  if (MODE == 0) return;
  block_partials<3>(v, red, A.partials + (size_t)ch * A.pstride * 3 + (size_t)tile * 3);
}

// ================================================================================ kernel wrappers ===

template <int C, int R, int TYL, int MODE>
__global__ __launch_bounds__(TYL * 64) void k_dir_fast(Geom g, DirArgs A, const float* __restrict__ u) {
  dir_fast_body<C, R, TYL, MODE>(g, A, u, blockIdx.x);
}

template <int C, int R, int r, int TH, int TW, int MODE>
__global__ __launch_bounds__(kBlock) void k_apply_fast(Geom g, ApplyArgs A, const float* __restrict__ u) {
  apply_fast_body<C, R, r, TH, TW, MODE>(g, A, u, blockIdx.x);
}

// Scene of workgroup b: the last table entry whose first block is <= b.
template <bool kDir>
__device__ __forceinline__ int find_scene(const SceneDesc* __restrict__ t, int count, int b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int b0 = kDir ? t[mid].dir_block0 : t[mid].apply_block0;
    if (b0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Batched CG iteration kernels (mode 2 or 3 / mode 1 of the single-scene kernels) over a table of scenes.
template <int C, int R, int TYL, int MODE>
__global__ __launch_bounds__(TYL * 64) void k_dir_fast_batch(const SceneDesc* __restrict__ t, int count, int parity,
                                                           ChanState* __restrict__ st, char* __restrict__ ws,
                                                           const float* __restrict__ taps) {
  const int si = find_scene<true>(t, count, blockIdx.x);
  const SceneDesc& d = t[si];
  const int local = blockIdx.x - d.dir_block0;  // scenes start on multiples of 8 workgroups (one per XCD)
  if (local >= d.dir_ntiles * d.g.N) return;
  DirArgs A{};
  A.mode = MODE;
  A.rin = (const float*)(ws + (MODE == 3 ? d.o_s : d.o_r[parity]));
  A.qin = (const float*)(ws + d.o_q);
  A.pin = (const float*)(ws + d.o_p[parity]);
  A.rout = (float*)(ws + d.o_r[1 - parity]);
  A.pout = (float*)(ws + d.o_p[1 - parity]);
  A.x = (float*)(ws + d.o_x);
  A.y = (float*)(ws + d.o_y);
  A.partials = (double*)(ws + d.o_partials);
  A.st = st + d.band0;
  A.pstride = d.pstride;
  A.tiles_x = (d.g.w + DirShape<C, R, TYL>::TXL - 1) / DirShape<C, R, TYL>::TXL;
  A.ntiles = d.dir_ntiles;
  A.PS = DirShape<C, R, TYL>::PS;
  dir_fast_body<C, R, TYL, MODE>(d.g, A, taps + (size_t)d.taps_index * kTapStride, local);
}

template <int C, int R, int r, int TH, int TW>
__global__ __launch_bounds__(kBlock) void k_apply_fast_batch(const SceneDesc* __restrict__ t, int count, int parity,
                                                             ChanState* __restrict__ st, char* __restrict__ ws,
                                                             const float* __restrict__ taps) {
  const int si = find_scene<false>(t, count, blockIdx.x);
  const SceneDesc& d = t[si];
  const int local = blockIdx.x - d.apply_block0;
  if (local >= d.apply_ntiles * d.g.N) return;
  ApplyArgs A{};
  A.mode = 1;
  A.p = (const float*)(ws + d.o_p[parity]);
  A.r = (const float*)(ws + d.o_r[parity]);
  A.y = (const float*)(ws + d.o_y);
  A.G = (const float*)(ws + d.o_G);
  A.MU = (const float*)(ws + d.o_MU);
  A.DI = (const float*)(ws + d.o_DI);
  A.q = (float*)(ws + d.o_q);
  A.partials = (double*)(ws + d.o_partials);
  A.st = st + d.band0;
  A.pstride = d.pstride;
  A.tiles_x = (d.g.W + TW - 1) / TW;
  A.ntiles = d.apply_ntiles;
  apply_fast_body<C, R, r, TH, TW, 1>(d.g, A, taps + (size_t)d.taps_index * kTapStride, local);
}

// ===================================================================================== dispatch ===

namespace {

template <typename Kern>
hipError_t set_lds_fast(Kern kern, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int C, int R, int TYL, int MODE>
hipError_t run_dir_fast_m(const Geom& g, DirArgs A, const float* u, hipStream_t s) {
  using S = DirShape<C, R, TYL>;
  const size_t bytes = (size_t)S::LDS_ALLOC * sizeof(float);
  hipError_t e = set_lds_fast(k_dir_fast<C, R, TYL, MODE>, bytes);
  if (e != hipSuccess) return e;
  A.PS = S::PS;
  A.tiles_x = (g.w + S::TXL - 1) / S::TXL;
  A.ntiles = A.tiles_x * ((g.h + S::TYL - 1) / S::TYL);
  hipLaunchKernelGGL((k_dir_fast<C, R, TYL, MODE>), dim3(A.ntiles * g.N), dim3(S::NW * 64), bytes, s, g, A, u);
  return hipGetLastError();
}

template <int C, int R, int TYL>
hipError_t run_dir_fast_t(const Geom& g, DirArgs A, const float* u, hipStream_t s) {
  switch (A.mode) {
    case 0: return run_dir_fast_m<C, R, TYL, 0>(g, A, u, s);
    case 1: return run_dir_fast_m<C, R, TYL, 1>(g, A, u, s);
    case 3: return run_dir_fast_m<C, R, TYL, 3>(g, A, u, s);
    default: return run_dir_fast_m<C, R, TYL, 2>(g, A, u, s);
  }
}

template <int C, int R>
hipError_t run_dir_fast(const Geom& g, DirArgs A, int tyl, const float* u, hipStream_t s) {
  return tyl == 8 ? run_dir_fast_t<C, R, 8>(g, A, u, s) : run_dir_fast_t<C, R, 4>(g, A, u, s);
}

template <int C, int R, int r, int TH, int TW, int MODE>
hipError_t run_apply_fast_m(const Geom& g, ApplyArgs A, const float* u, hipStream_t s) {
  using S = ApplyShape<C, R, r, TH, TW>;
  const size_t bytes = (size_t)S::total * sizeof(float);
  hipError_t e = set_lds_fast(k_apply_fast<C, R, r, TH, TW, MODE>, bytes);
  if (e != hipSuccess) return e;
  A.tiles_x = (g.W + TW - 1) / TW;
  A.ntiles = A.tiles_x * ((g.H + TH - 1) / TH);
  hipLaunchKernelGGL((k_apply_fast<C, R, r, TH, TW, MODE>), dim3(A.ntiles * g.N), dim3(kBlock), bytes, s, g, A, u);
  return hipGetLastError();
}

template <int C, int R, int r, int TH, int TW>
hipError_t run_apply_fast(const Geom& g, ApplyArgs A, const float* u, hipStream_t s) {
  return A.mode == 0 ? run_apply_fast_m<C, R, r, TH, TW, 0>(g, A, u, s) : run_apply_fast_m<C, R, r, TH, TW, 1>(g, A, u, s);
}

// The specialised (C, R, r) triples: the measured workloads (C = 4, n = 9..17, r = 1, 2), C = 2 with the same
// kernels, and the paper's 29 x 29 kernel at C = 4.  (At C = 2 a 29 x 29 kernel would need a 15 x 15
// neighbourhood of y per thread; it stays on the generic kernels.)

}  // namespace

// Every tile region of both fast kernels must overhang the image by less than one period (wrap1).
bool fast_path_fits(const Geom& g, int dir_rows, int apply_variant) {
  const int C = g.c, R = g.R, r = g.r;
  const int HYR = (R + C - 1) / C;
  const int k0_last = ((g.w - 1) / 64) * 64, m0_last = ((g.h - 1) / dir_rows) * dir_rows;
  if ((size_t)g.H * g.W >= ((size_t)1 << 29)) return false;  // byte offsets of a plane below kNoAccess
  if (C * HYR > g.W || C * HYR > g.H) return false;
  if (C * (k0_last + 64 + HYR) > 2 * g.W || C * (m0_last + dir_rows + HYR) > 2 * g.H) return false;
  if (apply_variant == kSweepVariant) return sweep_fits(g, kMinSegRows);
  const int TH = apply_variant == 0 ? 32 : 16, TW = 64, E = 2 * r + 2;
  const int i0_last = ((g.H - 1) / TH) * TH, j0_last = ((g.W - 1) / TW) * TW;
  if (E > g.H || E > g.W || i0_last + TH + E > 2 * g.H || j0_last + TW + E > 2 * g.W) return false;
  const int YL = R / C, YR = (C - 1 + R) / C;
  if (YL > g.h || YL > g.w) return false;
  if (i0_last / C + TH / C + YR > 2 * g.h || j0_last / C + TW / C + YR > 2 * g.w) return false;
  return true;
}

bool fast_path_available(int C, int R, int r) {
  if (r != 1 && r != 2) return false;
  if (C == 4) return (R >= 4 && R <= 8) || R == 14;
  if (C == 2) return R >= 4 && R <= 8;
  return false;
}

int fast_apply_lds_floats(int C, int R, int r, int variant) {
  if (variant == kSweepVariant) return fast_path_available(C, R, r) ? 1 : -1;  // no LDS tiles
#define LLP_LDS_CASE(CC, RR, rr)                                                           \
  if (C == CC && R == RR && r == rr)                                                       \
    return variant == 0 ? ApplyShape<CC, RR, rr, 32, 64>::total : ApplyShape<CC, RR, rr, 16, 64>::total;
  LLP_FAST_R_LIST2(LLP_LDS_CASE, 1)
  LLP_FAST_R_LIST2(LLP_LDS_CASE, 2)
  LLP_FAST_R_LIST4(LLP_LDS_CASE, 1)
  LLP_FAST_R_LIST4(LLP_LDS_CASE, 2)
#undef LLP_LDS_CASE
  return -1;
}

hipError_t launch_dir_fast(const Geom& g, DirArgs A, int tyl, const float* u, hipStream_t s) {
#define LLP_DIR_CASE(CC, RR, rr) \
  if (g.c == CC && g.R == RR) return run_dir_fast<CC, RR>(g, A, tyl, u, s);
  LLP_FAST_R_LIST2(LLP_DIR_CASE, 0)
  LLP_FAST_R_LIST4(LLP_DIR_CASE, 0)
#undef LLP_DIR_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_apply_fast(const Geom& g, int variant, ApplyArgs A, const float* u, hipStream_t s) {
#define LLP_APPLY_CASE(CC, RR, rr)                                                                         \
  if (g.c == CC && g.R == RR && g.r == rr)                                                                 \
    return variant == 0 ? run_apply_fast<CC, RR, rr, 32, 64>(g, A, u, s) : run_apply_fast<CC, RR, rr, 16, 64>(g, A, u, s);
  LLP_FAST_R_LIST2(LLP_APPLY_CASE, 1)
  LLP_FAST_R_LIST2(LLP_APPLY_CASE, 2)
  LLP_FAST_R_LIST4(LLP_APPLY_CASE, 1)
  LLP_FAST_R_LIST4(LLP_APPLY_CASE, 2)
#undef LLP_APPLY_CASE
  return hipErrorInvalidValue;
}

namespace {

template <int C, int R, int TYL, int MODE>
hipError_t run_dir_batch_m(const SceneDesc* t, int count, int blocks, int parity, ChanState* st, char* ws,
                           const float* taps, hipStream_t s) {
  const size_t bytes = (size_t)DirShape<C, R, TYL>::LDS_ALLOC * sizeof(float);
  hipError_t e = set_lds_fast(k_dir_fast_batch<C, R, TYL, MODE>, bytes);
  if (e != hipSuccess) return e;
  if (blocks == 0) return hipSuccess;  // prepare only (before a graph capture)
  hipLaunchKernelGGL((k_dir_fast_batch<C, R, TYL, MODE>), dim3(blocks), dim3(DirShape<C, R, TYL>::NW * 64), bytes, s,
                     t, count, parity, st, ws, taps);
  return hipGetLastError();
}

template <int C, int R, int TYL>
hipError_t run_dir_batch(const SceneDesc* t, int count, int blocks, int parity, ChanState* st, char* ws,
                         const float* taps, int mode, hipStream_t s) {
  return mode == 3 ? run_dir_batch_m<C, R, TYL, 3>(t, count, blocks, parity, st, ws, taps, s)
                   : run_dir_batch_m<C, R, TYL, 2>(t, count, blocks, parity, st, ws, taps, s);
}

template <int C, int R, int r, int TH, int TW>
hipError_t run_apply_batch(const SceneDesc* t, int count, int blocks, int parity, ChanState* st, char* ws,
                           const float* taps, hipStream_t s) {
  const size_t bytes = (size_t)ApplyShape<C, R, r, TH, TW>::total * sizeof(float);
  hipError_t e = set_lds_fast(k_apply_fast_batch<C, R, r, TH, TW>, bytes);
  if (e != hipSuccess) return e;
  if (blocks == 0) return hipSuccess;  // prepare only (before a graph capture)
  hipLaunchKernelGGL((k_apply_fast_batch<C, R, r, TH, TW>), dim3(blocks), dim3(kBlock), bytes, s, t, count, parity,
                     st, ws, taps);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_dir_fast_batch(const SceneDesc* table, int count, int total_blocks, int C, int R, int tyl,
                                 int parity, ChanState* st, char* ws, const float* taps, int mode, hipStream_t s) {
#define LLP_DIRB_CASE(CC, RR, rr)                                                                           \
  if (C == CC && R == RR)                                                                                   \
    return tyl == 8 ? run_dir_batch<CC, RR, 8>(table, count, total_blocks, parity, st, ws, taps, mode, s) \
                    : run_dir_batch<CC, RR, 4>(table, count, total_blocks, parity, st, ws, taps, mode, s);
  LLP_FAST_R_LIST2(LLP_DIRB_CASE, 0)
  LLP_FAST_R_LIST4(LLP_DIRB_CASE, 0)
#undef LLP_DIRB_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_apply_fast_batch(const SceneDesc* table, int count, int total_blocks, int C, int R, int r,
                                   int variant, int parity, ChanState* st, char* ws, const float* taps,
                                   hipStream_t s) {
#define LLP_APPLYB_CASE(CC, RR, rr)                                                                   \
  if (C == CC && R == RR && r == rr)                                                                  \
    return variant == 0                                                                                 \
               ? run_apply_batch<CC, RR, rr, 32, 64>(table, count, total_blocks, parity, st, ws, taps, s)   \
               : run_apply_batch<CC, RR, rr, 16, 64>(table, count, total_blocks, parity, st, ws, taps, s);
  LLP_FAST_R_LIST2(LLP_APPLYB_CASE, 1)
  LLP_FAST_R_LIST2(LLP_APPLYB_CASE, 2)
  LLP_FAST_R_LIST4(LLP_APPLYB_CASE, 1)
  LLP_FAST_R_LIST4(LLP_APPLYB_CASE, 2)
#undef LLP_APPLYB_CASE
  return hipErrorInvalidValue;
}

}  // namespace llp
