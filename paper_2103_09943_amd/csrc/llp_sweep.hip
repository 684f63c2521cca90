// Split evaluation of q = A p (eq. Z_ini_matting) for the specialised (c, R, r) classes, in two launches:
//
// k_data: q_D = B^T D^T y, one thread per LR cell: the thread holds the cell's y neighbourhood in registers and
//   forms the C x C outputs of the cell with taps that are uniform across the wave (scalar registers).  q_D is
//   written into the output array q.
//
// k_llp: q = q_D + lambda L^T M L p (eq. matting_matrix, eq. reg2) and, in CG mode, the partial sums of p^T q,
//   r^T q and q^T q.  A column sweep: each wave owns a strip of 64 columns (the outer E = 2r + 2 on each side
//   are halo, recomputed by the neighbouring strips) and a segment of rows, and walks down the rows one per
//   step.  A step loads one new row of p and produces, through a pipeline of register rings, one output row E
//   rows behind:
//       l = L p                       (row t-1)          horizontal neighbours by DPP lane shifts
//       S(l), S(G l)                  (row t-1-r)        window sums: horizontal by lane shifts, vertical over a
//       a = (S(Gl)/|w| - mu S(l)/|w|) dinv, b = S(l)/|w| - a mu                      ring of 2r+1 rows
//       S(a), S(b)                    (row t-1-2r)
//       M l = |w| l - G S(a) - S(b)   (row t-1-2r)
//       q = q_D + lambda L (M l)      (row t-2-2r = t-E)
//   Vertical window sums are recomputed from the rings at every step (no running sums, so no drift).  Every
//   row a wave touches is a real (periodic) image row, and the outputs of a segment depend only on the rows
//   the wave loads itself.  The kernel uses no LDS tiles and no barriers; the four waves of a workgroup are the
//   bands of one (strip, segment), so the PAN statistics they read are shared in the caches.
#include "llp_fast_util.h"

namespace llp {
using namespace dev;

namespace {

// Cross-lane shifts by one lane over the whole wave (DPP wave_shr:1 / wave_shl:1): lane i receives v of lane
// i-1 (from_left) or i+1 (from_right); the lane at the wave's edge receives 0 (it is halo).
__device__ __forceinline__ float from_left(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_right(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}

// Sum of v over lanes i-r .. i+r.
template <int r>
__device__ __forceinline__ float hbox(float v) {
  const float lf = from_left(v), rt = from_right(v);
  float s = v + lf + rt;
  if (r == 2) s += from_left(lf) + from_right(rt);
  return s;
}

__device__ __forceinline__ int wrap_row(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <int C, int R>
struct DataShape {
  static constexpr int YL = R / C, YR = (C - 1 + R) / C, YK = YL + YR + 1;
};

template <int C, int R>
__device__ __forceinline__ void data_body(const Geom& g, const float* __restrict__ y, const float* __restrict__ u,
                                          float* __restrict__ q, int bx, int by, int band) {
  using S = DataShape<C, R>;
  // one wave per LR row (uniform: its row offsets are scalar), one lane per LR column
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int k = bx * 64 + lane, m = by * 4 + wave;
  if (m >= g.h) return;
  const bool live = k < g.w;
  const __amdgpu_buffer_rsrc_t Ry = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(y + (size_t)band * g.h * g.w), (short)0, (int)((size_t)g.h * g.w * 4), 0x00020000);
  unsigned co[S::YK];
#pragma unroll
  for (int d = 0; d < S::YK; ++d) co[d] = (unsigned)wrap_row(min(k, g.w - 1) + d - S::YL, g.w) * 4u;
  float yv[S::YK][S::YK];
#pragma unroll
  for (int dy = 0; dy < S::YK; ++dy) {
    const unsigned ro = (unsigned)(wrap_row(m + dy - S::YL, g.h) * g.w) * 4u;
#pragma unroll
    for (int dx = 0; dx < S::YK; ++dx)
      yv[dy][dx] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(Ry, co[dx], ro, 0));
  }
  float qd[C][C];
  cell_data_term<C, R, S::YK, S::YL, 0, C>(yv, u, qd);
  if (!live) return;
  float* qb = q + (size_t)band * g.H * g.W;
#pragma unroll
  for (int f = 0; f < C; ++f) {
    float* dst = qb + (size_t)(C * m + f) * g.W + (size_t)C * k;
    if constexpr (C == 4) *(float4*)dst = make_float4(qd[f][0], qd[f][1], qd[f][2], qd[f][3]);
    else *(float2*)dst = make_float2(qd[f][0], qd[f][1]);
  }
}

template <int C, int R>
__global__ __launch_bounds__(kBlock) void k_data(Geom g, const float* __restrict__ y, const float* __restrict__ u,
                                                 float* __restrict__ q, const ChanState* __restrict__ st) {
  if (st && !st[blockIdx.z].active) return;
  data_body<C, R>(g, y, u, q, blockIdx.x, blockIdx.y, blockIdx.z);
}

struct SweepArgs {
  int mode;          // 0: q = A p; 1: also the partial dot products, inactive bands skipped
  const float* p;
  const float* r;    // residual (mode 1)
  const float *G, *MU, *DI;  // PAN statistics planes
  const float* y;    // D B p [N][h][w] (fused data term)
  const float* u;    // blur kernel taps [n][n] (fused data term)
  float* q;          // out: q; with a separate data-term launch also in: q_D
  double* partials;  // [N][pstride][3]
  ChanState* st;
  int pstride;
  int nstrips, nsegs, seg_rows;
};

template <int r>
struct SweepShape {
  static constexpr int E = 2 * r + 2, P = 2 * r + 1, OUTW = 64 - 2 * E;
};

// Data term fused into the sweep (C = 4): every fourth step the wave forms q_D = B^T D^T y for one LR row of
// the 16 LR cells under its strip on the matrix cores, as D = Y T with
//   Y[i][k] = y[I - YL + dy][J0 + i - YL + dx]      (cell i's neighbourhood, k = (dy, dx))
//   T[k][4 f + e] = u[C (dy - YL) + R - f][C (dx - YL) + R - e]  (zero outside the kernel)
// so D[i][4 f + e] is output (C I + f, C (J0 + i) + e).  The K dimension runs over the neighbourhood in steps of
// four columns of one row dy (columns past YK have zero taps), so the rows of y a K step reads are uniform
// across the wave.  D goes through LDS into the sweep's one-column-per-lane layout.
template <int C, int R>
struct FusedShape {
  static constexpr int YL = R / C, YR = (C - 1 + R) / C, YK = YL + YR + 1;
  static constexpr int NB = (YK + 3) / 4;  // blocks of four neighbourhood columns per row
  static constexpr int KS = YK * NB;       // K steps of four
};

template <int r, int MODE, int C, int R>
__device__ __forceinline__ void llp_body(const Geom& g, const SweepArgs& A, int bid) {
  using S = SweepShape<r>;
  constexpr int E = S::E, P = S::P;
  constexpr bool kFused = C == 4;
  static_assert(C == 0 || C == 4, "fused data term: C = 4 only");
  using FS = FusedShape<kFused ? C : 4, kFused ? R : 4>;
  // steps per unrolled block: the ring period P and, when fused, the LR row period 4
  constexpr int L = kFused ? (P == 5 ? 20 : 12) : P;
  static_assert(L % P == 0 && (!kFused || (L % 4 == 0 && (2 * E) % 4 == 0)), "block length");
  constexpr float nwf = (float)(P * P), inv_nw = 1.0f / (float)(P * P);
  // the wave index is uniform within the wave: readfirstlane lets the compiler keep everything derived from it
  // (band, plane pointers, buffer resources) in scalar registers
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  __shared__ __attribute__((aligned(16))) float qsh[kFused ? 4 * 512 : 4];
  int tile, grp;
  tile_and_band(A.nstrips * A.nsegs, (g.N + 3) / 4, bid, tile, grp);
  const int band = grp * 4 + wave;
  if (band >= g.N) return;  // no barriers in this kernel
  if (MODE == 1 && !A.st[band].active) return;
  const int strip = tile % A.nstrips, seg = tile / A.nstrips;
  const int H = g.H, W = g.W;
  const int j0 = strip * S::OUTW, i0 = seg * A.seg_rows;
  const int i1 = min(i0 + A.seg_rows, H);
  const int col = j0 - E + lane;
  const unsigned gc = (unsigned)pos_mod(col, W);
  const bool out_lane = lane >= E && lane < 64 - E && col < W;
  const size_t HW = (size_t)H * W;
  const float* __restrict__ pb = A.p + (size_t)band * HW;
  const float* __restrict__ rb = A.r + (size_t)band * HW;
  float* __restrict__ qb = A.q + (size_t)band * HW;
  const float lam = g.lam;
  float pr[P], gr[P], lr[P], h1[P], h2[P], ha[P], hb[P], mr[P];
#pragma unroll
  for (int k = 0; k < P; ++k) pr[k] = gr[k] = lr[k] = h1[k] = h2[k] = ha[k] = hb[k] = mr[k] = 0.0f;
  float p_old = 0.0f;  // p of row t-P-1 = t-E (the value evicted from the p ring one step earlier)
  double dsum[3] = {0.0, 0.0, 0.0};
  // Global values step t uses: p of row t, G of row t-1 (kept in a ring until row t-P needs it again), mu and
  // dinv of row t-1-r, and q_D (and r) of row t-E.  They are loaded P steps ahead into a buffer of P slots.
  struct In {
    float p, g, mu, di, qd, rc;
  };
  // Loads and stores go through buffer resources over one plane each: the row is a scalar byte offset, the
  // lane's column a fixed vector byte offset, so no per-access address arithmetic is left in the loop.
  const unsigned gc4 = gc * 4u, W4 = (unsigned)W * 4u, plane = (unsigned)(HW * 4);
  auto rsrc = [&](const void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)bytes, 0x00020000);
  };
  const __amdgpu_buffer_rsrc_t Rp = rsrc(pb, plane), Rq = rsrc(qb, plane);
  const __amdgpu_buffer_rsrc_t Rr = rsrc(MODE == 1 ? rb : pb, plane);
  const __amdgpu_buffer_rsrc_t Rg = rsrc(A.G, plane), Rm = rsrc(A.MU, plane), Rd = rsrc(A.DI, plane);
  auto ld = [&](__amdgpu_buffer_rsrc_t rs, unsigned off) -> float {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, gc4, off, 0));
  };

  // Fused data term: the lane's share of T (B operand), its y column offsets (A operand), its LDS slots.
  const int g16 = lane >> 4, m16 = lane & 15;
  float taps[kFused ? FS::KS : 1];
  unsigned ycol[kFused ? FS::NB : 1];
  __amdgpu_buffer_rsrc_t Ry = Rp;
  float* qw = qsh + wave * 512;
  int qr_off = 0;  // the lane's LDS word for its output column (row f, buffer 0)
  if constexpr (kFused) {
    constexpr int n = 2 * R + 1;
    const int f = m16 / C, e = m16 % C;
#pragma unroll
    for (int s = 0; s < FS::KS; ++s) {
      const int dy = s / FS::NB, dx = 4 * (s % FS::NB) + g16;
      const int a = C * (dy - FS::YL) + R - f, b = C * (dx - FS::YL) + R - e;
      taps[s] = (dx < FS::YK && a >= 0 && a < n && b >= 0 && b < n) ? A.u[a * n + b] : 0.0f;
    }
    const int J0 = j0 / C;
#pragma unroll
    for (int bk = 0; bk < FS::NB; ++bk) {
      const int dx = min(4 * bk + g16, FS::YK - 1);  // past the neighbourhood: any real column (zero taps)
      ycol[bk] = (unsigned)pos_mod(J0 + m16 - FS::YL + dx, g.w) * 4u;
    }
    Ry = rsrc(A.y + (size_t)band * g.h * g.w, (unsigned)((size_t)g.h * g.w * 4));
    const int oc = out_lane ? lane - E : 0;
    qr_off = (oc % C) * 16 + oc / C;
  }
  // Y operand of one LR row, loaded two steps before its product is formed.  The calls come once per LR row
  // in row order, from LR row (i0 - 2E + 4) / 4 on; ybase is that row minus YL, wrapped into [0, h).
  float yv[kFused ? FS::KS : 1];
  int ybase = kFused ? pos_mod((i0 - 2 * E + 4) / 4 - FS::YL, g.h) : 0;
  auto load_y = [&]() {
    if constexpr (kFused) {
#pragma unroll
      for (int dy = 0; dy < FS::YK; ++dy) {
        const int row = ybase + dy < g.h ? ybase + dy : ybase + dy - g.h;
        const unsigned ro = (unsigned)(row * g.w) * 4u;
#pragma unroll
        for (int bk = 0; bk < FS::NB; ++bk)
          yv[dy * FS::NB + bk] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(Ry, ycol[bk], ro, 0));
      }
      ybase = ybase + 1 == g.h ? 0 : ybase + 1;
    }
  };
  // D = Y T for one LR row into LDS buffer `buf`: word buf*256 + f*64 + e*16 + i holds output (f, e) of cell i.
  auto product = [&](int buf) {
    if constexpr (kFused) {
      typedef float f4 __attribute__((ext_vector_type(4)));
      f4 d = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int s = 0; s < FS::KS; ++s) d = __builtin_amdgcn_mfma_f32_16x16x4f32(yv[s], taps[s], d, 0, 0, 0);
      // lane holds D[4 g16 + v][m16], v = 0..3: cells 4 g16 .. 4 g16 + 3 of output (m16 / 4, m16 % 4)
      *(f4*)(qw + buf * 256 + (m16 / C) * 64 + (m16 % C) * 16 + 4 * g16) = d;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  };

  auto next = [&](unsigned o) { return o + W4 == plane ? 0u : o + W4; };
  const int tstart = i0 - E;
  unsigned o0 = (unsigned)wrap_row(tstart, H) * W4, o1 = (unsigned)wrap_row(tstart - 1, H) * W4,
           o2 = (unsigned)wrap_row(tstart - 1 - r, H) * W4, o3 = (unsigned)wrap_row(tstart - E, H) * W4;
  auto load = [&](In& v) {
    v.p = ld(Rp, o0);
    v.g = ld(Rg, o1);
    v.mu = ld(Rm, o2);
    v.di = ld(Rd, o2);
    if (!kFused) v.qd = ld(Rq, o3);
    if (MODE == 1) v.rc = ld(Rr, o3);
    o0 = next(o0);
    o1 = next(o1);
    o2 = next(o2);
    o3 = next(o3);
  };
  // L steps from row tb with the values in cv; the slot of row x in every ring is (x - tb) mod P.  Step k
  // takes what it needs from cv[k mod P] and then refills it with the values of step k + P.  When fused, the
  // output row t - E of step k is C I + (k mod 4) (segments start on multiples of 4): its q_D row was formed
  // at the previous k = 3 (mod 4) step from y loaded at the k = 1 step before that.
  auto block = [&](int tb, In(&cv)[P]) {
    float dacc[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kk = 0; kk < L; ++kk) {
      const int k = kk % P;
      const int t = tb + kk;
      const In& cur = cv[k];
      const int km1 = (k + P - 1) % P, km2 = (k + P - 2) % P, kr = (k + r) % P;
      const int c3 = t - E;
      if (kFused && kk % 4 == 1) load_y();  // LR row (c3 + 3) / 4
      const float p_c3 = p_old;  // p of row t-E
      p_old = pr[k];
      pr[k] = cur.p;
      // l of row t-1
      const float pc = pr[km1];
      const float l = 4.0f * pc - pr[km2] - pr[k] - from_left(pc) - from_right(pc);
      lr[km1] = l;
      gr[km1] = cur.g;
      h1[km1] = hbox<r>(l);
      h2[km1] = hbox<r>(cur.g * l);
      // window sums centred on row t-1-r, and that window's a, b
      float sl = h1[0], sg = h2[0];
#pragma unroll
      for (int s = 1; s < P; ++s) {
        sl += h1[s];
        sg += h2[s];
      }
      const float mu = cur.mu, di = cur.di;
      const float m1 = sl * inv_nw, m2 = sg * inv_nw;
      const float av = (m2 - mu * m1) * di;
      const float bv = m1 - av * mu;
      ha[kr] = hbox<r>(av);
      hb[kr] = hbox<r>(bv);
      // M l on row t-1-2r = t-P (slot k)
      float sa = ha[0], sb = hb[0];
#pragma unroll
      for (int s = 1; s < P; ++s) {
        sa += ha[s];
        sb += hb[s];
      }
      mr[k] = nwf * lr[k] - gr[k] * sa - sb;
      // q on row t-E
      if (c3 >= i0 && c3 < i1) {
        const float mc = mr[km1];
        const float ql = lam * (4.0f * mc - mr[km2] - mr[k] - from_left(mc) - from_right(mc));
        if (out_lane) {
          float qd;
          if constexpr (kFused) qd = qw[((c3 >> 2) & 1) * 256 + (kk % 4) * 64 + qr_off];
          else qd = cur.qd;
          const float qv = qd + ql;
          __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(qv), Rq, gc4, (unsigned)c3 * W4, 0);
          if (MODE == 1) {
            dacc[0] = fmaf(p_c3, qv, dacc[0]);
            dacc[1] = fmaf(cur.rc, qv, dacc[1]);
            dacc[2] = fmaf(qv, qv, dacc[2]);
          }
        }
      }
      if (kFused && kk % 4 == 3) product(((c3 + 1) >> 2) & 1);
      load(cv[k]);
    }
    if (MODE == 1) {
#pragma unroll
      for (int j = 0; j < 3; ++j) dsum[j] += (double)dacc[j];
    }
  };
  In buf[P];
#pragma unroll
  for (int k = 0; k < P; ++k) load(buf[k]);
  for (int tb = tstart; tb < i1 + E; tb += L) block(tb, buf);
  if (MODE == 0) return;
#pragma unroll
  for (int j = 0; j < 3; ++j) dsum[j] = wave_sum(dsum[j]);
  if (lane == 0) {
    double* dst = A.partials + (size_t)band * A.pstride * 3 + (size_t)tile * 3;
    dst[0] = dsum[0];
    dst[1] = dsum[1];
    dst[2] = dsum[2];
  }
}

template <int r, int MODE, int C, int R>
__global__ __launch_bounds__(kBlock) void k_llp(Geom g, SweepArgs A) {
  llp_body<r, MODE, C, R>(g, A, blockIdx.x);
}

// ------------------------------------------------------------------------------------------------ batched ---

template <bool kData>
__device__ __forceinline__ int find_scene_split(const SceneDesc* __restrict__ t, int count, int b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int b0 = kData ? t[mid].data_block0 : t[mid].apply_block0;
    if (b0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int C, int R>
__global__ __launch_bounds__(kBlock) void k_data_batch(const SceneDesc* __restrict__ t, int count,
                                                       const ChanState* __restrict__ st, char* __restrict__ ws,
                                                       const float* __restrict__ taps) {
  const int si = find_scene_split<true>(t, count, blockIdx.x);
  const SceneDesc& d = t[si];
  const int local = blockIdx.x - d.data_block0;
  const int bx_n = (d.g.w + 63) / 64, by_n = (d.g.h + 3) / 4;
  if (local >= bx_n * by_n * d.g.N) return;
  const int band = local / (bx_n * by_n), rem = local % (bx_n * by_n);
  if (!st[d.band0 + band].active) return;
  data_body<C, R>(d.g, (const float*)(ws + d.o_y), taps + (size_t)d.taps_index * kTapStride,
                  (float*)(ws + d.o_q), rem % bx_n, rem / bx_n, band);
}

template <int r, int C, int R>
__global__ __launch_bounds__(kBlock) void k_llp_batch(const SceneDesc* __restrict__ t, int count, int parity,
                                                      ChanState* __restrict__ st, char* __restrict__ ws,
                                                      const float* __restrict__ taps) {
  const int si = find_scene_split<false>(t, count, blockIdx.x);
  const SceneDesc& d = t[si];
  const int local = blockIdx.x - d.apply_block0;
  const int nstrips = (d.g.W + SweepShape<r>::OUTW - 1) / SweepShape<r>::OUTW;
  const int nsegs = d.apply_ntiles / nstrips;
  if (local >= d.apply_ntiles * ((d.g.N + 3) / 4)) return;
  SweepArgs A{};
  A.mode = 1;
  A.p = (const float*)(ws + d.o_p[parity]);
  A.r = (const float*)(ws + d.o_r[parity]);
  A.G = (const float*)(ws + d.o_G);
  A.MU = (const float*)(ws + d.o_MU);
  A.DI = (const float*)(ws + d.o_DI);
  A.y = (const float*)(ws + d.o_y);
  A.u = taps + (size_t)d.taps_index * kTapStride;
  A.q = (float*)(ws + d.o_q);
  A.partials = (double*)(ws + d.o_partials);
  A.st = st + d.band0;
  A.pstride = d.pstride;
  A.nstrips = nstrips;
  A.nsegs = nsegs;
  A.seg_rows = d.seg_rows;
  llp_body<r, 1, C, R>(d.g, A, local);
}

}  // namespace

// ================================================================================================== host ===

int sweep_out_width(int r) { return 64 - 2 * (2 * r + 2); }

// (c, R) classes whose sweep forms the data term itself (no k_data launch).
bool sweep_fused(int C, int R) {
#define LLP_FUSED_CASE(CC, RR, rr) \
  if (C == CC && R == RR) return true;
  LLP_FAST_R_LIST4(LLP_FUSED_CASE, 0)
#undef LLP_FUSED_CASE
  return false;
}

bool sweep_fits(const Geom& g, int seg_rows) {
  const int E = 2 * g.r + 2;
  if (g.r != 1 && g.r != 2) return false;
  if ((size_t)g.H * g.W * 16 >= ((size_t)1 << 31)) return false;  // byte offsets fit a buffer resource
  if (seg_rows < 4 || seg_rows % 4 != 0 || g.H < 3 * E) return false;  // rows wrap at most once
  const int YL = g.R / g.c, YR = (g.c - 1 + g.R) / g.c;
  return YL <= g.h && YR <= g.h && YL <= g.w && YR <= g.w;
}

int sweep_ntiles(const Geom& g, int seg_rows) {
  const int ow = sweep_out_width(g.r);
  return ((g.W + ow - 1) / ow) * ((g.H + seg_rows - 1) / seg_rows);
}

int sweep_data_blocks(const Geom& g) {
  return sweep_fused(g.c, g.R) ? 0 : ((g.w + 63) / 64) * ((g.h + 3) / 4) * g.N;
}

namespace {

template <int C, int R>
hipError_t run_data(const Geom& g, const float* y, const float* u, float* q, const ChanState* st, hipStream_t s) {
  hipLaunchKernelGGL((k_data<C, R>), dim3((g.w + 63) / 64, (g.h + 3) / 4, g.N), dim3(kBlock), 0, s, g, y, u, q, st);
  return hipGetLastError();
}

hipError_t launch_data(const Geom& g, const float* y, const float* u, float* q, const ChanState* st,
                       hipStream_t s) {
#define LLP_DATA_CASE(CC, RR, rr) \
  if (g.c == CC && g.R == RR) return run_data<CC, RR>(g, y, u, q, st, s);
  LLP_FAST_R_LIST2(LLP_DATA_CASE, 0)
#undef LLP_DATA_CASE
  return hipErrorInvalidValue;
}

template <int r, int C, int R>
void run_llp(const Geom& g, const SweepArgs& A, dim3 grid, hipStream_t s) {
  if (A.mode == 0) hipLaunchKernelGGL((k_llp<r, 0, C, R>), grid, dim3(kBlock), 0, s, g, A);
  else hipLaunchKernelGGL((k_llp<r, 1, C, R>), grid, dim3(kBlock), 0, s, g, A);
}

}  // namespace

// q = A p by the split kernels (mode 0: q only; mode 1: CG step with dot products, inactive bands skipped).
hipError_t launch_apply_sweep(const Geom& g, int seg_rows, int mode, const float* p, const float* rres,
                              const float* y, const float* u, const float* G, const float* mu, const float* dinv,
                              float* q, double* partials, ChanState* st, hipStream_t s) {
  if (!sweep_fits(g, seg_rows)) return hipErrorInvalidValue;
  const bool fused = sweep_fused(g.c, g.R);
  if (!fused) {
    hipError_t e = launch_data(g, y, u, q, mode == 1 ? st : nullptr, s);
    if (e != hipSuccess) return e;
  }
  SweepArgs A{};
  A.mode = mode;
  A.p = p;
  A.r = rres;
  A.G = G;
  A.MU = mu;
  A.DI = dinv;
  A.y = y;
  A.u = u;
  A.q = q;
  A.partials = partials;
  A.st = st;
  A.pstride = (int)max_partials_per_band(g);
  const int ow = sweep_out_width(g.r);
  A.nstrips = (g.W + ow - 1) / ow;
  A.nsegs = (g.H + seg_rows - 1) / seg_rows;
  A.seg_rows = seg_rows;
  const dim3 grid(A.nstrips * A.nsegs * ((g.N + 3) / 4));
  if (!fused) {
    if (g.r == 1) run_llp<1, 0, 0>(g, A, grid, s);
    else run_llp<2, 0, 0>(g, A, grid, s);
    return hipGetLastError();
  }
#define LLP_LLP_CASE(CC, RR, rr) \
  if (g.c == CC && g.R == RR && g.r == rr) run_llp<rr, CC, RR>(g, A, grid, s);
  LLP_FAST_R_LIST4(LLP_LLP_CASE, 1)
  LLP_FAST_R_LIST4(LLP_LLP_CASE, 2)
#undef LLP_LLP_CASE
  return hipGetLastError();
}

namespace {

template <int C, int R>
hipError_t run_data_batch(const SceneDesc* table, int count, int blocks, const ChanState* st, char* ws,
                          const float* taps, hipStream_t s) {
  hipLaunchKernelGGL((k_data_batch<C, R>), dim3(blocks), dim3(kBlock), 0, s, table, count, st, ws, taps);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_apply_sweep_batch(const SceneDesc* table, int count, int data_blocks, int llp_blocks, int C,
                                    int R, int r, int parity, ChanState* st, char* ws, const float* taps,
                                    hipStream_t s) {
  const bool fused = sweep_fused(C, R);
  if (data_blocks > 0 && !fused) {
    hipError_t e = hipErrorInvalidValue;
#define LLP_DATAB_CASE(CC, RR, rr) \
  if (C == CC && R == RR) e = run_data_batch<CC, RR>(table, count, data_blocks, st, ws, taps, s);
    LLP_FAST_R_LIST2(LLP_DATAB_CASE, 0)
#undef LLP_DATAB_CASE
    if (e != hipSuccess) return e;
  }
  if (llp_blocks > 0) {
    const dim3 grid(llp_blocks);
    if (!fused) {
      if (r == 1)
        hipLaunchKernelGGL((k_llp_batch<1, 0, 0>), grid, dim3(kBlock), 0, s, table, count, parity, st, ws, taps);
      else if (r == 2)
        hipLaunchKernelGGL((k_llp_batch<2, 0, 0>), grid, dim3(kBlock), 0, s, table, count, parity, st, ws, taps);
      else return hipErrorInvalidValue;
    } else {
#define LLP_LLPB_CASE(CC, RR, rr)                                                                              \
  if (C == CC && R == RR && r == rr)                                                                           \
    hipLaunchKernelGGL((k_llp_batch<rr, CC, RR>), grid, dim3(kBlock), 0, s, table, count, parity, st, ws, taps);
      LLP_FAST_R_LIST4(LLP_LLPB_CASE, 1)
      LLP_FAST_R_LIST4(LLP_LLPB_CASE, 2)
#undef LLP_LLPB_CASE
    }
  }
  return hipGetLastError();
}

}  // namespace llp
