// C ABI of libllp (declared in include/llp.h): argument validation, workspaces and the host side of the
// conjugate-gradient solve of eq. (Z_ini_matting), Sec. III-B, for one scene.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "llp_ctx.h"

using namespace llp;
using namespace llp::host;

namespace llp {
namespace host {



size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

llp_status validate(const llp_shape* s, const llp_params* p, Geom* g) {
  if (!s) return LLP_E_ARG;
  if (s->N < 1 || s->h < 1 || s->w < 1 || s->c < 1 || s->n < 1) return LLP_E_SHAPE;
  if ((s->n & 1) == 0) return LLP_E_SHAPE;
  if (s->c > kMaxScale || s->n > LLP_MAX_KERNEL) return LLP_E_UNSUPPORTED;
  const long long H = (long long)s->c * s->h, W = (long long)s->c * s->w;
  if (H > 65536 || W > 65536) return LLP_E_UNSUPPORTED;
  if ((long long)s->N * H * W >= (1LL << 31)) return LLP_E_UNSUPPORTED;
  if (s->n > H || s->n > W) return LLP_E_SHAPE;
  g->N = s->N;
  g->h = s->h;
  g->w = s->w;
  g->c = s->c;
  g->n = s->n;
  g->R = (s->n - 1) / 2;
  g->H = (int)H;
  g->W = (int)W;
  g->r = 0;
  g->lam = 0.0f;
  g->eps = 0.0f;
  if (p) {
    if (p->r < 0) return LLP_E_ARG;
    if (p->r > LLP_MAX_RADIUS) return LLP_E_UNSUPPORTED;
    if (2 * p->r + 1 > H || 2 * p->r + 1 > W) return LLP_E_SHAPE;
    if (!isfinite(p->lambda) || p->lambda < 0.0f) return LLP_E_ARG;
    if (!isfinite(p->eps) || p->eps < 0.0f) return LLP_E_ARG;
    if (p->max_iters < 0 || !isfinite(p->tol)) return LLP_E_ARG;
    if (p->init_mode < 0 || p->init_mode > 2) return LLP_E_ARG;
    if (p->precond < 0 || p->precond > 1) return LLP_E_ARG;
    g->r = p->r;
    g->lam = p->lambda;
    g->eps = p->eps;
  }
  if (ref_y_lds(*g) > kRefMaxLds || ref_res_lds(*g) > kRefMaxLds) return LLP_E_UNSUPPORTED;
  if (p && p->precond && !pc_supported(*g)) return LLP_E_UNSUPPORTED;
  return LLP_OK;
}

bool pick_config(const Geom& g, OpConfig* cfg, bool allow_fast, int want_dir_rows, int want_apply_variant) {
  cfg->fast = 0;
  // Untuned defaults, from the autotuner's measurements on gfx950: the column sweep needs enough segments to
  // fill the chip, so small images keep the 16 x 64 tiles; short segments suit r = 1, longer ones r = 2.
  cfg->seg_rows = g.r == 1 ? kMinSegRows : (g.H >= 1024 ? 4 * kMinSegRows : 2 * kMinSegRows);
  const bool big = (size_t)g.H * g.W >= (size_t)600 * 600;
  if (allow_fast && fast_path_available(g.c, g.R, g.r)) {
    const int order_big[3] = {kSweepVariant, 1, 0}, order_small[3] = {1, kSweepVariant, 0};
    for (int v : big ? order_big : order_small) {
      if (want_apply_variant >= 0 && v != want_apply_variant) continue;
      const int f = fast_apply_lds_floats(g.c, g.R, g.r, v);
      const int rows = want_dir_rows == 8 ? 8 : 4;
      if (f > 0 && f <= kMaxLdsFloats && fast_path_fits(g, rows, v)) {
        cfg->fast = 1;
        cfg->dir_rows = rows;
        cfg->apply_variant = v;
        return true;
      }
    }
  }
  cfg->dir_rows = 0;
  for (int tyl : {8, 4}) {
    if (dir_lds_floats(g.c, tyl, g.R, nullptr) <= kMaxLdsFloats) {
      cfg->dir_rows = tyl;
      break;
    }
  }
  cfg->apply_variant = -1;
  for (int v = 0; v < kApplyVariants; ++v) {
    int TH = 0, TW = 0;
    if (apply_tile(g.c, v, &TH, &TW) != 0) continue;
    if (apply_lds_floats(g.c, TH, TW, g.R, g.r, nullptr, nullptr, nullptr, nullptr) <= kMaxLdsFloats) {
      cfg->apply_variant = v;
      break;
    }
  }
  return cfg->dir_rows > 0 && cfg->apply_variant >= 0;
}

llp_status ensure_workspace(llp_ctx* ctx, const Geom& g, bool precond) {
  const size_t HW = (size_t)g.H * g.W;
  const size_t planes = 3 * HW + 6 * (size_t)g.N * HW + (size_t)g.N * g.h * g.w;
  const size_t pstride = max_partials_per_band(g);
  size_t off = 0;
  const size_t o_planes = off;
  off = align_up(off + planes * sizeof(float), 256);
  const size_t o_part = off;
  off = align_up(off + (size_t)g.N * pstride * 3 * sizeof(double), 256);
  const size_t o_st = off;
  off = align_up(off + (size_t)g.N * sizeof(ChanState), 256);
  const size_t o_res = off;
  off = align_up(off + (size_t)g.N * kResultSlots * sizeof(double), 256);
  const size_t o_flags = off;
  off = align_up(off + 16 * sizeof(int), 256);
  const size_t o_xacc = off;
  off = align_up(off + (size_t)g.N * HW * sizeof(double), 256);
  const size_t o_y64 = off;
  off = align_up(off + (size_t)g.N * g.h * g.w * sizeof(double), 256);
  const size_t o_ref = off;
  off = align_up(off + sizeof(RefDesc), 256);
  // preconditioner: s, spectra, kernel DFT, twiddles, mbar and its partials, the descriptor
  const bool pc = precond && pc_supported(g);
  const size_t o_s = off;
  if (pc) off = align_up(off + (size_t)g.N * HW * sizeof(float), 256);
  const size_t o_spec = off;
  if (pc) off = align_up(off + pc_spec_floats(g) * sizeof(float), 256);
  const size_t o_uhat = off;
  if (pc) off = align_up(off + pc_uhat_floats(g) * sizeof(float), 256);
  const size_t o_tw = off;
  if (pc) off = align_up(off + pc_tw_floats(g) * sizeof(float), 256);
  const size_t o_mbar = off;
  off = align_up(off + (1 + kPcMbarBlocks) * sizeof(double), 256);
  const size_t o_pc = off;
  off = align_up(off + sizeof(PcDesc), 256);
  const size_t need = off;
  if (need > ctx->ws_bytes) {
    if (ctx->ws) {
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(ctx->ws));
      ctx->ws = nullptr;
      ctx->ws_bytes = 0;
    }
    if (hipMalloc(&ctx->ws, need) != hipSuccess) {
      ctx->ws = nullptr;
      return LLP_E_OOM;
    }
    ctx->ws_bytes = need;
  }
  char* base = (char*)ctx->ws;
  float* pl = (float*)(base + o_planes);
  ctx->G = pl;
  ctx->MU = pl + HW;
  ctx->DI = pl + 2 * HW;
  const size_t NHW = (size_t)g.N * HW;
  ctx->b = pl + 3 * HW;
  ctx->r[0] = ctx->b + NHW;
  ctx->r[1] = ctx->r[0] + NHW;
  ctx->p[0] = ctx->r[1] + NHW;
  ctx->p[1] = ctx->p[0] + NHW;
  ctx->q = ctx->p[1] + NHW;
  ctx->y = ctx->q + NHW;
  ctx->partials = (double*)(base + o_part);
  ctx->st = (ChanState*)(base + o_st);
  ctx->results = (double*)(base + o_res);
  ctx->flags = (int*)(base + o_flags);
  ctx->xacc = (double*)(base + o_xacc);
  ctx->y64 = (double*)(base + o_y64);
  ctx->d_ref = (RefDesc*)(base + o_ref);
  if (!ctx->h_ref && hipHostMalloc((void**)&ctx->h_ref, sizeof(RefDesc), hipHostMallocDefault) != hipSuccess)
    return LLP_E_OOM;
  ctx->s = pc ? (float*)(base + o_s) : nullptr;
  ctx->spec = pc ? (float*)(base + o_spec) : nullptr;
  ctx->uhat = pc ? (float*)(base + o_uhat) : nullptr;
  ctx->tw = pc ? (float*)(base + o_tw) : nullptr;
  ctx->mbar = (double*)(base + o_mbar);
  ctx->d_pc = (PcDesc*)(base + o_pc);
  if (!ctx->h_pc && hipHostMalloc((void**)&ctx->h_pc, sizeof(PcDesc), hipHostMallocDefault) != hipSuccess)
    return LLP_E_OOM;
  if (pc && ctx->h_tw_cap < pc_tw_floats(g)) {
    if (ctx->h_tw) (void)hipHostFree(ctx->h_tw);
    ctx->h_tw = nullptr;
    ctx->h_tw_cap = 0;
    if (hipHostMalloc((void**)&ctx->h_tw, pc_tw_floats(g) * sizeof(float), hipHostMallocDefault) != hipSuccess)
      return LLP_E_OOM;
    ctx->h_tw_cap = pc_tw_floats(g);
  }
  if (ctx->h_cap < g.N) {
    if (ctx->h_st) (void)hipHostFree(ctx->h_st);
    if (ctx->h_results) (void)hipHostFree(ctx->h_results);
    ctx->h_st = nullptr;
    ctx->h_results = nullptr;
    ctx->h_cap = 0;
    if (hipHostMalloc((void**)&ctx->h_st, sizeof(ChanState) * g.N, hipHostMallocDefault) != hipSuccess)
      return LLP_E_OOM;
    if (hipHostMalloc((void**)&ctx->h_results, sizeof(double) * kResultSlots * g.N, hipHostMallocDefault) !=
        hipSuccess)
      return LLP_E_OOM;
    ctx->h_cap = g.N;
  }
  if (!ctx->h_flags && hipHostMalloc((void**)&ctx->h_flags, 16 * sizeof(int), hipHostMallocDefault) != hipSuccess)
    return LLP_E_OOM;
  return LLP_OK;
}

int timing_begin(llp_ctx* ctx, hipStream_t s) {
  if (!ctx->profiling) return -1;
  const size_t i = ctx->tev_used;
  while (ctx->tev.size() < 2 * (i + 1)) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    ctx->tev.push_back(e);
  }
  if (ctx->tslot.size() < i + 1) ctx->tslot.resize(i + 1);
  if (hipEventRecord(ctx->tev[2 * i], s) != hipSuccess) return -1;
  ctx->tslot[i] = -1;
  ctx->tev_used = i + 1;
  return (int)i;
}

void timing_end(llp_ctx* ctx, hipStream_t s, int pair, int slot) {
  if (pair < 0) return;
  if (hipEventRecord(ctx->tev[2 * pair + 1], s) == hipSuccess) ctx->tslot[pair] = slot;
}

llp_status collect_times(llp_ctx* ctx) {
  for (size_t i = 0; i < ctx->tev_used; ++i) {
    if (ctx->tslot[i] < 0) continue;
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->tev[2 * i], ctx->tev[2 * i + 1]));
    llp_kernel_times& t = ctx->times;
    switch (ctx->tslot[i]) {
      case kTApply: t.apply_ms += ms, ++t.apply_launches; break;
      case kTDir: t.dir_ms += ms, ++t.dir_launches; break;
      case kTPcRows: t.pc_rows_ms += ms, ++t.pc_rows_launches; break;
      case kTPcCols: t.pc_cols_ms += ms, ++t.pc_cols_launches; break;
      case kTPcRowsInv: t.pc_rows_inv_ms += ms, ++t.pc_rows_inv_launches; break;
      default: t.ref_ms += ms, ++t.ref_passes; break;
    }
  }
  ctx->tev_used = 0;
  return LLP_OK;
}

llp_status check_inputs(llp_ctx* ctx, const Geom& g, const float* lrms, const float* pan, const float* kernel,
                        hipStream_t s) {
  HIP_TRY(hipMemsetAsync(ctx->flags, 0, sizeof(int), s));
  HIP_TRY(launch_check_finite(lrms, (size_t)g.N * g.h * g.w, ctx->flags, s));
  HIP_TRY(launch_check_finite(pan, (size_t)g.H * g.W, ctx->flags, s));
  HIP_TRY(launch_check_finite(kernel, (size_t)g.n * g.n, ctx->flags, s));
  return LLP_OK;
}

// q = A z: y = D B z on the LR lattice, then q = B^T D^T y + lambda L^T M L z.
llp_status apply_A_into(llp_ctx* ctx, const Geom& g, const OpConfig& cfg, const float* z, const float* kernel,
                        float* q, hipStream_t s) {
  HIP_TRY(launch_dir(g, cfg, 0, 0, 0, z, nullptr, nullptr, nullptr, nullptr, nullptr, ctx->y, kernel, ctx->partials,
                     ctx->st, 0, 0.0f, s));
  HIP_TRY(launch_apply(g, cfg, 0, z, nullptr, ctx->y, kernel, ctx->G, ctx->MU, ctx->DI, q, ctx->partials,
                       ctx->st, s));
  return LLP_OK;
}


void ref_plan(RefDesc* tab, int count, RefPlan* plan) {
  RefPlan P;
  P.count = count;
  for (int i = 0; i < count; ++i) {
    RefDesc& d = tab[i];
    d.e_block0 = P.eblocks;
    d.y_block0 = P.yblocks;
    d.r_block0 = P.rblocks;
    P.eblocks += ref_elem_blocks(d.g);
    P.yblocks += ref_y_blocks(d.g);
    P.rblocks += ref_res_blocks(d.g);
    P.bands += d.g.N;
    const size_t yl = ref_y_lds(d.g), rl = ref_res_lds(d.g);
    if (yl > P.ylds) P.ylds = yl;
    if (rl > P.rlds) P.rlds = rl;
  }
  *plan = P;
}

llp_status ref_pass(const RefDesc* d_tab, const RefPlan& P, ChanState* st, double* results, int fin_op, int force,
                    int rpar, int write_r, int max_iters, float tol, int plain_cg, hipStream_t s) {
  if (fin_op != kRefOut) HIP_TRY(launch_ref_elem(kRefFlush, d_tab, P.count, P.eblocks, st, force, s));
  HIP_TRY(launch_ref_y(d_tab, P.count, P.yblocks, P.ylds, st, force, s));
  HIP_TRY(launch_ref_res(d_tab, P.count, P.rblocks, P.rlds, st, force, rpar, write_r, s));
  HIP_TRY(launch_ref_fin(fin_op, d_tab, P.count, P.bands, st, results, force, plain_cg, max_iters, tol, s));
  return LLP_OK;
}

bool ctx_config(llp_ctx* ctx, const Geom& g, OpConfig* cfg, bool batched) {
  if (ctx->want_dir_rows == 0 && ctx->want_apply_variant < 0 && ctx->want_seg_rows == 0) {
    const int bucket = area_bucket(g);
    for (int want : {batched ? 1 : 0, 0}) {
      for (const TuneEntry& t : ctx->tuned) {
        if (t.c != g.c || t.R != g.R || t.r != g.r || t.bucket != bucket || t.batched != want) continue;
        if (t.cfg.fast && (!ctx->allow_fast || !fast_path_available(g.c, g.R, g.r) ||
                           !fast_path_fits(g, t.cfg.dir_rows, t.cfg.apply_variant) ||
                           (t.cfg.apply_variant == kSweepVariant && !sweep_fits(g, t.cfg.seg_rows))))
          break;
        *cfg = t.cfg;
        return true;
      }
    }
  }
  if (!pick_config(g, cfg, ctx->allow_fast, ctx->want_dir_rows, ctx->want_apply_variant)) return false;
  if (ctx->want_seg_rows >= kMinSegRows) cfg->seg_rows = ctx->want_seg_rows / 4 * 4;
  return true;
}

// The preconditioner's descriptor for the context's buffers (z the float32 iterate, s the output plane), its
// twiddles, the kernel DFT and mbar: the per-scene set-up of the Fourier-domain passes.
llp_status pc_setup(llp_ctx* ctx, const Geom& g, const float* kernel, float* sout, PcPlan* PP,
                    hipStream_t s) {
  PcDesc& pd = *ctx->h_pc;
  memset(&pd, 0, sizeof(pd));
  pc_fill(pd, g, ctx->tw);
  pd.spec = (float2*)ctx->spec;
  pd.uhat = (float2*)ctx->uhat;
  pd.u = kernel;
  pd.DI = ctx->DI;
  pd.mbar = ctx->mbar;
  pd.r[0] = ctx->r[0];
  pd.r[1] = ctx->r[1];
  pd.p[0] = ctx->p[0];
  pd.p[1] = ctx->p[1];
  pd.q = ctx->q;
  pd.s = sout;
  pd.partials = ctx->partials;
  pd.pstride = (int)max_partials_per_band(g);
  pd.band0 = 0;
  pc_plan(&pd, 1, PP);
  pc_twiddles(g, ctx->h_tw);
  HIP_TRY(hipMemcpyAsync(ctx->tw, ctx->h_tw, pc_tw_floats(g) * sizeof(float), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(ctx->d_pc, &pd, sizeof(PcDesc), hipMemcpyHostToDevice, s));
  HIP_TRY(launch_pc_rows(kPcRowsKernel, ctx->d_pc, *PP, ctx->st, 0, 0, s));
  HIP_TRY(launch_pc_cols(kPcColsKernel, ctx->d_pc, *PP, ctx->st, s));
  HIP_TRY(launch_pc_mbar(ctx->d_pc, 1, ctx->mbar + 1, s));
  return LLP_OK;
}

llp_status solve_scene(llp_ctx* ctx, const Geom& g, const OpConfig& cfg, const llp_params* params,
                       const float* lrms, const float* pan, const float* kernel, const float* init, float* hrms,
                       llp_report* rep, hipStream_t stream) {
  llp_status v;
  v = ensure_workspace(ctx, g, params->precond != 0);
  if (v != LLP_OK) return v;
  hipStream_t s = stream;
  const size_t NHW = (size_t)g.N * g.H * g.W;
  const int max_iters = params->max_iters;
  const float tol = params->tol;

  v = check_inputs(ctx, g, lrms, pan, kernel, s);
  if (v != LLP_OK) return v;
  // Per scene: the statistics that define M_LY, then the right-hand sides and ||b||.
  HIP_TRY(launch_pan_stats(g, pan, ctx->G, ctx->MU, ctx->DI, s));
  HIP_TRY(launch_rhs(g, lrms, kernel, ctx->b, ctx->partials, ctx->st, s));
  const int from_init = params->init_mode != 0;
  if (params->init_mode == 1 && init != hrms)
    HIP_TRY(hipMemcpyAsync(hrms, init, NHW * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (params->init_mode == 2) {  // the network's estimate, kept only for bands it brings closer than Z = 0
    v = cnn_warm_start(ctx, g, lrms, pan, hrms, nullptr, s);
    if (v != LLP_OK) return v;
  }
  HIP_TRY(launch_init(g, from_init, ctx->b, ctx->r[0], ctx->st, s));
  // The iterate is xacc (FP64) + hrms (float32, advanced by the iteration kernels between replacements).
  RefDesc& rd = *ctx->h_ref;
  memset(&rd, 0, sizeof(rd));
  rd.g = g;
  rd.Y = pan;
  rd.u = kernel;
  rd.b = ctx->b;
  rd.z = hrms;
  rd.xacc = ctx->xacc;
  rd.r[0] = ctx->r[0];
  rd.r[1] = ctx->r[1];
  rd.p[0] = ctx->p[0];
  rd.p[1] = ctx->p[1];
  rd.y64 = ctx->y64;
  rd.partials = ctx->partials;
  rd.pstride = (int)max_partials_per_band(g);
  rd.band0 = 0;
  RefPlan P;
  ref_plan(&rd, 1, &P);
  HIP_TRY(hipMemcpyAsync(ctx->d_ref, &rd, sizeof(RefDesc), hipMemcpyHostToDevice, s));
  HIP_TRY(launch_ref_elem(from_init ? kRefStartFrom : kRefStartZero, ctx->d_ref, 1, P.eblocks, ctx->st, 1, s));
  if (from_init) {  // r_0 = b - A Z0 in FP64; ||r_0||^2 decides a network start
    v = ref_pass(ctx->d_ref, P, ctx->st, ctx->results, kRefStart, 1, 0, 1, max_iters, tol, 1, s);
    if (v != LLP_OK) return v;
  }
  if (params->init_mode == 2) HIP_TRY(launch_fallback(g, ctx->results, ctx->st, ctx->b, ctx->r[0], ctx->xacc, s));

  // CG.  k_dir(k) produces x_k, r_k, p_k and y = D B p_k; k_apply(k) produces q_k = A p_k, alpha_k, beta_k.
  // Residual and direction alternate between two buffers so that no tile reads a neighbour's new values.
  // After every chunk of kCheckEvery iterations a residual-replacement pass runs for the bands that are due.
  // Preconditioned: k_apply, alpha; r_k, x_k and the forward rows of the transform; the columns with the group
  // solve; the inverse rows giving s_k = P^{-1} r_k, beta; p_k = s_k + beta p_{k-1} and y = D B p_k; the
  // stopping rule.
  const bool pc = params->precond != 0;
  const int nb_dir = dir_ntiles(g, cfg), nb_apply = apply_ntiles(g, cfg);
  PcPlan PP;
  if (pc) {
    v = pc_setup(ctx, g, kernel, ctx->s, &PP, s);
    if (v != LLP_OK) return v;
    // s_0 = P^{-1} r_0, rho_0 = r_0^T s_0, p_0 = s_0, y = D B p_0
    HIP_TRY(launch_pc_rows(kPcRowsStart, ctx->d_pc, PP, ctx->st, 0, 0, s));
    HIP_TRY(launch_pc_cols(kPcColsSolve, ctx->d_pc, PP, ctx->st, s));
    HIP_TRY(launch_pc_rows_inv(ctx->d_pc, PP, ctx->st, 0, s));
    HIP_TRY(launch_finalize(g, kFinPcgStart, ctx->partials, g.h, ctx->st, nullptr, 0, 0, max_iters, tol, s));
    HIP_TRY(launch_dir(g, cfg, 1, 0, 0, ctx->s, nullptr, nullptr, nullptr, ctx->p[0], hrms, ctx->y, kernel,
                       ctx->partials, ctx->st, max_iters, tol, s));
  } else {
    HIP_TRY(launch_dir(g, cfg, 1, 0, 0, ctx->r[0], nullptr, nullptr, nullptr, ctx->p[0], hrms, ctx->y, kernel,
                       ctx->partials, ctx->st, max_iters, tol, s));
    HIP_TRY(launch_finalize(g, kFinDir, ctx->partials, nb_dir, ctx->st, nullptr, 0, 0, max_iters, tol, s));
  }
  const bool tol_mode = tol > 0.0f;
  int chunk_no = 0;
  for (int k = 1; k <= max_iters;) {
    const int todo = max_iters - k + 1 < kCheckEvery ? max_iters - k + 1 : kCheckEvery;
    for (int t = 0; t < todo; ++t, ++k) {
      const int prev = (k - 1) & 1, cur = k & 1;
      int tp = timing_begin(ctx, s);
      HIP_TRY(launch_apply(g, cfg, 1, ctx->p[prev], ctx->r[prev], ctx->y, kernel, ctx->G, ctx->MU, ctx->DI,
                           ctx->q, ctx->partials, ctx->st, s));
      timing_end(ctx, s, tp, kTApply);
      if (pc) {
        HIP_TRY(launch_finalize(g, kFinPcgAlpha, ctx->partials, nb_apply, ctx->st, nullptr, 0, 0, 0, 0.0f, s));
        tp = timing_begin(ctx, s);
        HIP_TRY(launch_pc_rows(kPcRowsUpdate, ctx->d_pc, PP, ctx->st, prev, cur, s));
        timing_end(ctx, s, tp, kTPcRows);
        tp = timing_begin(ctx, s);
        HIP_TRY(launch_pc_cols(kPcColsSolve, ctx->d_pc, PP, ctx->st, s));
        timing_end(ctx, s, tp, kTPcCols);
        tp = timing_begin(ctx, s);
        HIP_TRY(launch_pc_rows_inv(ctx->d_pc, PP, ctx->st, cur, s));
        timing_end(ctx, s, tp, kTPcRowsInv);
        HIP_TRY(launch_finalize(g, kFinPcgBeta, ctx->partials, g.h, ctx->st, nullptr, 0, 0, 0, 0.0f, s));
        tp = timing_begin(ctx, s);
        HIP_TRY(launch_dir(g, cfg, 3, 0, k, ctx->s, nullptr, ctx->p[prev], nullptr, ctx->p[cur], hrms, ctx->y,
                           kernel, ctx->partials, ctx->st, max_iters, tol, s));
        timing_end(ctx, s, tp, kTDir);
        HIP_TRY(launch_finalize(g, kFinPcgStop, ctx->partials, 0, ctx->st, nullptr, 0, -1, max_iters, tol, s));
        continue;
      }
      HIP_TRY(launch_finalize(g, kFinApply, ctx->partials, nb_apply, ctx->st, nullptr, 0, 0, 0, 0.0f, s));
      tp = timing_begin(ctx, s);
      HIP_TRY(launch_dir(g, cfg, 2, k == max_iters, k, ctx->r[prev], ctx->q, ctx->p[prev], ctx->r[cur],
                         ctx->p[cur], hrms, ctx->y, kernel, ctx->partials, ctx->st, max_iters, tol, s));
      timing_end(ctx, s, tp, kTDir);
      HIP_TRY(launch_finalize(g, kFinDir, ctx->partials, nb_dir, ctx->st, nullptr, 0, -1, max_iters, tol, s));
    }
    // the next iteration (k) reads the buffers of parity (k - 1) & 1
    const int tr = timing_begin(ctx, s);
    v = ref_pass(ctx->d_ref, P, ctx->st, ctx->results, kRefStep, 0, (k - 1) & 1, 1, max_iters, tol, pc ? 0 : 1, s);
    if (v != LLP_OK) return v;
    timing_end(ctx, s, tr, kTRef);
    if (!tol_mode) continue;
    // Poll the band states of the chunk before last while this one runs (at most two chunks in flight).
    const int slot = chunk_no & 1;
    if (chunk_no >= 2) {
      HIP_TRY(hipEventSynchronize(ctx->ev[slot]));
      bool any = false;
      for (int i = 0; i < g.N; ++i) any |= ctx->h_st[i].active != 0 || ctx->h_st[i].pending != 0;
      if (!any) break;
    }
    HIP_TRY(hipMemcpyAsync(ctx->h_st, ctx->st, sizeof(ChanState) * g.N, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(ctx->ev[slot], s));
    ++chunk_no;
  }

  // The returned HRMS: float32(xacc + z).  With a report: the FP64 residual of the iterate before that rounding,
  // the FP64 residual of the float32 output, and the objective of the output.
  if (rep) {
    // the FP64 residual of every band's returned iterate (a band stopped by the tolerance has it already)
    v = ref_pass(ctx->d_ref, P, ctx->st, ctx->results, kRefFinal, 2, 0, 0, max_iters, tol, 1, s);
    if (v != LLP_OK) return v;
  }
  HIP_TRY(launch_ref_elem(rep ? kRefOutputBack : kRefOutput, ctx->d_ref, 1, P.eblocks, ctx->st, 1, s));
  if (rep) {
    v = ref_pass(ctx->d_ref, P, ctx->st, ctx->results, kRefOut, 1, 0, 0, max_iters, tol, 1, s);
    if (v != LLP_OK) return v;
    HIP_TRY(launch_objective(g, hrms, lrms, kernel, ctx->G, ctx->MU, ctx->DI, ctx->partials, ctx->st,
                             ctx->results, s));
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
      R.init = cs.init;
      R.status = st;
      const double bn2 = cs.bnorm2;
      R.rel_residual = bn2 > 0 ? sqrt(cs.rho / bn2) : sqrt(cs.rho);
      const double tr = ctx->h_results[i * kResultSlots + kSlotTrueRes];
      R.true_rel_residual = bn2 > 0 ? sqrt(tr / bn2) : sqrt(tr);
      const double orr = ctx->h_results[i * kResultSlots + kSlotOutRes];
      R.out_rel_residual = bn2 > 0 ? sqrt(orr / bn2) : sqrt(orr);
      R.objective = 0.5 * ctx->h_results[i * kResultSlots + kSlotObjData] +
                    0.5 * (double)g.lam * ctx->h_results[i * kResultSlots + kSlotObjLlp];
    }
  }
  return worst;
}

}  // namespace host
}  // namespace llp

extern "C" {

const char* llp_status_str(int status) {
  switch (status) {
    case LLP_OK: return "ok";
    case LLP_NOT_CONVERGED: return "tolerance not reached within max_iters";
    case LLP_E_ARG: return "invalid argument";
    case LLP_E_SHAPE: return "inconsistent shape";
    case LLP_E_UNSUPPORTED: return "unsupported size for this library";
    case LLP_E_HIP: return "HIP runtime error";
    case LLP_E_OOM: return "out of device memory";
    case LLP_E_BREAKDOWN: return "CG breakdown: p^T A p <= 0 or not finite";
    case LLP_E_NONFINITE: return "non-finite input";
    default: return "unknown status";
  }
}

llp_status llp_validate(const llp_shape* shape, const llp_params* params) {
  Geom g;
  llp_status v = validate(shape, params, &g);
  if (v != LLP_OK) return v;
  OpConfig cfg;
  if (params && !pick_config(g, &cfg)) return LLP_E_UNSUPPORTED;
  return LLP_OK;
}

llp_status llp_create(llp_ctx** out, int device) {
  if (!out) return LLP_E_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return LLP_E_ARG;
  HIP_TRY(hipSetDevice(device));
  HIP_TRY(ref_prepare());
  HIP_TRY(pc_prepare());
  llp_ctx* ctx = new (std::nothrow) llp_ctx();
  if (!ctx) return LLP_E_OOM;
  ctx->device = device;
  const char* fg = getenv("LLP_FORCE_GENERIC");
  ctx->allow_fast = !(fg && fg[0] && fg[0] != '0');
  if (const char* e = getenv("LLP_DIR_ROWS")) ctx->want_dir_rows = atoi(e);
  if (const char* e = getenv("LLP_APPLY_VARIANT")) ctx->want_apply_variant = atoi(e);
  if (const char* e = getenv("LLP_SEG_ROWS")) ctx->want_seg_rows = atoi(e);
  for (auto& e : ctx->ev) {
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      llp_destroy(ctx);
      return LLP_E_HIP;
    }
  }
  *out = ctx;
  return LLP_OK;
}

void llp_destroy(llp_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->h_st) (void)hipHostFree(ctx->h_st);
  if (ctx->h_results) (void)hipHostFree(ctx->h_results);
  if (ctx->h_flags) (void)hipHostFree(ctx->h_flags);
  if (ctx->h_ref) (void)hipHostFree(ctx->h_ref);
  if (ctx->h_pc) (void)hipHostFree(ctx->h_pc);
  if (ctx->h_tw) (void)hipHostFree(ctx->h_tw);
  for (auto& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : ctx->tev) (void)hipEventDestroy(e);
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->bws) (void)hipFree(ctx->bws);
  for (auto& h : ctx->h_bst)
    if (h) (void)hipHostFree(h);
  if (ctx->h_bres) (void)hipHostFree(ctx->h_bres);
  if (ctx->h_bflags) (void)hipHostFree(ctx->h_bflags);
  if (ctx->h_table) (void)hipHostFree(ctx->h_table);
  if (ctx->h_rtable) (void)hipHostFree(ctx->h_rtable);
  if (ctx->h_ptable) (void)hipHostFree(ctx->h_ptable);
  if (ctx->h_btw) (void)hipHostFree(ctx->h_btw);
  if (ctx->bev_in) (void)hipEventDestroy(ctx->bev_in);
  if (ctx->bstream) (void)hipStreamDestroy(ctx->bstream);
  cnn_free(ctx->cnn);
  if (ctx->prior_ws) (void)hipFree(ctx->prior_ws);
  if (ctx->ke_ws) (void)hipFree(ctx->ke_ws);
  delete ctx;
}

llp_status llp_pan_stats(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* pan,
                         float* G, float* mu, float* dinv, hipStream_t stream) {
  if (!ctx || !params || !pan || !G || !mu || !dinv) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, params, &g);
  if (v != LLP_OK) return v;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(launch_pan_stats(g, pan, G, mu, dinv, stream));
  return LLP_OK;
}

llp_status llp_rhs(llp_ctx* ctx, const llp_shape* shape, const float* lrms, const float* kernel, float* b,
                   hipStream_t stream) {
  if (!ctx || !lrms || !kernel || !b) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, nullptr, &g);
  if (v != LLP_OK) return v;
  HIP_TRY(hipSetDevice(ctx->device));
  v = ensure_workspace(ctx, g);
  if (v != LLP_OK) return v;
  HIP_TRY(launch_rhs(g, lrms, kernel, b, ctx->partials, ctx->st, stream));
  return LLP_OK;
}

llp_status llp_apply_A(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* pan,
                       const float* kernel, const float* z, float* Az, hipStream_t stream) {
  if (!ctx || !params || !pan || !kernel || !z || !Az || z == Az) return LLP_E_ARG;
  if (!aligned16(z) || !aligned16(Az)) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, params, &g);
  if (v != LLP_OK) return v;
  OpConfig cfg;
  if (!ctx_config(ctx, g, &cfg)) return LLP_E_UNSUPPORTED;
  HIP_TRY(hipSetDevice(ctx->device));
  v = ensure_workspace(ctx, g);
  if (v != LLP_OK) return v;
  HIP_TRY(launch_pan_stats(g, pan, ctx->G, ctx->MU, ctx->DI, stream));
  return apply_A_into(ctx, g, cfg, z, kernel, Az, stream);
}

llp_status llp_apply_data(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* kernel,
                          const float* z, float* out, hipStream_t stream) {
  if (!ctx || !params || !kernel || !z || !out || z == out) return LLP_E_ARG;
  if (!aligned16(z) || !aligned16(out)) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, params, &g);
  if (v != LLP_OK) return v;
  OpConfig cfg;
  if (!ctx_config(ctx, g, &cfg)) return LLP_E_UNSUPPORTED;
  HIP_TRY(hipSetDevice(ctx->device));
  v = ensure_workspace(ctx, g);
  if (v != LLP_OK) return v;
  // The solve's operator kernels with lambda = 0 and zero PAN statistics: the LLP part is then exactly 0.
  const size_t HW = (size_t)g.H * g.W;
  HIP_TRY(hipMemsetAsync(ctx->G, 0, 3 * HW * sizeof(float), stream));
  Geom gd = g;
  gd.lam = 0.0f;
  return apply_A_into(ctx, gd, cfg, z, kernel, out, stream);
}

llp_status llp_apply_llp(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* pan,
                         const float* kernel, const float* z, float* out, hipStream_t stream) {
  if (!ctx || !params || !pan || !kernel || !z || !out || z == out) return LLP_E_ARG;
  if (!aligned16(z) || !aligned16(out)) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, params, &g);
  if (v != LLP_OK) return v;
  OpConfig cfg;
  if (!ctx_config(ctx, g, &cfg)) return LLP_E_UNSUPPORTED;
  HIP_TRY(hipSetDevice(ctx->device));
  v = ensure_workspace(ctx, g);
  if (v != LLP_OK) return v;
  HIP_TRY(launch_pan_stats(g, pan, ctx->G, ctx->MU, ctx->DI, stream));
  // The solve's operator kernel with y = D B z replaced by 0: its data part B^T D^T y is then exactly 0.
  HIP_TRY(hipMemsetAsync(ctx->y, 0, (size_t)g.N * g.h * g.w * sizeof(float), stream));
  HIP_TRY(launch_apply(g, cfg, 0, z, nullptr, ctx->y, kernel, ctx->G, ctx->MU, ctx->DI, out, ctx->partials,
                       ctx->st, stream));
  return LLP_OK;
}

// Shared body of llp_precond_apply and llp_apply_data_fourier: z through the forward passes, the group
// operation `op`, the inverse passes, into out.
static llp_status fourier_apply(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* pan,
                                const float* kernel, const float* z, float* out, int op, hipStream_t stream) {
  if (!ctx || !params || !kernel || !z || !out || z == out || (op == kPcColsSolve && !pan)) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, params, &g);
  if (v != LLP_OK) return v;
  if (op == kPcColsData) g.lam = 1.0f;  // lambda and r matter only to the preconditioner
  if (op == kPcColsData && g.r < 1) g.r = 1;
  if (!pc_supported(g)) return LLP_E_UNSUPPORTED;
  HIP_TRY(hipSetDevice(ctx->device));
  v = ensure_workspace(ctx, g, true);
  if (v != LLP_OK) return v;
  const size_t NHW = (size_t)g.N * g.H * g.W;
  if (op == kPcColsSolve) HIP_TRY(launch_pan_stats(g, pan, ctx->G, ctx->MU, ctx->DI, stream));
  else HIP_TRY(hipMemsetAsync(ctx->DI, 0, (size_t)g.H * g.W * sizeof(float), stream));
  HIP_TRY(launch_init(g, 1, ctx->b, ctx->r[0], ctx->st, stream));  // every band active; r untouched
  HIP_TRY(hipMemcpyAsync(ctx->r[0], z, NHW * sizeof(float), hipMemcpyDeviceToDevice, stream));
  PcPlan PP;
  v = pc_setup(ctx, g, kernel, out, &PP, stream);
  if (v != LLP_OK) return v;
  HIP_TRY(launch_pc_rows(kPcRowsStart, ctx->d_pc, PP, ctx->st, 0, 0, stream));
  HIP_TRY(launch_pc_cols(op, ctx->d_pc, PP, ctx->st, stream));
  HIP_TRY(launch_pc_rows_inv(ctx->d_pc, PP, ctx->st, 0, stream));
  return LLP_OK;
}

llp_status llp_precond_apply(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* pan,
                             const float* kernel, const float* r, float* out, hipStream_t stream) {
  return fourier_apply(ctx, shape, params, pan, kernel, r, out, kPcColsSolve, stream);
}

llp_status llp_apply_data_fourier(llp_ctx* ctx, const llp_shape* shape, const llp_params* params,
                                  const float* kernel, const float* z, float* out, hipStream_t stream) {
  return fourier_apply(ctx, shape, params, nullptr, kernel, z, out, kPcColsData, stream);
}

// Algorithm "Fast Pansharpening" after Z^0 (Sec. III-B): the A, C step of eq. (ac_h_compute) and the Z step of
// eq. (Z_solution) with weight lambda |w|.  The guided filter's output is Lhat = l - (M l)/|w| (l = L Z0, M the
// matting matrix of L Y), so the Z step's normal equations P1 Z = B^T D^T X + lambda |w| L^T Lhat, with
// P1 = B^T D^T D B + lambda |w| L^T L, have the solution Z = Z0 + P1^{-1} (b - A Z0): A, C never need to be
// stored.  b - A Z0 is formed with the solve's operator kernels, P1^{-1} with the preconditioner's transforms
// (its scalar mbar set to |w|).
llp_status llp_polish(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* lrms,
                      const float* pan, const float* kernel, const float* z0, float* z, hipStream_t stream) {
  if (!ctx || !params || !lrms || !pan || !kernel || !z0 || !z || z0 == z) return LLP_E_ARG;
  if (!aligned16(z0) || !aligned16(z)) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, params, &g);
  if (v != LLP_OK) return v;
  if (!pc_supported(g)) return LLP_E_UNSUPPORTED;
  OpConfig cfg;
  if (!ctx_config(ctx, g, &cfg)) return LLP_E_UNSUPPORTED;
  HIP_TRY(hipSetDevice(ctx->device));
  v = ensure_workspace(ctx, g, true);
  if (v != LLP_OK) return v;
  const size_t NHW = (size_t)g.N * g.H * g.W;
  HIP_TRY(launch_pan_stats(g, pan, ctx->G, ctx->MU, ctx->DI, stream));
  HIP_TRY(launch_rhs(g, lrms, kernel, ctx->b, ctx->partials, ctx->st, stream));
  v = apply_A_into(ctx, g, cfg, z0, kernel, ctx->q, stream);
  if (v != LLP_OK) return v;
  HIP_TRY(launch_pc_axpy(ctx->b, ctx->q, ctx->r[0], -1.0f, NHW, stream));  // r = b - A Z0
  HIP_TRY(launch_init(g, 1, ctx->b, ctx->r[0], ctx->st, stream));           // every band active; r untouched
  PcPlan PP;
  v = pc_setup(ctx, g, kernel, ctx->s, &PP, stream);
  if (v != LLP_OK) return v;
  HIP_TRY(launch_pc_set_mbar(ctx->d_pc, 1, (double)((2 * g.r + 1) * (2 * g.r + 1)), stream));
  HIP_TRY(launch_pc_rows(kPcRowsStart, ctx->d_pc, PP, ctx->st, 0, 0, stream));
  HIP_TRY(launch_pc_cols(kPcColsSolve, ctx->d_pc, PP, ctx->st, stream));
  HIP_TRY(launch_pc_rows_inv(ctx->d_pc, PP, ctx->st, 0, stream));
  HIP_TRY(launch_pc_axpy(z0, ctx->s, z, 1.0f, NHW, stream));  // Z = Z0 + P1^{-1} r
  return LLP_OK;
}

llp_status llp_objective(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* lrms,
                         const float* pan, const float* kernel, const float* z, double* obj, hipStream_t stream) {
  if (!ctx || !params || !lrms || !pan || !kernel || !z || !obj) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, params, &g);
  if (v != LLP_OK) return v;
  HIP_TRY(hipSetDevice(ctx->device));
  v = ensure_workspace(ctx, g);
  if (v != LLP_OK) return v;
  HIP_TRY(launch_pan_stats(g, pan, ctx->G, ctx->MU, ctx->DI, stream));
  HIP_TRY(launch_objective(g, z, lrms, kernel, ctx->G, ctx->MU, ctx->DI, ctx->partials, ctx->st, ctx->results,
                           stream));
  HIP_TRY(hipMemcpyAsync(ctx->h_results, ctx->results, sizeof(double) * kResultSlots * g.N, hipMemcpyDeviceToHost,
                         stream));
  HIP_TRY(hipStreamSynchronize(stream));
  for (int i = 0; i < g.N; ++i)
    obj[i] = 0.5 * ctx->h_results[i * kResultSlots + kSlotObjData] +
             0.5 * (double)g.lam * ctx->h_results[i * kResultSlots + kSlotObjLlp];
  return LLP_OK;
}

llp_status llp_pansharpen(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* lrms,
                          const float* pan, const float* kernel, const float* init, float* hrms, llp_report* rep,
                          hipStream_t stream) {
  if (!ctx || !params || !lrms || !pan || !kernel || !hrms) return LLP_E_ARG;
  if (params->init_mode == 1 && !init) return LLP_E_ARG;
  if (params->init_mode == 2 && !ctx->cnn) return LLP_E_ARG;
  if (!aligned16(hrms) || (params->init_mode == 1 && !aligned16(init))) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, params, &g);
  if (v != LLP_OK) return v;
  OpConfig cfg;
  if (!ctx_config(ctx, g, &cfg)) return LLP_E_UNSUPPORTED;
  HIP_TRY(hipSetDevice(ctx->device));
  return solve_scene(ctx, g, cfg, params, lrms, pan, kernel, init, hrms, rep, stream);
}

llp_status llp_set_profiling(llp_ctx* ctx, int enable) {
  if (!ctx) return LLP_E_ARG;
  ctx->profiling = enable != 0;
  return LLP_OK;
}

llp_status llp_get_kernel_times(llp_ctx* ctx, llp_kernel_times* out, int reset) {
  if (!ctx || !out) return LLP_E_ARG;
  *out = ctx->times;
  if (reset) ctx->times = llp_kernel_times{};
  return LLP_OK;
}

}  // extern "C"
