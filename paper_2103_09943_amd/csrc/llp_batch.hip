// C ABI of libllp, batched solve (llp_pansharpen_batch): all bands of many scenes of different sizes advance
// through the CG iterations together (the parallel loop over bands of Algorithm "Fast Pansharpening",
// Sec. III-B, extended over scenes).
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "llp_ctx.h"

using namespace llp;
using namespace llp::host;

namespace {

constexpr int kTuneIters = 8;  // CG iterations per timed candidate of LLP_BATCH_AUTOTUNE
// One scene of a batch as the host plans it.
struct BatchScene {
  int idx;     // position in the caller's arrays
  int rep0;    // first report of the scene in the caller's report array
  Geom g;
  OpConfig cfg;
  long long cls;  // class key: (c, R, r, dir_rows, apply_variant)
};

long long class_key(const Geom& g, const OpConfig& cfg) {
  const long long seg = cfg.apply_variant == kSweepVariant ? cfg.seg_rows : 0;
  return (((((long long)g.c * 64 + g.R) * 16 + g.r) * 16 + cfg.dir_rows) * 16 + cfg.apply_variant) * 8192 + seg;
}

// One batched launch per class and kernel: scenes [first, first + count) of the table.
struct BatchClass {
  int C, R, r, dir_rows, variant;
  int first, count;
  int dir_blocks, apply_blocks;
  int data_blocks;  // column sweep, c = 2: k_data workgroups
};

llp_status ensure_batch_mirrors(llp_ctx* ctx, int bands, int scenes) {
  if (ctx->hb_bands < bands) {
    for (auto& h : ctx->h_bst) {
      if (h) (void)hipHostFree(h);
      h = nullptr;
    }
    if (ctx->h_bres) (void)hipHostFree(ctx->h_bres);
    ctx->h_bres = nullptr;
    ctx->hb_bands = 0;
    for (auto& h : ctx->h_bst)
      if (hipHostMalloc((void**)&h, sizeof(ChanState) * bands, hipHostMallocDefault) != hipSuccess) return LLP_E_OOM;
    if (hipHostMalloc((void**)&ctx->h_bres, sizeof(double) * kResultSlots * bands, hipHostMallocDefault) !=
        hipSuccess)
      return LLP_E_OOM;
    ctx->hb_bands = bands;
  }
  if (ctx->hb_scenes < scenes) {
    if (ctx->h_bflags) (void)hipHostFree(ctx->h_bflags);
    if (ctx->h_table) (void)hipHostFree(ctx->h_table);
    if (ctx->h_rtable) (void)hipHostFree(ctx->h_rtable);
    if (ctx->h_ptable) (void)hipHostFree(ctx->h_ptable);
    ctx->h_bflags = nullptr;
    ctx->h_table = nullptr;
    ctx->h_rtable = nullptr;
    ctx->h_ptable = nullptr;
    ctx->hb_scenes = 0;
    if (hipHostMalloc((void**)&ctx->h_bflags, sizeof(int) * scenes, hipHostMallocDefault) != hipSuccess)
      return LLP_E_OOM;
    if (hipHostMalloc((void**)&ctx->h_table, sizeof(SceneDesc) * scenes, hipHostMallocDefault) != hipSuccess)
      return LLP_E_OOM;
    if (hipHostMalloc((void**)&ctx->h_rtable, sizeof(RefDesc) * scenes, hipHostMallocDefault) != hipSuccess)
      return LLP_E_OOM;
    if (hipHostMalloc((void**)&ctx->h_ptable, sizeof(PcDesc) * scenes, hipHostMallocDefault) != hipSuccess)
      return LLP_E_OOM;
    ctx->hb_scenes = scenes;
  }
  return LLP_OK;
}

llp_status ensure_batch_twiddles(llp_ctx* ctx, size_t floats) {
  if (ctx->h_btw_cap >= floats) return LLP_OK;
  if (ctx->h_btw) (void)hipHostFree(ctx->h_btw);
  ctx->h_btw = nullptr;
  ctx->h_btw_cap = 0;
  if (hipHostMalloc((void**)&ctx->h_btw, floats * sizeof(float), hipHostMallocDefault) != hipSuccess) return LLP_E_OOM;
  ctx->h_btw_cap = floats;
  return LLP_OK;
}

// Enqueues `count` CG iterations of every class; the first reads the buffers of `parity`.  With `prof` set,
// every class launch is bracketed by timing events of that context.
// Preconditioned (d_pc, PP given): after the operator, alpha; the update and forward rows, the columns with the
// group solve, the inverse rows (s = P^{-1} r), beta; p = s + beta p and y = D B p; the stopping rule.
llp_status enqueue_batch_iters(const std::vector<BatchClass>& classes, const SceneDesc* d_table, int nscenes,
                               int nbands, ChanState* st, char* ws, const float* taps, int count, int parity,
                               int max_iters, float tol, hipStream_t s, llp_ctx* prof, const RefDesc* d_ref,
                               const RefPlan& rplan, double* results, const PcDesc* d_pc, const PcPlan* PP) {
  for (int j = 0; j < count; ++j) {
    const int par = (parity + j) & 1;
    if (d_pc) {
      for (size_t c = 0; c < classes.size(); ++c) {
        const BatchClass& k = classes[c];
        const int tp = prof ? timing_begin(prof, s) : -1;
        if (k.variant == kSweepVariant)
          HIP_TRY(launch_apply_sweep_batch(d_table + k.first, k.count, k.data_blocks, k.apply_blocks, k.C, k.R, k.r,
                                           par, st, ws, taps, s));
        else
          HIP_TRY(launch_apply_fast_batch(d_table + k.first, k.count, k.apply_blocks, k.C, k.R, k.r, k.variant, par,
                                          st, ws, taps, s));
        if (prof) timing_end(prof, s, tp, kTApply);
      }
      HIP_TRY(launch_finalize_batch(kFinPcgAlpha, d_table, nscenes, nbands, st, ws, max_iters, tol, s));
      int tp = prof ? timing_begin(prof, s) : -1;
      HIP_TRY(launch_pc_rows(kPcRowsUpdate, d_pc, *PP, st, par, 1 - par, s));
      if (prof) timing_end(prof, s, tp, kTPcRows);
      tp = prof ? timing_begin(prof, s) : -1;
      HIP_TRY(launch_pc_cols(kPcColsSolve, d_pc, *PP, st, s));
      if (prof) timing_end(prof, s, tp, kTPcCols);
      tp = prof ? timing_begin(prof, s) : -1;
      HIP_TRY(launch_pc_rows_inv(d_pc, *PP, st, 1 - par, s));
      if (prof) timing_end(prof, s, tp, kTPcRowsInv);
      HIP_TRY(launch_finalize_batch(kFinPcgBeta, d_table, nscenes, nbands, st, ws, max_iters, tol, s));
      for (size_t c = 0; c < classes.size(); ++c) {
        const BatchClass& k = classes[c];
        tp = prof ? timing_begin(prof, s) : -1;
        HIP_TRY(launch_dir_fast_batch(d_table + k.first, k.count, k.dir_blocks, k.C, k.R, k.dir_rows, par, st, ws,
                                      taps, 3, s));
        if (prof) timing_end(prof, s, tp, kTDir);
      }
      HIP_TRY(launch_finalize_batch(kFinPcgStop, d_table, nscenes, nbands, st, ws, max_iters, tol, s));
      continue;
    }
    for (size_t c = 0; c < classes.size(); ++c) {
      const BatchClass& k = classes[c];
      const int tp = prof ? timing_begin(prof, s) : -1;
      if (k.variant == kSweepVariant)
        HIP_TRY(launch_apply_sweep_batch(d_table + k.first, k.count, k.data_blocks, k.apply_blocks, k.C, k.R, k.r,
                                         par, st, ws, taps, s));
      else
        HIP_TRY(launch_apply_fast_batch(d_table + k.first, k.count, k.apply_blocks, k.C, k.R, k.r, k.variant, par,
                                        st, ws, taps, s));
      if (prof) timing_end(prof, s, tp, kTApply);
    }
    HIP_TRY(launch_finalize_batch(kFinApply, d_table, nscenes, nbands, st, ws, max_iters, tol, s));
    for (size_t c = 0; c < classes.size(); ++c) {
      const BatchClass& k = classes[c];
      const int tp = prof ? timing_begin(prof, s) : -1;
      HIP_TRY(launch_dir_fast_batch(d_table + k.first, k.count, k.dir_blocks, k.C, k.R, k.dir_rows, par, st, ws,
                                    taps, 2, s));
      if (prof) timing_end(prof, s, tp, kTDir);
    }
    HIP_TRY(launch_finalize_batch(kFinDir, d_table, nscenes, nbands, st, ws, max_iters, tol, s));
  }
  // residual replacement for the bands that are due; the next iteration reads the buffers of parity + count
  const int tr = prof ? timing_begin(prof, s) : -1;
  const llp_status v =
      ref_pass(d_ref, rplan, st, results, kRefStep, 0, (parity + count) & 1, 1, max_iters, tol, d_pc ? 0 : 1, s);
  if (prof) timing_end(prof, s, tr, kTRef);
  return v;
}
}  // namespace

extern "C" {

llp_status llp_pansharpen_batch(llp_ctx* ctx, int S, const llp_shape* shapes, const llp_params* params,
                                const float* const* lrms, const float* const* pan, const float* const* kernel,
                                const float* const* init, float* const* hrms, llp_report* rep, int flags,
                                hipStream_t stream) {
  if (!ctx || !params || S < 0 || (flags & ~(LLP_BATCH_NO_GRAPH | LLP_BATCH_SERIAL | LLP_BATCH_AUTOTUNE)) != 0) return LLP_E_ARG;
  if (S == 0) return LLP_OK;
  if (!shapes || !lrms || !pan || !kernel || !hrms) return LLP_E_ARG;
  const bool from_init = params->init_mode == 1;  // caller's starts
  const bool net_init = params->init_mode == 2;   // network starts
  if ((from_init && !init) || (net_init && !ctx->cnn)) return LLP_E_ARG;
  // Host-side planning: validate every scene, tune the classes not yet tuned (if asked), pick every scene's
  // kernels, group the specialised ones into classes.
  std::vector<Geom> geoms(S);
  for (int i = 0; i < S; ++i) {
    if (!lrms[i] || !pan[i] || !kernel[i] || !hrms[i] || (from_init && !init[i])) return LLP_E_ARG;
    if (!aligned16(hrms[i]) || (from_init && !aligned16(init[i]))) return LLP_E_ARG;
    llp_status v = validate(&shapes[i], params, &geoms[i]);
    if (v != LLP_OK) return v;
  }
  const bool batched = S > 1;  // launches carry the workgroups of several scenes
  if (flags & LLP_BATCH_AUTOTUNE) {
    for (int i = 0; i < S; ++i) {
      const Geom& g = geoms[i];
      const int bucket = area_bucket(g);
      bool have = false;  // an entry of the mode the planner will look up first, or a single-scene one for a
                          // scene that is never batched
      for (const TuneEntry& t : ctx->tuned)
        have |= t.c == g.c && t.R == g.R && t.r == g.r && t.bucket == bucket &&
                (t.batched == (batched ? 1 : 0) || (t.batched == 0 && !t.cfg.fast));
      if (have) continue;
      // scenes no specialised kernel fits are solved one by one: they get a single-scene entry
      llp_status v = LLP_E_UNSUPPORTED;
      if (batched)
        v = llp_autotune_batch(ctx, &shapes[i], params, lrms[i], pan[i], kernel[i], 0, kTuneIters, nullptr, stream);
      if (v == LLP_E_UNSUPPORTED)
        v = llp_autotune(ctx, &shapes[i], params, lrms[i], pan[i], kernel[i], nullptr, kTuneIters, nullptr, stream);
      if (v != LLP_OK) return v;
    }
  }
  std::vector<BatchScene> fast, slow;
  int total_bands = 0;
  for (int i = 0; i < S; ++i) {
    BatchScene b;
    b.idx = i;
    b.rep0 = total_bands;
    b.g = geoms[i];
    if (!ctx_config(ctx, b.g, &b.cfg, batched)) return LLP_E_UNSUPPORTED;
    b.cls = class_key(b.g, b.cfg);
    total_bands += b.g.N;
    if (b.cfg.fast && !(flags & LLP_BATCH_SERIAL)) fast.push_back(b);
    else slow.push_back(b);
  }
  HIP_TRY(hipSetDevice(ctx->device));
  if (!ctx->bstream) {
    HIP_TRY(hipStreamCreateWithFlags(&ctx->bstream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&ctx->bev_in, hipEventDisableTiming));
  }
  hipStream_t s = ctx->bstream;
  HIP_TRY(hipEventRecord(ctx->bev_in, stream));
  HIP_TRY(hipStreamWaitEvent(s, ctx->bev_in, 0));
  const int max_iters = params->max_iters;
  const float tol = params->tol;
  const bool tol_mode = tol > 0.0f;
  llp_status worst = LLP_OK;
  auto merge = [&worst](int st) {
    if (st < 0 && (worst >= 0 || st < worst)) worst = (llp_status)st;
    if (st > 0 && worst == LLP_OK) worst = (llp_status)st;
  };

  const bool pc = params->precond != 0;  // validate() has checked that every scene supports it
  if (!fast.empty()) {
    std::stable_sort(fast.begin(), fast.end(),
                     [](const BatchScene& a, const BatchScene& b) { return a.cls < b.cls; });
    const int nf = (int)fast.size();
    // Workspace: per scene the planes and partials of the single-scene solve, then the band states, the
    // result slots, the input flags and the scene table.
    std::vector<size_t> o_pl(nf), o_part(nf), o_pcs(nf), tw_off(nf);
    size_t off = 0, tw_total = 0;
    int nbands = 0;
    for (int i = 0; i < nf; ++i) {
      const Geom& g = fast[i].g;
      const size_t HW = (size_t)g.H * g.W;
      o_pl[i] = off;
      // the statistics G, mu, dinv, b, r (2), p (2), q, the iterate's float32 part x, and y; then the iterate's
      // FP64 part and D B x in FP64
      off = align_up(off + (3 * HW + 7 * (size_t)g.N * HW + (size_t)g.N * g.h * g.w) * sizeof(float), 256);
      off = align_up(off + ((size_t)g.N * HW + (size_t)g.N * g.h * g.w) * sizeof(double), 256);
      if (pc) {  // s, the spectra of the band pairs, U
        o_pcs[i] = off;
        off = align_up(off + (size_t)g.N * HW * sizeof(float), 256);
        off = align_up(off + pc_spec_floats(g) * sizeof(float), 256);
        off = align_up(off + pc_uhat_floats(g) * sizeof(float), 256);
        tw_off[i] = tw_total;
        tw_total += pc_tw_floats(g);
      }
      o_part[i] = off;
      off = align_up(off + (size_t)g.N * max_partials_per_band(g) * 3 * sizeof(double), 256);
      nbands += g.N;
    }
    const size_t o_st = off;
    off = align_up(off + (size_t)nbands * sizeof(ChanState), 256);
    const size_t o_res = off;
    off = align_up(off + (size_t)nbands * kResultSlots * sizeof(double), 256);
    const size_t o_flags = off;
    off = align_up(off + (size_t)nf * sizeof(int), 256);
    const size_t o_table = off;
    off = align_up(off + (size_t)nf * sizeof(SceneDesc), 256);
    const size_t o_taps = off;
    off = align_up(off + (size_t)nf * kTapStride * sizeof(float), 256);
    const size_t o_ref = off;
    off = align_up(off + (size_t)nf * sizeof(RefDesc), 256);
    const size_t o_pct = off;  // preconditioned: the transform table, mbar and its partials, the twiddles
    if (pc) off = align_up(off + (size_t)nf * sizeof(PcDesc), 256);
    const size_t o_mbar = off;
    if (pc) off = align_up(off + (size_t)nf * (1 + kPcMbarBlocks) * sizeof(double), 256);
    const size_t o_tw = off;
    if (pc) off = align_up(off + tw_total * sizeof(float), 256);
    if (off > ctx->bws_bytes) {
      if (ctx->bws) {
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipFree(ctx->bws));
        ctx->bws = nullptr;
        ctx->bws_bytes = 0;
      }
      if (ctx->gexec) {
        (void)hipGraphExecDestroy(ctx->gexec);
        ctx->gexec = nullptr;
        ctx->gkey.clear();
      }
      if (hipMalloc(&ctx->bws, off) != hipSuccess) {
        ctx->bws = nullptr;
        return LLP_E_OOM;
      }
      ctx->bws_bytes = off;
    }
    llp_status v = ensure_batch_mirrors(ctx, nbands, nf);
    if (v != LLP_OK) return v;
    if (pc) {
      v = ensure_batch_twiddles(ctx, tw_total);
      if (v != LLP_OK) return v;
    }
    char* base = (char*)ctx->bws;
    ChanState* st = (ChanState*)(base + o_st);
    double* results = (double*)(base + o_res);
    int* bflags = (int*)(base + o_flags);
    SceneDesc* d_table = (SceneDesc*)(base + o_table);
    float* d_taps = (float*)(base + o_taps);
    RefDesc* d_ref = (RefDesc*)(base + o_ref);
    PcDesc* d_pc = pc ? (PcDesc*)(base + o_pct) : nullptr;
    double* d_mbar = (double*)(base + o_mbar);
    float* d_tw = (float*)(base + o_tw);
    SceneDesc* tab = ctx->h_table;
    RefDesc* rtab = ctx->h_rtable;
    PcDesc* ptab = ctx->h_ptable;
    std::vector<BatchClass> classes;
    int band = 0;
    for (int i = 0; i < nf; ++i) {
      const BatchScene& bs = fast[i];
      const Geom& g = bs.g;
      const size_t HW = (size_t)g.H * g.W, NHW = (size_t)g.N * HW;
      SceneDesc& d = tab[i];
      memset(&d, 0, sizeof(d));
      d.g = g;
      d.X = lrms[bs.idx];
      d.Y = pan[bs.idx];
      d.u = kernel[bs.idx];
      float* pl = (float*)(base + o_pl[i]);
      d.G = pl;
      d.MU = pl + HW;
      d.DI = pl + 2 * HW;
      d.b = pl + 3 * HW;
      d.r[0] = d.b + NHW;
      d.r[1] = d.r[0] + NHW;
      d.p[0] = d.r[1] + NHW;
      d.p[1] = d.p[0] + NHW;
      d.q = d.p[1] + NHW;
      d.x = d.q + NHW;  // the iterate lives in the workspace during the solve; copied to hrms at the end
      d.y = d.x + NHW;
      d.partials = (double*)(base + o_part[i]);
      RefDesc& rd = rtab[i];
      memset(&rd, 0, sizeof(rd));
      rd.g = g;
      rd.Y = d.Y;
      rd.u = d.u;
      rd.b = d.b;
      rd.z = d.x;
      rd.xacc = (double*)(base + align_up(o_pl[i] + (3 * HW + 7 * NHW + (size_t)g.N * g.h * g.w) * sizeof(float),
                                          256));
      rd.y64 = rd.xacc + NHW;
      for (int j = 0; j < 2; ++j) {
        rd.r[j] = d.r[j];
        rd.p[j] = d.p[j];
      }
      rd.partials = d.partials;
      rd.pstride = (int)max_partials_per_band(g);
      rd.band0 = band;
      auto rel = [base](const void* ptr) { return (size_t)((const char*)ptr - base); };
      d.o_x = rel(d.x);
      d.o_r[0] = rel(d.r[0]);
      d.o_r[1] = rel(d.r[1]);
      d.o_p[0] = rel(d.p[0]);
      d.o_p[1] = rel(d.p[1]);
      d.o_q = rel(d.q);
      d.o_y = rel(d.y);
      d.o_G = rel(d.G);
      d.o_MU = rel(d.MU);
      d.o_DI = rel(d.DI);
      d.o_partials = rel(d.partials);
      if (pc) {
        float* sv = (float*)(base + o_pcs[i]);
        float* spec = (float*)(base + align_up(o_pcs[i] + NHW * sizeof(float), 256));
        float* uhat = (float*)((char*)spec + align_up(pc_spec_floats(g) * sizeof(float), 256));
        d.o_s = rel(sv);
        PcDesc& pd = ptab[i];
        memset(&pd, 0, sizeof(pd));
        pc_fill(pd, g, d_tw + tw_off[i]);
        pd.spec = (float2*)spec;
        pd.uhat = (float2*)uhat;
        pd.u = d.u;
        pd.DI = d.DI;
        pd.mbar = d_mbar + i;
        for (int j = 0; j < 2; ++j) {
          pd.r[j] = d.r[j];
          pd.p[j] = d.p[j];
        }
        pd.q = d.q;
        pd.s = sv;
        pd.partials = d.partials;
        pd.pstride = (int)max_partials_per_band(g);
        pd.band0 = band;
        pc_twiddles(g, ctx->h_btw + tw_off[i]);
      }
      d.taps_index = i;
      d.pstride = (int)max_partials_per_band(g);
      d.band0 = band;
      d.dir_ntiles = dir_ntiles(g, bs.cfg);
      d.apply_ntiles = apply_ntiles(g, bs.cfg);
      band += g.N;
      if (classes.empty() || bs.cls != fast[classes.back().first].cls) {
        BatchClass k;
        k.C = g.c;
        k.R = g.R;
        k.r = g.r;
        k.dir_rows = bs.cfg.dir_rows;
        k.variant = bs.cfg.apply_variant;
        k.first = i;
        k.count = 0;
        k.dir_blocks = 0;
        k.apply_blocks = 0;
        k.data_blocks = 0;
        classes.push_back(k);
      }
      BatchClass& k = classes.back();
      // Scenes start on multiples of 8 workgroups, so that the XCD-aware tile order holds within each scene.
      d.dir_block0 = k.dir_blocks;
      d.apply_block0 = k.apply_blocks;
      d.data_block0 = k.data_blocks;
      d.seg_rows = bs.cfg.seg_rows;
      k.dir_blocks += (int)align_up((size_t)d.dir_ntiles * g.N, 8);
      if (bs.cfg.apply_variant == kSweepVariant) {  // four bands per k_llp workgroup
        k.apply_blocks += (int)align_up((size_t)d.apply_ntiles * ((g.N + 3) / 4), 8);
        k.data_blocks += sweep_data_blocks(g);
      } else {
        k.apply_blocks += (int)align_up((size_t)d.apply_ntiles * g.N, 8);
      }
      k.count += 1;
    }
    RefPlan rplan;
    ref_plan(rtab, nf, &rplan);
    PcPlan pplan;
    if (pc) {
      pc_plan(ptab, nf, &pplan);
      HIP_TRY(hipMemcpyAsync(d_pc, ptab, sizeof(PcDesc) * nf, hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(d_tw, ctx->h_btw, tw_total * sizeof(float), hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipMemcpyAsync(d_table, tab, sizeof(SceneDesc) * nf, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_ref, rtab, sizeof(RefDesc) * nf, hipMemcpyHostToDevice, s));
    for (int i = 0; i < nf; ++i)
      HIP_TRY(hipMemcpyAsync(d_taps + (size_t)i * kTapStride, tab[i].u, sizeof(float) * tab[i].g.n * tab[i].g.n,
                             hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemsetAsync(bflags, 0, sizeof(int) * nf, s));
    // Per scene: input checks, PAN statistics, right-hand side, the start Z0 (into the float32 part x).
    for (int i = 0; i < nf; ++i) {
      const SceneDesc& d = tab[i];
      const Geom& g = d.g;
      ChanState* sst = st + d.band0;
      HIP_TRY(launch_check_finite(d.X, (size_t)g.N * g.h * g.w, bflags + i, s));
      HIP_TRY(launch_check_finite(d.Y, (size_t)g.H * g.W, bflags + i, s));
      HIP_TRY(launch_check_finite(d.u, (size_t)g.n * g.n, bflags + i, s));
      HIP_TRY(launch_pan_stats(g, d.Y, d.G, d.MU, d.DI, s));
      HIP_TRY(launch_rhs(g, d.X, d.u, d.b, d.partials, sst, s));
      if (from_init) {
        const float* z0 = init[fast[i].idx];
        if (z0 != d.x)
          HIP_TRY(hipMemcpyAsync(d.x, z0, (size_t)g.N * g.H * g.W * sizeof(float), hipMemcpyDeviceToDevice, s));
      }
      if (net_init) {
        v = cnn_warm_start(ctx, g, d.X, d.Y, d.x, nullptr, s);
        if (v != LLP_OK) return v;
      }
      HIP_TRY(launch_init(g, from_init || net_init, d.b, d.r[0], sst, s));
    }
    if (pc) {  // every scene's kernel spectrum U in the cell layout, and mbar (from the statistics)
      HIP_TRY(launch_pc_rows(kPcRowsKernel, d_pc, pplan, st, 0, 0, s));
      HIP_TRY(launch_pc_cols(kPcColsKernel, d_pc, pplan, st, s));
      HIP_TRY(launch_pc_mbar(d_pc, nf, d_mbar + nf, s));
    }
    // All scenes: the iterate's FP64 part from the start; for a given start r_0 = b - A Z0 in FP64.
    HIP_TRY(launch_ref_elem((from_init || net_init) ? kRefStartFrom : kRefStartZero, d_ref, nf, rplan.eblocks, st, 1,
                            s));
    if (from_init || net_init) {
      v = ref_pass(d_ref, rplan, st, results, kRefStart, 1, 0, 1, max_iters, tol, 1, s);
      if (v != LLP_OK) return v;
    }
    // Per scene: network-start check.  Then p_0, y = D B p_0 and rho_0; preconditioned, s_0 = P^{-1} r_0 for all
    // scenes first, rho_0 = r_0^T s_0 and p_0 = s_0.
    if (net_init)
      for (int i = 0; i < nf; ++i) {
        const SceneDesc& d = tab[i];
        HIP_TRY(launch_fallback(d.g, results + (size_t)d.band0 * kResultSlots, st + d.band0, d.b, d.r[0],
                                rtab[i].xacc, s));
      }
    if (pc) {
      HIP_TRY(launch_pc_rows(kPcRowsStart, d_pc, pplan, st, 0, 0, s));
      HIP_TRY(launch_pc_cols(kPcColsSolve, d_pc, pplan, st, s));
      HIP_TRY(launch_pc_rows_inv(d_pc, pplan, st, 0, s));
      HIP_TRY(launch_finalize_batch(kFinPcgStart, d_table, nf, nbands, st, base, max_iters, tol, s));
    }
    for (int i = 0; i < nf; ++i) {
      const SceneDesc& d = tab[i];
      const Geom& g = d.g;
      const OpConfig& cfg = fast[i].cfg;
      ChanState* sst = st + d.band0;
      HIP_TRY(launch_dir(g, cfg, 1, 0, 0, pc ? (const float*)(base + d.o_s) : d.r[0], nullptr, nullptr, nullptr,
                         d.p[0], d.x, d.y, d.u, d.partials, sst, max_iters, tol, s));
      if (!pc) HIP_TRY(launch_finalize(g, kFinDir, d.partials, d.dir_ntiles, sst, nullptr, 0, 0, max_iters, tol, s));
    }

    // CG iterations of all bands together, in chunks of kCheckEvery (even: every chunk starts on parity 0).
    // Timing (llp_set_profiling) needs events between the launches: then the chunks are enqueued directly.
    llp_ctx* prof = ctx->profiling ? ctx : nullptr;
    const bool use_graph = !(flags & LLP_BATCH_NO_GRAPH) && !prof;
    if (use_graph && max_iters > 0) {
      uint32_t tol_bits = 0;
      memcpy(&tol_bits, &tol, sizeof(tol_bits));
      std::vector<long long> key = {(long long)(uintptr_t)d_table, (long long)(uintptr_t)st, nf, nbands, max_iters,
                                    (long long)tol_bits, (long long)(uintptr_t)d_ref, rplan.eblocks, rplan.yblocks,
                                    rplan.rblocks, (long long)rplan.ylds, (long long)rplan.rlds, (long long)pc};
      if (pc)
        for (long long x : {(long long)(uintptr_t)d_pc, (long long)pplan.row_blocks, (long long)pplan.col_blocks,
                            (long long)pplan.row_lds, (long long)pplan.col_lds, (long long)pplan.mixed,
                            (long long)pplan.cus})
          key.push_back(x);
      for (const BatchClass& k : classes)
        for (long long x : {(long long)k.C, (long long)k.R, (long long)k.r, (long long)k.dir_rows,
                            (long long)k.variant, (long long)k.first, (long long)k.count, (long long)k.dir_blocks,
                            (long long)k.apply_blocks, (long long)k.data_blocks})
          key.push_back(x);
      if (!ctx->gexec || key != ctx->gkey) {
        if (ctx->gexec) {
          HIP_TRY(hipStreamSynchronize(s));
          (void)hipGraphExecDestroy(ctx->gexec);
          ctx->gexec = nullptr;
          ctx->gkey.clear();
        }
        for (const BatchClass& k : classes) {  // LDS limits are set outside the capture
          if (k.variant != kSweepVariant)
            HIP_TRY(launch_apply_fast_batch(d_table, k.count, 0, k.C, k.R, k.r, k.variant, 0, st, base, d_taps, s));
          HIP_TRY(launch_dir_fast_batch(d_table, k.count, 0, k.C, k.R, k.dir_rows, 0, st, base, d_taps, pc ? 3 : 2,
                                        s));
        }
        hipStream_t cs = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        llp_status cv = LLP_OK;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) cv = LLP_E_HIP;
        if (cv == LLP_OK)
          cv = enqueue_batch_iters(classes, d_table, nf, nbands, st, base, d_taps, kCheckEvery, 0, max_iters, tol, cs,
                                   nullptr, d_ref, rplan, results, d_pc, pc ? &pplan : nullptr);
        if (hipStreamEndCapture(cs, &graph) != hipSuccess && cv == LLP_OK) cv = LLP_E_HIP;
        (void)hipStreamDestroy(cs);
        if (cv == LLP_OK && hipGraphInstantiate(&ctx->gexec, graph, nullptr, nullptr, 0) != hipSuccess) {
          ctx->gexec = nullptr;
          cv = LLP_E_HIP;
        }
        if (graph) (void)hipGraphDestroy(graph);
        if (cv != LLP_OK) return cv;
        ctx->gkey = key;
      }
    }
    int chunk_no = 0;
    for (int k = 1; k <= max_iters; k += kCheckEvery) {
      if (use_graph) HIP_TRY(hipGraphLaunch(ctx->gexec, s));
      else {
        v = enqueue_batch_iters(classes, d_table, nf, nbands, st, base, d_taps, kCheckEvery, 0, max_iters, tol, s,
                                prof, d_ref, rplan, results, d_pc, pc ? &pplan : nullptr);
        if (v != LLP_OK) return v;
      }
      if (!tol_mode) continue;
      // Poll the band states of the chunk before last while this one runs (at most two chunks in flight).
      const int slot = chunk_no & 1;
      if (chunk_no >= 2) {
        HIP_TRY(hipEventSynchronize(ctx->ev[slot]));
        bool any = false;
        for (int i = 0; i < nbands; ++i) any |= ctx->h_bst[slot][i].active != 0 || ctx->h_bst[slot][i].pending != 0;
        if (!any) break;
      }
      HIP_TRY(hipMemcpyAsync(ctx->h_bst[slot], st, sizeof(ChanState) * nbands, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipEventRecord(ctx->ev[slot], s));
      ++chunk_no;
    }

    // The returned HRMS float32(xacc + x); with a report, the FP64 residuals of the iterate and of that output
    // and the output's objective.
    if (rep) {
      // the FP64 residual of every band's returned iterate (a band stopped by the tolerance has it already)
      v = ref_pass(d_ref, rplan, st, results, kRefFinal, 2, 0, 0, max_iters, tol, 1, s);
      if (v != LLP_OK) return v;
    }
    HIP_TRY(launch_ref_elem(rep ? kRefOutputBack : kRefOutput, d_ref, nf, rplan.eblocks, st, 1, s));
    if (rep) {
      v = ref_pass(d_ref, rplan, st, results, kRefOut, 1, 0, 0, max_iters, tol, 1, s);
      if (v != LLP_OK) return v;
      for (int i = 0; i < nf; ++i) {
        const SceneDesc& d = tab[i];
        ChanState* sst = st + d.band0;
        double* sres = results + (size_t)d.band0 * kResultSlots;
        HIP_TRY(launch_objective(d.g, d.x, d.X, d.u, d.G, d.MU, d.DI, d.partials, sst, sres, s));
      }
      HIP_TRY(hipMemcpyAsync(ctx->h_bres, results, sizeof(double) * kResultSlots * nbands, hipMemcpyDeviceToHost,
                             s));
    }
    HIP_TRY(hipMemcpyAsync(ctx->h_bst[0], st, sizeof(ChanState) * nbands, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(ctx->h_bflags, bflags, sizeof(int) * nf, hipMemcpyDeviceToHost, s));
    for (int i = 0; i < nf; ++i)  // the iterates to the caller's HRMS buffers
      HIP_TRY(hipMemcpyAsync(hrms[fast[i].idx], tab[i].x, sizeof(float) * tab[i].g.N * tab[i].g.H * tab[i].g.W,
                             hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (prof) {
      v = collect_times(ctx);
      if (v != LLP_OK) return v;
    }

    bool nonfinite = false;
    for (int i = 0; i < nf; ++i) {
      const SceneDesc& d = tab[i];
      nonfinite |= ctx->h_bflags[i] != 0;
      for (int c = 0; c < d.g.N; ++c) {
        const ChanState& cs = ctx->h_bst[0][d.band0 + c];
        const int bst = ctx->h_bflags[i] ? LLP_E_NONFINITE
                                          : ((cs.active || cs.pending) ? (tol_mode ? LLP_NOT_CONVERGED : LLP_OK)
                                                                       : cs.status);
        merge(bst);
        if (rep) {
          llp_report& R = rep[fast[i].rep0 + c];
          const double* res = ctx->h_bres + (size_t)(d.band0 + c) * kResultSlots;
          R.iters = cs.iters;
          R.init = cs.init;
          R.status = bst;
          const double bn2 = cs.bnorm2;
          R.rel_residual = bn2 > 0 ? sqrt(cs.rho / bn2) : sqrt(cs.rho);
          R.true_rel_residual = bn2 > 0 ? sqrt(res[kSlotTrueRes] / bn2) : sqrt(res[kSlotTrueRes]);
          R.out_rel_residual = bn2 > 0 ? sqrt(res[kSlotOutRes] / bn2) : sqrt(res[kSlotOutRes]);
          R.objective = 0.5 * res[kSlotObjData] + 0.5 * (double)d.g.lam * res[kSlotObjLlp];
        }
      }
    }
    if (nonfinite) merge(LLP_E_NONFINITE);
  }

  // Scenes without specialised kernels (or all scenes, with LLP_BATCH_SERIAL): one solve each.
  for (const BatchScene& b : slow) {
    const int st = llp_pansharpen(ctx, &shapes[b.idx], params, lrms[b.idx], pan[b.idx], kernel[b.idx],
                                  from_init ? init[b.idx] : nullptr, hrms[b.idx], rep ? rep + b.rep0 : nullptr, s);
    if (st == LLP_E_HIP || st == LLP_E_OOM || st == LLP_E_ARG) return (llp_status)st;
    if (st == LLP_E_NONFINITE && rep)
      for (int c = 0; c < b.g.N; ++c) rep[b.rep0 + c].status = LLP_E_NONFINITE;
    merge(st);
  }
  return worst;
}

}  // extern "C"
