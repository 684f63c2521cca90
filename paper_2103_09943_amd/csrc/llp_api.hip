// C ABI of libllp (declared in include/llp.h): argument validation, workspaces and the host side of the
// conjugate-gradient solve of eq. (Z_ini_matting), Sec. III-B.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "llp.h"
#include "llp_internal.h"

using namespace llp;

struct llp_ctx {
  int device = 0;
  bool allow_fast = true;  // false when LLP_FORCE_GENERIC is set at creation: generic kernels only
  int want_dir_rows = 0;   // launch-shape overrides (0: default), from LLP_DIR_ROWS / LLP_APPLY_VARIANT
  int want_apply_variant = -1;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // views into ws
  float *G = nullptr, *MU = nullptr, *DI = nullptr, *b = nullptr, *q = nullptr, *y = nullptr;
  float* r[2] = {nullptr, nullptr};  // residual, alternating between iterations
  float* p[2] = {nullptr, nullptr};  // direction, alternating between iterations
  double* partials = nullptr;
  ChanState* st = nullptr;
  double* results = nullptr;
  int* flags = nullptr;
  // pinned host mirrors
  ChanState* h_st = nullptr;
  double* h_results = nullptr;
  int* h_flags = nullptr;
  int h_cap = 0;  // bands the mirrors hold
  hipEvent_t ev[2] = {nullptr, nullptr};
  // kernel timing (llp_set_profiling)
  bool profiling = false;
  std::vector<hipEvent_t> tev;  // timing events, 4 per iteration (around k_apply and around k_dir)
  size_t tev_used = 0;
  llp_kernel_times times = {0.0, 0, 0.0, 0};
  // llp_pansharpen_batch: own stream, workspace, pinned mirrors and the cached graph of an iteration chunk
  hipStream_t bstream = nullptr;
  hipEvent_t bev_in = nullptr;
  void* bws = nullptr;
  size_t bws_bytes = 0;
  ChanState* h_bst[2] = {nullptr, nullptr};
  double* h_bres = nullptr;
  int* h_bflags = nullptr;
  SceneDesc* h_table = nullptr;
  int hb_bands = 0, hb_scenes = 0;  // capacities of the batch mirrors
  hipGraphExec_t gexec = nullptr;
  std::vector<long long> gkey;  // what the cached graph was captured for
};

namespace {

constexpr int kCheckEvery = 8;            // CG iterations between convergence polls in tolerance mode
constexpr int kMaxLdsFloats = 160 * 1024 / 4;

#define HIP_TRY(expr)                      \
  do {                                     \
    hipError_t e_ = (expr);                \
    if (e_ != hipSuccess) return LLP_E_HIP; \
  } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Image buffers are read and written with 16-byte vector accesses.
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
    if (p->init_mode != 0 && p->init_mode != 1) return LLP_E_ARG;
    g->r = p->r;
    g->lam = p->lambda;
    g->eps = p->eps;
  }
  return LLP_OK;
}

// Launch configuration of the iteration kernels: the first shapes (in preference order) whose LDS fits.
bool pick_config(const Geom& g, OpConfig* cfg, bool allow_fast = true, int want_dir_rows = 0,
                 int want_apply_variant = -1) {
  cfg->fast = 0;
  if (allow_fast && fast_path_available(g.c, g.R, g.r)) {
    for (int v : {1, 0}) {  // 16 x 64 tiles first (measured faster on the 2048^2 scene)
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

llp_status ensure_workspace(llp_ctx* ctx, const Geom& g) {
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

// Timing event number i of the current call (grown on demand).
hipEvent_t timing_event(llp_ctx* ctx) {
  if (ctx->tev_used == ctx->tev.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->tev.push_back(e);
  }
  return ctx->tev[ctx->tev_used++];
}

llp_status collect_times(llp_ctx* ctx) {
  for (size_t i = 0; i + 3 < ctx->tev_used; i += 4) {
    float a = 0.0f, b = 0.0f;
    HIP_TRY(hipEventElapsedTime(&a, ctx->tev[i], ctx->tev[i + 1]));
    HIP_TRY(hipEventElapsedTime(&b, ctx->tev[i + 2], ctx->tev[i + 3]));
    ctx->times.apply_ms += a;
    ctx->times.dir_ms += b;
    ctx->times.apply_launches += 1;
    ctx->times.dir_launches += 1;
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


// ------------------------------------------------------------------------------------------- batched solve ---

// One scene of a batch as the host plans it.
struct BatchScene {
  int idx;     // position in the caller's arrays
  int rep0;    // first report of the scene in the caller's report array
  Geom g;
  OpConfig cfg;
  long long cls;  // class key: (c, R, r, dir_rows, apply_variant)
};

long long class_key(const Geom& g, const OpConfig& cfg) {
  return ((((long long)g.c * 64 + g.R) * 16 + g.r) * 16 + cfg.dir_rows) * 16 + cfg.apply_variant;
}

// One batched launch per class and kernel: scenes [first, first + count) of the table.
struct BatchClass {
  int C, R, r, dir_rows, variant;
  int first, count;
  int dir_blocks, apply_blocks;
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
    ctx->h_bflags = nullptr;
    ctx->h_table = nullptr;
    ctx->hb_scenes = 0;
    if (hipHostMalloc((void**)&ctx->h_bflags, sizeof(int) * scenes, hipHostMallocDefault) != hipSuccess)
      return LLP_E_OOM;
    if (hipHostMalloc((void**)&ctx->h_table, sizeof(SceneDesc) * scenes, hipHostMallocDefault) != hipSuccess)
      return LLP_E_OOM;
    ctx->hb_scenes = scenes;
  }
  return LLP_OK;
}

// Enqueues `count` CG iterations of every class; the first reads the buffers of `parity`.  With `prof` set,
// every class launch is bracketed by timing events of that context.
llp_status enqueue_batch_iters(const std::vector<BatchClass>& classes, const SceneDesc* d_table, int nscenes,
                               int nbands, ChanState* st, int count, int parity, int max_iters, float tol,
                               hipStream_t s, llp_ctx* prof) {
  std::vector<hipEvent_t> ev(prof ? 4 * classes.size() : 0);
  for (int j = 0; j < count; ++j) {
    const int par = (parity + j) & 1;
    for (auto& e : ev)
      if (!(e = timing_event(prof))) return LLP_E_HIP;
    for (size_t c = 0; c < classes.size(); ++c) {
      const BatchClass& k = classes[c];
      if (prof) HIP_TRY(hipEventRecord(ev[4 * c], s));
      HIP_TRY(launch_apply_fast_batch(d_table + k.first, k.count, k.apply_blocks, k.C, k.R, k.r, k.variant, par, st,
                                      s));
      if (prof) HIP_TRY(hipEventRecord(ev[4 * c + 1], s));
    }
    HIP_TRY(launch_finalize_batch(kFinApply, d_table, nscenes, nbands, st, max_iters, tol, s));
    for (size_t c = 0; c < classes.size(); ++c) {
      const BatchClass& k = classes[c];
      if (prof) HIP_TRY(hipEventRecord(ev[4 * c + 2], s));
      HIP_TRY(launch_dir_fast_batch(d_table + k.first, k.count, k.dir_blocks, k.C, k.R, k.dir_rows, par, st, s));
      if (prof) HIP_TRY(hipEventRecord(ev[4 * c + 3], s));
    }
    HIP_TRY(launch_finalize_batch(kFinDir, d_table, nscenes, nbands, st, max_iters, tol, s));
  }
  return LLP_OK;
}

}  // namespace

extern "C" {

const char* llp_status_str(int status) {
  switch (status) {
    case LLP_OK: return "ok";
    case LLP_NOT_CONVERGED: return "tolerance not reached within max_iters";
    case LLP_E_ARG: return "invalid argument";
    case LLP_E_SHAPE: return "inconsistent shape";
    case LLP_E_UNSUPPORTED: return "unsupported size for this build";
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
  llp_ctx* ctx = new (std::nothrow) llp_ctx();
  if (!ctx) return LLP_E_OOM;
  ctx->device = device;
  const char* fg = getenv("LLP_FORCE_GENERIC");
  ctx->allow_fast = !(fg && fg[0] && fg[0] != '0');
  if (const char* e = getenv("LLP_DIR_ROWS")) ctx->want_dir_rows = atoi(e);
  if (const char* e = getenv("LLP_APPLY_VARIANT")) ctx->want_apply_variant = atoi(e);
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
  if (ctx->bev_in) (void)hipEventDestroy(ctx->bev_in);
  if (ctx->bstream) (void)hipStreamDestroy(ctx->bstream);
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
  if (!pick_config(g, &cfg, ctx->allow_fast, ctx->want_dir_rows, ctx->want_apply_variant)) return LLP_E_UNSUPPORTED;
  HIP_TRY(hipSetDevice(ctx->device));
  v = ensure_workspace(ctx, g);
  if (v != LLP_OK) return v;
  HIP_TRY(launch_pan_stats(g, pan, ctx->G, ctx->MU, ctx->DI, stream));
  return apply_A_into(ctx, g, cfg, z, kernel, Az, stream);
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
  if (!aligned16(hrms) || (params->init_mode == 1 && !aligned16(init))) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, params, &g);
  if (v != LLP_OK) return v;
  OpConfig cfg;
  if (!pick_config(g, &cfg, ctx->allow_fast, ctx->want_dir_rows, ctx->want_apply_variant)) return LLP_E_UNSUPPORTED;
  HIP_TRY(hipSetDevice(ctx->device));
  v = ensure_workspace(ctx, g);
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
  const int from_init = params->init_mode == 1;
  if (from_init) {
    if (init != hrms) HIP_TRY(hipMemcpyAsync(hrms, init, NHW * sizeof(float), hipMemcpyDeviceToDevice, s));
    v = apply_A_into(ctx, g, cfg, hrms, kernel, ctx->q, s);
    if (v != LLP_OK) return v;
  }
  HIP_TRY(launch_init(g, from_init, ctx->b, ctx->q, ctx->r[0], hrms, ctx->st, s));

  // CG.  k_dir(k) produces x_k, r_k, p_k and y = D B p_k; k_apply(k) produces q_k = A p_k, alpha_k, beta_k.
  // Residual and direction alternate between two buffers so that no tile reads a neighbour's new values.
  const int nb_dir = dir_ntiles(g, cfg), nb_apply = apply_ntiles(g, cfg);
  HIP_TRY(launch_dir(g, cfg, 1, 0, 0, ctx->r[0], nullptr, nullptr, nullptr, ctx->p[0], hrms, ctx->y, kernel,
                     ctx->partials, ctx->st, max_iters, tol, s));
  HIP_TRY(launch_finalize(g, kFinDir, ctx->partials, nb_dir, ctx->st, nullptr, 0, 0, max_iters, tol, s));
  const bool tol_mode = tol > 0.0f;
  int chunk_no = 0;
  for (int k = 1; k <= max_iters;) {
    const int todo = tol_mode ? (max_iters - k + 1 < kCheckEvery ? max_iters - k + 1 : kCheckEvery)
                              : max_iters - k + 1;
    for (int t = 0; t < todo; ++t, ++k) {
      const int prev = (k - 1) & 1, cur = k & 1;
      hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
      if (ctx->profiling) {
        for (auto& ev : e)
          if (!(ev = timing_event(ctx))) return LLP_E_HIP;
        HIP_TRY(hipEventRecord(e[0], s));
      }
      HIP_TRY(launch_apply(g, cfg, 1, ctx->p[prev], ctx->r[prev], ctx->y, kernel, ctx->G, ctx->MU, ctx->DI, ctx->q,
                           ctx->partials, ctx->st, s));
      if (ctx->profiling) HIP_TRY(hipEventRecord(e[1], s));
      HIP_TRY(launch_finalize(g, kFinApply, ctx->partials, nb_apply, ctx->st, nullptr, 0, 0, 0, 0.0f, s));
      if (ctx->profiling) HIP_TRY(hipEventRecord(e[2], s));
      HIP_TRY(launch_dir(g, cfg, 2, k == max_iters, k, ctx->r[prev], ctx->q, ctx->p[prev], ctx->r[cur],
                         ctx->p[cur], hrms, ctx->y, kernel, ctx->partials, ctx->st, max_iters, tol, s));
      if (ctx->profiling) HIP_TRY(hipEventRecord(e[3], s));
      HIP_TRY(launch_finalize(g, kFinDir, ctx->partials, nb_dir, ctx->st, nullptr, 0, k, max_iters, tol, s));
    }
    if (!tol_mode) break;
    // Poll the band states of the chunk before last while this one runs (at most two chunks in flight).
    const int slot = chunk_no & 1;
    if (chunk_no >= 2) {
      HIP_TRY(hipEventSynchronize(ctx->ev[slot]));
      bool any = false;
      for (int i = 0; i < g.N; ++i) any |= ctx->h_st[i].active != 0;
      if (!any) break;
    }
    HIP_TRY(hipMemcpyAsync(ctx->h_st, ctx->st, sizeof(ChanState) * g.N, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(ctx->ev[slot], s));
    ++chunk_no;
  }

  // The true residual and the objective of the returned iterate.
  if (rep) {
    v = apply_A_into(ctx, g, cfg, hrms, kernel, ctx->q, s);
    if (v != LLP_OK) return v;
    HIP_TRY(launch_residual_norm(g, ctx->b, ctx->q, ctx->partials, ctx->st, ctx->results, s));
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
    const int st = cs.active ? (tol_mode ? LLP_NOT_CONVERGED : LLP_OK) : cs.status;
    if (st < 0 && (worst >= 0 || st < worst)) worst = (llp_status)st;
    if (st > 0 && worst == LLP_OK) worst = (llp_status)st;
    if (rep) {
      llp_report& R = rep[i];
      R.iters = cs.iters;
      R.status = st;
      const double bn2 = cs.bnorm2;
      R.rel_residual = bn2 > 0 ? sqrt(cs.rho / bn2) : sqrt(cs.rho);
      const double tr = ctx->h_results[i * kResultSlots + kSlotTrueRes];
      R.true_rel_residual = bn2 > 0 ? sqrt(tr / bn2) : sqrt(tr);
      R.objective = 0.5 * ctx->h_results[i * kResultSlots + kSlotObjData] +
                    0.5 * (double)g.lam * ctx->h_results[i * kResultSlots + kSlotObjLlp];
    }
  }
  return worst;
}

llp_status llp_pansharpen_batch(llp_ctx* ctx, int S, const llp_shape* shapes, const llp_params* params,
                                const float* const* lrms, const float* const* pan, const float* const* kernel,
                                const float* const* init, float* const* hrms, llp_report* rep, int flags,
                                hipStream_t stream) {
  if (!ctx || !params || S < 0 || (flags & ~(LLP_BATCH_NO_GRAPH | LLP_BATCH_SERIAL)) != 0) return LLP_E_ARG;
  if (S == 0) return LLP_OK;
  if (!shapes || !lrms || !pan || !kernel || !hrms) return LLP_E_ARG;
  const bool from_init = params->init_mode == 1;
  if (from_init && !init) return LLP_E_ARG;
  // Host-side planning: validate every scene, pick its kernels, group the specialised ones into classes.
  std::vector<BatchScene> fast, slow;
  int total_bands = 0;
  for (int i = 0; i < S; ++i) {
    if (!lrms[i] || !pan[i] || !kernel[i] || !hrms[i] || (from_init && !init[i])) return LLP_E_ARG;
    if (!aligned16(hrms[i]) || (from_init && !aligned16(init[i]))) return LLP_E_ARG;
    BatchScene b;
    b.idx = i;
    b.rep0 = total_bands;
    llp_status v = validate(&shapes[i], params, &b.g);
    if (v != LLP_OK) return v;
    if (!pick_config(b.g, &b.cfg, ctx->allow_fast, ctx->want_dir_rows, ctx->want_apply_variant))
      return LLP_E_UNSUPPORTED;
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

  if (!fast.empty()) {
    std::stable_sort(fast.begin(), fast.end(),
                     [](const BatchScene& a, const BatchScene& b) { return a.cls < b.cls; });
    const int nf = (int)fast.size();
    // Workspace: per scene the planes and partials of the single-scene solve, then the band states, the
    // result slots, the input flags and the scene table.
    std::vector<size_t> o_pl(nf), o_part(nf);
    size_t off = 0;
    int nbands = 0;
    for (int i = 0; i < nf; ++i) {
      const Geom& g = fast[i].g;
      const size_t HW = (size_t)g.H * g.W;
      o_pl[i] = off;
      off = align_up(off + (3 * HW + 6 * (size_t)g.N * HW + (size_t)g.N * g.h * g.w) * sizeof(float), 256);
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
    char* base = (char*)ctx->bws;
    ChanState* st = (ChanState*)(base + o_st);
    double* results = (double*)(base + o_res);
    int* bflags = (int*)(base + o_flags);
    SceneDesc* d_table = (SceneDesc*)(base + o_table);
    SceneDesc* tab = ctx->h_table;
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
      d.x = hrms[bs.idx];
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
      d.y = d.q + NHW;
      d.partials = (double*)(base + o_part[i]);
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
        classes.push_back(k);
      }
      BatchClass& k = classes.back();
      // Scenes start on multiples of 8 workgroups, so that the XCD-aware tile order holds within each scene.
      d.dir_block0 = k.dir_blocks;
      d.apply_block0 = k.apply_blocks;
      k.dir_blocks += (int)align_up((size_t)d.dir_ntiles * g.N, 8);
      k.apply_blocks += (int)align_up((size_t)d.apply_ntiles * g.N, 8);
      k.count += 1;
    }
    HIP_TRY(hipMemcpyAsync(d_table, tab, sizeof(SceneDesc) * nf, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(bflags, 0, sizeof(int) * nf, s));
    // Per scene: input checks, PAN statistics, right-hand side, start of CG (x_0, r_0, p_0, rho_0).
    for (int i = 0; i < nf; ++i) {
      const SceneDesc& d = tab[i];
      const Geom& g = d.g;
      const OpConfig& cfg = fast[i].cfg;
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
        HIP_TRY(launch_dir(g, cfg, 0, 0, 0, d.x, nullptr, nullptr, nullptr, nullptr, nullptr, d.y, d.u, d.partials,
                           sst, 0, 0.0f, s));
        HIP_TRY(launch_apply(g, cfg, 0, d.x, nullptr, d.y, d.u, d.G, d.MU, d.DI, d.q, d.partials, sst, s));
      }
      HIP_TRY(launch_init(g, from_init, d.b, d.q, d.r[0], d.x, sst, s));
      HIP_TRY(launch_dir(g, cfg, 1, 0, 0, d.r[0], nullptr, nullptr, nullptr, d.p[0], d.x, d.y, d.u, d.partials,
                         sst, max_iters, tol, s));
      HIP_TRY(launch_finalize(g, kFinDir, d.partials, d.dir_ntiles, sst, nullptr, 0, 0, max_iters, tol, s));
    }

    // CG iterations of all bands together, in chunks of kCheckEvery (even: every chunk starts on parity 0).
    // Timing (llp_set_profiling) needs events between the launches: then the chunks are enqueued directly.
    llp_ctx* prof = ctx->profiling ? ctx : nullptr;
    const bool use_graph = !(flags & LLP_BATCH_NO_GRAPH) && !prof;
    if (use_graph && max_iters > 0) {
      uint32_t tol_bits = 0;
      memcpy(&tol_bits, &tol, sizeof(tol_bits));
      std::vector<long long> key = {(long long)(uintptr_t)d_table, (long long)(uintptr_t)st, nf, nbands, max_iters,
                                    (long long)tol_bits};
      for (const BatchClass& k : classes)
        for (long long x : {(long long)k.C, (long long)k.R, (long long)k.r, (long long)k.dir_rows,
                            (long long)k.variant, (long long)k.first, (long long)k.count, (long long)k.dir_blocks,
                            (long long)k.apply_blocks})
          key.push_back(x);
      if (!ctx->gexec || key != ctx->gkey) {
        if (ctx->gexec) {
          HIP_TRY(hipStreamSynchronize(s));
          (void)hipGraphExecDestroy(ctx->gexec);
          ctx->gexec = nullptr;
          ctx->gkey.clear();
        }
        for (const BatchClass& k : classes) {  // LDS limits are set outside the capture
          HIP_TRY(launch_apply_fast_batch(d_table, k.count, 0, k.C, k.R, k.r, k.variant, 0, st, s));
          HIP_TRY(launch_dir_fast_batch(d_table, k.count, 0, k.C, k.R, k.dir_rows, 0, st, s));
        }
        hipStream_t cs = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        llp_status cv = LLP_OK;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) cv = LLP_E_HIP;
        if (cv == LLP_OK)
          cv = enqueue_batch_iters(classes, d_table, nf, nbands, st, kCheckEvery, 0, max_iters, tol, cs, nullptr);
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
        v = enqueue_batch_iters(classes, d_table, nf, nbands, st, kCheckEvery, 0, max_iters, tol, s, prof);
        if (v != LLP_OK) return v;
      }
      if (!tol_mode) continue;
      // Poll the band states of the chunk before last while this one runs (at most two chunks in flight).
      const int slot = chunk_no & 1;
      if (chunk_no >= 2) {
        HIP_TRY(hipEventSynchronize(ctx->ev[slot]));
        bool any = false;
        for (int i = 0; i < nbands; ++i) any |= ctx->h_bst[slot][i].active != 0;
        if (!any) break;
      }
      HIP_TRY(hipMemcpyAsync(ctx->h_bst[slot], st, sizeof(ChanState) * nbands, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipEventRecord(ctx->ev[slot], s));
      ++chunk_no;
    }

    // True residual and objective of every returned iterate.
    if (rep) {
      for (int i = 0; i < nf; ++i) {
        const SceneDesc& d = tab[i];
        const OpConfig& cfg = fast[i].cfg;
        ChanState* sst = st + d.band0;
        double* sres = results + (size_t)d.band0 * kResultSlots;
        HIP_TRY(launch_dir(d.g, cfg, 0, 0, 0, d.x, nullptr, nullptr, nullptr, nullptr, nullptr, d.y, d.u,
                           d.partials, sst, 0, 0.0f, s));
        HIP_TRY(launch_apply(d.g, cfg, 0, d.x, nullptr, d.y, d.u, d.G, d.MU, d.DI, d.q, d.partials, sst, s));
        HIP_TRY(launch_residual_norm(d.g, d.b, d.q, d.partials, sst, sres, s));
        HIP_TRY(launch_objective(d.g, d.x, d.X, d.u, d.G, d.MU, d.DI, d.partials, sst, sres, s));
      }
      HIP_TRY(hipMemcpyAsync(ctx->h_bres, results, sizeof(double) * kResultSlots * nbands, hipMemcpyDeviceToHost,
                             s));
    }
    HIP_TRY(hipMemcpyAsync(ctx->h_bst[0], st, sizeof(ChanState) * nbands, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(ctx->h_bflags, bflags, sizeof(int) * nf, hipMemcpyDeviceToHost, s));
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
                                          : (cs.active ? (tol_mode ? LLP_NOT_CONVERGED : LLP_OK) : cs.status);
        merge(bst);
        if (rep) {
          llp_report& R = rep[fast[i].rep0 + c];
          const double* res = ctx->h_bres + (size_t)(d.band0 + c) * kResultSlots;
          R.iters = cs.iters;
          R.status = bst;
          const double bn2 = cs.bnorm2;
          R.rel_residual = bn2 > 0 ? sqrt(cs.rho / bn2) : sqrt(cs.rho);
          R.true_rel_residual = bn2 > 0 ? sqrt(res[kSlotTrueRes] / bn2) : sqrt(res[kSlotTrueRes]);
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

llp_status llp_set_profiling(llp_ctx* ctx, int enable) {
  if (!ctx) return LLP_E_ARG;
  ctx->profiling = enable != 0;
  return LLP_OK;
}

llp_status llp_get_kernel_times(llp_ctx* ctx, llp_kernel_times* out, int reset) {
  if (!ctx || !out) return LLP_E_ARG;
  *out = ctx->times;
  if (reset) ctx->times = llp_kernel_times{0.0, 0, 0.0, 0};
  return LLP_OK;
}

}  // extern "C"
