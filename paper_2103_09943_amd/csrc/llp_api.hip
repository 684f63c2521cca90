// C ABI of libllp (declared in include/llp.h): argument validation, workspaces and the host side of the
// conjugate-gradient solve of eq. (Z_ini_matting), Sec. III-B.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "llp.h"
#include "llp_internal.h"

using namespace llp;

struct llp_ctx {
  int device = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // views into ws
  float *G = nullptr, *MU = nullptr, *DI = nullptr, *b = nullptr, *r = nullptr, *p0 = nullptr, *p1 = nullptr,
        *q = nullptr;
  double* partials = nullptr;
  unsigned* counters = nullptr;  // own allocation: stays at zero between kernels whatever the geometry
  int cnt_cap = 0;
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
  std::vector<hipEvent_t> tev;  // timing events, 3 per iteration
  size_t tev_used = 0;
  llp_kernel_times times = {0.0, 0, 0.0, 0};
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

llp_status validate(const llp_shape* s, const llp_params* p, Geom* g) {
  if (!s) return LLP_E_ARG;
  if (s->N < 1 || s->h < 1 || s->w < 1 || s->c < 1 || s->n < 1) return LLP_E_SHAPE;
  if ((s->n & 1) == 0) return LLP_E_SHAPE;
  if (s->c > LLP_MAX_SCALE || s->n > LLP_MAX_KERNEL) return LLP_E_UNSUPPORTED;
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

// Tile variant for the operator kernel: the first (in preference order) whose LDS layout fits.
int pick_variant(const Geom& g) {
  static const int order[] = {0, 2, 1, 4, 3};
  for (int v : order) {
    const ApplyLayout L = apply_layout(kTileVariants[v].TH, kTileVariants[v].TW, g.R, g.r, g.c, g.n);
    if (L.total <= kMaxLdsFloats) return v;
  }
  return -1;
}

llp_status ensure_workspace(llp_ctx* ctx, const Geom& g) {
  const size_t HW = (size_t)g.H * g.W;
  const size_t planes = 3 * HW + 5 * (size_t)g.N * HW;
  const size_t pstride = max_partials_per_band(g);
  size_t off = 0;
  const size_t o_planes = off;
  off = align_up(off + planes * sizeof(float), 256);
  const size_t o_part = off;
  off = align_up(off + (size_t)g.N * pstride * sizeof(double), 256);
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
  ctx->r = ctx->b + NHW;
  ctx->p0 = ctx->r + NHW;
  ctx->p1 = ctx->p0 + NHW;
  ctx->q = ctx->p1 + NHW;
  ctx->partials = (double*)(base + o_part);
  ctx->st = (ChanState*)(base + o_st);
  ctx->results = (double*)(base + o_res);
  ctx->flags = (int*)(base + o_flags);
  // Reduction counters: every reduction kernel's last block resets its band's counter, so the array is all
  // zero between kernels; it is zeroed once when (re)allocated and never moves with the geometry.
  if (ctx->cnt_cap < g.N) {
    if (ctx->counters) {
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(ctx->counters));
      ctx->counters = nullptr;
      ctx->cnt_cap = 0;
    }
    if (hipMalloc((void**)&ctx->counters, sizeof(unsigned) * g.N) != hipSuccess) return LLP_E_OOM;
    HIP_TRY(hipMemset(ctx->counters, 0, sizeof(unsigned) * g.N));
    ctx->cnt_cap = g.N;
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
  for (size_t i = 0; i + 2 < ctx->tev_used; i += 3) {
    float a = 0.0f, b = 0.0f;
    HIP_TRY(hipEventElapsedTime(&a, ctx->tev[i], ctx->tev[i + 1]));
    HIP_TRY(hipEventElapsedTime(&b, ctx->tev[i + 1], ctx->tev[i + 2]));
    ctx->times.apply_ms += a;
    ctx->times.update_ms += b;
    ctx->times.apply_launches += 1;
    ctx->times.update_launches += 1;
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
  if (params && pick_variant(g) < 0) return LLP_E_UNSUPPORTED;
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
  if (ctx->counters) (void)hipFree(ctx->counters);
  if (ctx->h_st) (void)hipHostFree(ctx->h_st);
  if (ctx->h_results) (void)hipHostFree(ctx->h_results);
  if (ctx->h_flags) (void)hipHostFree(ctx->h_flags);
  for (auto& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : ctx->tev) (void)hipEventDestroy(e);
  delete ctx;
}

llp_status llp_pan_stats(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* pan,
                         float* G, float* mu, float* dinv, hipStream_t stream) {
  if (!ctx || !params || !pan || !G || !mu || !dinv) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, params, &g);
  if (v != LLP_OK) return v;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(launch_pan_stats(g, pan, G, mu, dinv, nullptr, stream));
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
  HIP_TRY(launch_rhs(g, lrms, kernel, b, ctx->partials, ctx->counters, ctx->st, stream));
  return LLP_OK;
}

llp_status llp_apply_A(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* pan,
                       const float* kernel, const float* z, float* Az, hipStream_t stream) {
  if (!ctx || !params || !pan || !kernel || !z || !Az || z == Az) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, params, &g);
  if (v != LLP_OK) return v;
  const int variant = pick_variant(g);
  if (variant < 0) return LLP_E_UNSUPPORTED;
  HIP_TRY(hipSetDevice(ctx->device));
  v = ensure_workspace(ctx, g);
  if (v != LLP_OK) return v;
  HIP_TRY(launch_pan_stats(g, pan, ctx->G, ctx->MU, ctx->DI, nullptr, stream));
  HIP_TRY(launch_apply(g, variant, 0, z, nullptr, nullptr, kernel, ctx->G, ctx->MU, ctx->DI, Az, ctx->partials,
                       ctx->counters, ctx->st, stream));
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
  HIP_TRY(launch_pan_stats(g, pan, ctx->G, ctx->MU, ctx->DI, nullptr, stream));
  HIP_TRY(launch_objective(g, z, lrms, kernel, ctx->G, ctx->MU, ctx->DI, ctx->partials, ctx->counters, ctx->results,
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
  Geom g;
  llp_status v = validate(shape, params, &g);
  if (v != LLP_OK) return v;
  const int variant = pick_variant(g);
  if (variant < 0) return LLP_E_UNSUPPORTED;
  HIP_TRY(hipSetDevice(ctx->device));
  v = ensure_workspace(ctx, g);
  if (v != LLP_OK) return v;
  hipStream_t s = stream;
  const size_t NHW = (size_t)g.N * g.H * g.W;

  v = check_inputs(ctx, g, lrms, pan, kernel, s);
  if (v != LLP_OK) return v;
  // Per scene: the statistics that define M_LY, then the right-hand sides and ||b||.
  HIP_TRY(launch_pan_stats(g, pan, ctx->G, ctx->MU, ctx->DI, nullptr, s));
  HIP_TRY(launch_rhs(g, lrms, kernel, ctx->b, ctx->partials, ctx->counters, ctx->st, s));
  const int from_init = params->init_mode == 1;
  if (from_init) {
    if (init != hrms) HIP_TRY(hipMemcpyAsync(hrms, init, NHW * sizeof(float), hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_apply(g, variant, 0, hrms, nullptr, nullptr, kernel, ctx->G, ctx->MU, ctx->DI, ctx->q,
                         ctx->partials, ctx->counters, ctx->st, s));
  }
  HIP_TRY(launch_init_residual(g, from_init, ctx->b, ctx->q, ctx->r, hrms, ctx->partials, ctx->counters, ctx->st,
                               params->max_iters, params->tol, s));

  // CG iterations.  Two direction buffers alternate so that a tile never reads a neighbour's new direction.
  const bool tol_mode = params->tol > 0.0f;
  int chunk_no = 0;
  for (int it = 0; it < params->max_iters;) {
    const int todo = tol_mode ? (params->max_iters - it < kCheckEvery ? params->max_iters - it : kCheckEvery)
                              : params->max_iters - it;
    for (int k = 0; k < todo; ++k, ++it) {
      float* p_prev = (it & 1) ? ctx->p1 : ctx->p0;
      float* p_cur = (it & 1) ? ctx->p0 : ctx->p1;
      hipEvent_t t0 = nullptr, t1 = nullptr, t2 = nullptr;
      if (ctx->profiling) {
        t0 = timing_event(ctx);
        t1 = timing_event(ctx);
        t2 = timing_event(ctx);
        if (!t0 || !t1 || !t2) return LLP_E_HIP;
        HIP_TRY(hipEventRecord(t0, s));
      }
      HIP_TRY(launch_apply(g, variant, 1, ctx->r, p_prev, p_cur, kernel, ctx->G, ctx->MU, ctx->DI, ctx->q,
                           ctx->partials, ctx->counters, ctx->st, s));
      if (ctx->profiling) HIP_TRY(hipEventRecord(t1, s));
      HIP_TRY(launch_cg_update(g, hrms, ctx->r, p_cur, ctx->q, ctx->partials, ctx->counters, ctx->st,
                               params->max_iters, params->tol, s));
      if (ctx->profiling) HIP_TRY(hipEventRecord(t2, s));
    }
    if (!tol_mode) break;
    // Poll the band states of the previous chunk while this one runs; keep at most two chunks in flight.
    const int slot = chunk_no & 1;
    if (chunk_no >= 2) {
      HIP_TRY(hipEventSynchronize(ctx->ev[slot]));
      bool any = false;
      const ChanState* hs = ctx->h_st;
      for (int i = 0; i < g.N; ++i) any |= hs[i].active != 0;
      if (!any) break;
    }
    HIP_TRY(hipMemcpyAsync(ctx->h_st, ctx->st, sizeof(ChanState) * g.N, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(ctx->ev[slot], s));
    ++chunk_no;
  }

  // Final states, the true residual and the objective of the returned iterate.
  if (rep) {
    HIP_TRY(launch_apply(g, variant, 0, hrms, nullptr, nullptr, kernel, ctx->G, ctx->MU, ctx->DI, ctx->q,
                         ctx->partials, ctx->counters, ctx->st, s));
    HIP_TRY(launch_residual_norm(g, ctx->b, ctx->q, ctx->partials, ctx->counters, ctx->results, s));
    HIP_TRY(launch_objective(g, hrms, lrms, kernel, ctx->G, ctx->MU, ctx->DI, ctx->partials, ctx->counters,
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
