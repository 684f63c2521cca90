// C ABI of the warm-start network (declared in include/llp.h): weights, inference (the initial guess of the
// CG solve) and training (loss, gradients, Adam), on the kernels of llp_cnn.hip.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <new>

#include "llp_ctx.h"

using namespace llp;
using namespace llp::host;

namespace {

constexpr size_t kInferBytes = (size_t)4 << 30;  // activation budget of one inference chunk of bands
constexpr size_t kActBytesPerPixel = 32 * 2;     // one padded bfloat16 activation

int fwd_blocks(int l) { return cnn_layer_cout(l) > 16 ? 2 : 1; }
const float* bias_of(const CnnState* c, int l) {
  return c->master + cnn_layer_offset(l) + cnn_layer_cout(l) * cnn_layer_cin(l) * 9;
}

llp_status prep_all(CnnState* c, hipStream_t s) {
  for (int l = 0; l < kCnnLayers; ++l) {
    const float* W = c->master + cnn_layer_offset(l);
    HIP_TRY(cnn_launch_prep(W, cnn_layer_cout(l), cnn_layer_cin(l), fwd_blocks(l), 0, c->fwd[l], s));
    if (l > 0) HIP_TRY(cnn_launch_prep(W, cnn_layer_cout(l), cnn_layer_cin(l), 2, 1, c->bwd[l], s));
  }
  return LLP_OK;
}

// Workspace views for `nb` bands of HW pixels; train: all five activations and the gradient buffers.
struct CnnViews {
  float *stats, *xup, *net;
  double* spart;  // partial sums of the band statistics
  uint16_t* act[kCnnLayers];
  uint16_t* gbuf[2];
  float* wpart;
  double *lpart, *loss;
};

llp_status cnn_workspace(CnnState* c, int N, int nb, size_t HW, bool train, CnnViews* v) {
  const int nact = train ? kCnnLayers : 2;
  const size_t act = align_up((size_t)nb * HW * kActBytesPerPixel, 256);
  size_t off = 0;
  const size_t o_stats = off;
  off = align_up(off + sizeof(float) * 2 * (N + 1), 256);
  const size_t o_spart = off;  // chunks of the band statistics: N LRMS bands and the PAN image
  off = align_up(off + sizeof(double) * 2 * ((size_t)N * cnn_stats_parts(HW / 1) + cnn_stats_parts(HW)), 256);
  const size_t o_xup = off;
  off = align_up(off + sizeof(float) * nb * HW, 256);
  const size_t o_net = off;
  off = align_up(off + sizeof(float) * nb * HW, 256);
  const size_t o_act = off;
  off += act * nact;
  const size_t o_g = off;
  if (train) off += 2 * act;
  const size_t o_wp = off;
  if (train) off = align_up(off + sizeof(float) * cnn_wgrad_parts() * cnn_wgrad_part_floats(), 256);
  const size_t o_lp = off;
  const size_t nlp = ((size_t)nb * HW + 255) / 256;
  if (train) off = align_up(off + sizeof(double) * (nlp + 1), 256);
  if (off > c->ws_bytes) {
    if (c->ws) {
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(c->ws));
      c->ws = nullptr;
      c->ws_bytes = 0;
    }
    if (hipMalloc(&c->ws, off) != hipSuccess) {
      c->ws = nullptr;
      return LLP_E_OOM;
    }
    c->ws_bytes = off;
  }
  char* base = (char*)c->ws;
  v->stats = (float*)(base + o_stats);
  v->spart = (double*)(base + o_spart);
  v->xup = (float*)(base + o_xup);
  v->net = (float*)(base + o_net);
  for (int l = 0; l < kCnnLayers; ++l) v->act[l] = l < nact ? (uint16_t*)(base + o_act + act * l) : nullptr;
  v->gbuf[0] = train ? (uint16_t*)(base + o_g) : nullptr;
  v->gbuf[1] = train ? (uint16_t*)(base + o_g + act) : nullptr;
  v->wpart = train ? (float*)(base + o_wp) : nullptr;
  v->lpart = train ? (double*)(base + o_lp) : nullptr;
  v->loss = train ? v->lpart + nlp : nullptr;
  return LLP_OK;
}

CnnGeom cnn_geom(const Geom& g, int nb) { return CnnGeom{nb, g.H, g.W, g.h, g.w, g.c}; }

// Forward pass over all bands keeping every activation, the loss against Z and the gradient in c->grad.
llp_status loss_grad(llp_ctx* ctx, const Geom& g, const float* X, const float* Y, const float* Z, hipStream_t s,
                     CnnViews* out) {
  CnnState* c = ctx->cnn;
  const size_t HW = (size_t)g.H * g.W;
  CnnViews v;
  llp_status st = cnn_workspace(c, g.N, g.N, HW, true, &v);
  if (st != LLP_OK) return st;
  const CnnGeom cg = cnn_geom(g, g.N);
  HIP_TRY(cnn_launch_stats(X, (size_t)g.h * g.w, (size_t)g.h * g.w, g.N, v.spart, v.stats, s));
  HIP_TRY(cnn_launch_stats(Y, 0, HW, 1, v.spart, v.stats + 2 * g.N, s));
  HIP_TRY(cnn_launch_input(cg, X, Y, v.stats, v.stats + 2 * g.N, v.xup, v.act[0], s));
  for (int l = 0; l < kCnnLayers - 1; ++l)
    HIP_TRY(cnn_launch_conv(cg, 2, 0, v.act[l], c->fwd[l], bias_of(c, l), v.act[l + 1], nullptr, nullptr, nullptr,
                            nullptr, nullptr, s));
  HIP_TRY(cnn_launch_conv(cg, 1, 1, v.act[kCnnLayers - 1], c->fwd[kCnnLayers - 1], bias_of(c, kCnnLayers - 1),
                          nullptr, nullptr, v.net, nullptr, v.xup, v.stats, s));
  HIP_TRY(cnn_launch_loss(cg, v.net, Z, v.xup, v.stats, v.gbuf[0], v.lpart, v.loss, s));
  // backward: gradient of layer l's output in gbuf[cur]; weight gradient, then the input gradient
  int cur = 0;
  for (int l = kCnnLayers - 1; l >= 0; --l) {
    HIP_TRY(cnn_launch_wgrad(cg, v.gbuf[cur], v.act[l], v.wpart, cnn_layer_cout(l), cnn_layer_cin(l),
                             c->grad + cnn_layer_offset(l), s));
    if (l > 0) {
      HIP_TRY(cnn_launch_conv(cg, 2, 2, v.gbuf[cur], c->bwd[l], nullptr, v.gbuf[1 - cur], v.act[l], nullptr, nullptr,
                              nullptr, nullptr, s));
      cur = 1 - cur;
    }
  }
  *out = v;
  return LLP_OK;
}

}  // namespace

namespace llp {
namespace host {

void cnn_free(CnnState* c) {
  if (!c) return;
  if (c->mem) (void)hipFree(c->mem);
  if (c->ws) (void)hipFree(c->ws);
  if (c->h_loss) (void)hipHostFree(c->h_loss);
  delete c;
}

llp_status cnn_warm_start(llp_ctx* ctx, const Geom& g, const float* X, const float* Y, float* z0, float* netout,
                          hipStream_t s) {
  CnnState* c = ctx->cnn;
  if (!c) return LLP_E_ARG;
  const size_t HW = (size_t)g.H * g.W;
  size_t nb = kInferBytes / (HW * 2 * kActBytesPerPixel + 1);
  if (nb < 1) nb = 1;
  if (nb > (size_t)g.N) nb = g.N;
  CnnViews v;
  llp_status st = cnn_workspace(c, g.N, (int)nb, HW, false, &v);
  if (st != LLP_OK) return st;
  HIP_TRY(cnn_launch_stats(X, (size_t)g.h * g.w, (size_t)g.h * g.w, g.N, v.spart, v.stats, s));
  HIP_TRY(cnn_launch_stats(Y, 0, HW, 1, v.spart, v.stats + 2 * g.N, s));
  for (int b0 = 0; b0 < g.N; b0 += (int)nb) {
    const int n = g.N - b0 < (int)nb ? g.N - b0 : (int)nb;
    const CnnGeom cg = cnn_geom(g, n);
    HIP_TRY(cnn_launch_input(cg, X + (size_t)b0 * g.h * g.w, Y, v.stats + 2 * b0, v.stats + 2 * g.N, v.xup,
                             v.act[0], s));
    for (int l = 0; l < kCnnLayers - 1; ++l)
      HIP_TRY(cnn_launch_conv(cg, 2, 0, v.act[l & 1], c->fwd[l], bias_of(c, l), v.act[(l + 1) & 1], nullptr, nullptr,
                              nullptr, nullptr, nullptr, s));
    HIP_TRY(cnn_launch_conv(cg, 1, 1, v.act[(kCnnLayers - 1) & 1], c->fwd[kCnnLayers - 1],
                            bias_of(c, kCnnLayers - 1), nullptr, nullptr, netout ? netout + (size_t)b0 * HW : nullptr,
                            z0 ? z0 + (size_t)b0 * HW : nullptr, v.xup, v.stats + 2 * b0, s));
  }
  return LLP_OK;
}

}  // namespace host
}  // namespace llp

extern "C" {

llp_status llp_cnn_set_weights(llp_ctx* ctx, const float* params, int count) {
  if (!ctx || !params || count != LLP_CNN_PARAMS) return LLP_E_ARG;
  for (int i = 0; i < count; ++i)
    if (!isfinite(params[i])) return LLP_E_NONFINITE;
  HIP_TRY(hipSetDevice(ctx->device));
  if (!ctx->cnn) {
    CnnState* c = new (std::nothrow) CnnState();
    if (!c) return LLP_E_OOM;
    const size_t pbytes = align_up(sizeof(float) * kCnnParams, 256);
    const size_t tile = align_up(cnn_tile_bytes(2), 256);
    if (hipMalloc(&c->mem, 4 * pbytes + 2 * kCnnLayers * tile) != hipSuccess ||
        hipHostMalloc((void**)&c->h_loss, sizeof(double), hipHostMallocDefault) != hipSuccess) {
      cnn_free(c);
      return LLP_E_OOM;
    }
    char* b = (char*)c->mem;
    c->master = (float*)b;
    c->m = (float*)(b + pbytes);
    c->v = (float*)(b + 2 * pbytes);
    c->grad = (float*)(b + 3 * pbytes);
    for (int l = 0; l < kCnnLayers; ++l) {
      c->fwd[l] = b + 4 * pbytes + (size_t)(2 * l) * tile;
      c->bwd[l] = b + 4 * pbytes + (size_t)(2 * l + 1) * tile;
    }
    ctx->cnn = c;
  }
  CnnState* c = ctx->cnn;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(c->master, params, sizeof(float) * kCnnParams, hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(c->m, 0, sizeof(float) * kCnnParams));
  HIP_TRY(hipMemset(c->v, 0, sizeof(float) * kCnnParams));
  c->steps = 0;
  llp_status st = prep_all(c, 0);
  if (st != LLP_OK) return st;
  HIP_TRY(hipDeviceSynchronize());
  return LLP_OK;
}

llp_status llp_cnn_get_weights(llp_ctx* ctx, float* params, int count) {
  if (!ctx || !params || count != LLP_CNN_PARAMS) return LLP_E_ARG;
  if (!ctx->cnn) return LLP_E_ARG;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(params, ctx->cnn->master, sizeof(float) * kCnnParams, hipMemcpyDeviceToHost));
  return LLP_OK;
}

llp_status llp_cnn_warm_start(llp_ctx* ctx, const llp_shape* shape, const float* lrms, const float* pan,
                              float* z0, float* net_out, hipStream_t stream) {
  if (!ctx || !lrms || !pan || (!z0 && !net_out)) return LLP_E_ARG;
  if (!ctx->cnn) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, nullptr, &g);
  if (v != LLP_OK) return v;
  HIP_TRY(hipSetDevice(ctx->device));
  return cnn_warm_start(ctx, g, lrms, pan, z0, net_out, stream);
}

llp_status llp_cnn_loss_grad(llp_ctx* ctx, const llp_shape* shape, const float* lrms, const float* pan,
                             const float* target, double* loss, float* grads, hipStream_t stream) {
  if (!ctx || !lrms || !pan || !target) return LLP_E_ARG;
  if (!ctx->cnn) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, nullptr, &g);
  if (v != LLP_OK) return v;
  HIP_TRY(hipSetDevice(ctx->device));
  CnnViews views;
  v = loss_grad(ctx, g, lrms, pan, target, stream, &views);
  if (v != LLP_OK) return v;
  HIP_TRY(hipMemcpyAsync(ctx->cnn->h_loss, views.loss, sizeof(double), hipMemcpyDeviceToHost, stream));
  if (grads)
    HIP_TRY(hipMemcpyAsync(grads, ctx->cnn->grad, sizeof(float) * kCnnParams, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (loss) *loss = *ctx->cnn->h_loss;
  return LLP_OK;
}

llp_status llp_cnn_train_step(llp_ctx* ctx, const llp_shape* shape, const float* lrms, const float* pan,
                              const float* target, float lr, double* loss, hipStream_t stream) {
  if (!ctx || !lrms || !pan || !target || !(lr > 0.0f) || !isfinite(lr)) return LLP_E_ARG;
  if (!ctx->cnn) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, nullptr, &g);
  if (v != LLP_OK) return v;
  HIP_TRY(hipSetDevice(ctx->device));
  CnnState* c = ctx->cnn;
  CnnViews views;
  v = loss_grad(ctx, g, lrms, pan, target, stream, &views);
  if (v != LLP_OK) return v;
  c->steps += 1;
  HIP_TRY(cnn_launch_adam(c->master, c->grad, c->m, c->v, kCnnParams, lr, c->steps, stream));
  v = prep_all(c, stream);
  if (v != LLP_OK) return v;
  if (loss) {
    HIP_TRY(hipMemcpyAsync(c->h_loss, views.loss, sizeof(double), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    *loss = *c->h_loss;
  }
  return LLP_OK;
}

}  // extern "C"
