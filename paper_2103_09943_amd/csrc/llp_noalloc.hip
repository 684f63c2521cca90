// llp_apply_A_noalloc: the product with the matrix of eq. (Z_ini_matting) for callers that cannot allocate
// device memory.  The PAN statistics (G, mu, dinv) and y = D B z, which llp_apply_A keeps in its context's
// workspace, live here in one file-scope device array of fixed size; each device holds its own copy for the
// life of the process.  Its address is looked up once per device with the device current, and only that
// address is passed to kernels.
#include <mutex>

#include "llp_ctx.h"

using namespace llp;
using namespace llp::host;

namespace {

constexpr int kMaxDevices = 64;
__device__ __align__(256) float scratch[LLP_NOALLOC_SCRATCH_FLOATS];

std::mutex g_mutex;
float* g_scratch[kMaxDevices] = {};  // device address of `scratch` on every device seen so far

// The scratch array's address on the current device (looked up on the first call on that device).
llp_status scratch_on_current_device(float** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LLP_E_HIP;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LLP_E_HIP;
    g_scratch[dev] = (float*)p;
  }
  *out = g_scratch[dev];
  return LLP_OK;
}

}  // namespace

extern "C" llp_status llp_apply_A_noalloc(const llp_shape* shape, const llp_params* params, const float* pan,
                                          const float* kernel, const float* z, float* Az, hipStream_t stream) {
  if (!params || !pan || !kernel || !z || !Az || z == Az) return LLP_E_ARG;
  if (!aligned16(z) || !aligned16(Az)) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, params, &g);
  if (v != LLP_OK) return v;
  // Each region starts on a 256-byte boundary (the kernels use vector loads on all of them).
  const size_t HW = ((size_t)g.H * g.W + 63) & ~(size_t)63;
  const size_t need = 3 * HW + (size_t)g.N * g.h * g.w;
  if (need > (size_t)LLP_NOALLOC_SCRATCH_FLOATS) return LLP_E_UNSUPPORTED;
  OpConfig cfg;
  if (!pick_config(g, &cfg)) return LLP_E_UNSUPPORTED;
  float* base = nullptr;
  v = scratch_on_current_device(&base);
  if (v != LLP_OK) return v;
  float* G = base;
  float* MU = G + HW;
  float* DI = MU + HW;
  float* y = DI + HW;
  // Every scratch region is written before it is read: the statistics by the first launch, y by the second.
  HIP_TRY(launch_pan_stats(g, pan, G, MU, DI, stream));
  HIP_TRY(launch_dir(g, cfg, 0, 0, 0, z, nullptr, nullptr, nullptr, nullptr, nullptr, y, kernel, nullptr, nullptr, 0,
                     0.0f, stream));
  HIP_TRY(launch_apply(g, cfg, 0, z, nullptr, y, kernel, G, MU, DI, Az, nullptr, nullptr, stream));
  return LLP_OK;
}
