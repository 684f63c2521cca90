// Internal declarations shared by the kernels (llp_kernels.hip) and the C ABI (llp_api.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace llp {

// Sizes of one scene, plus the solver's scalar parameters.
struct Geom {
  int N, H, W, h, w, c, n, R, r;
  float lam, eps;
};

// Per-band conjugate-gradient state, resident in device memory for the whole solve.
struct ChanState {
  double rho;     // r^T r of the current residual
  double bnorm2;  // ||b||^2
  double alpha;   // step of the current iteration
  double beta;    // rho_new / rho_old, used to form the next direction
  double gamma;   // p^T A p of the current iteration
  int iters;      // iterations completed
  int active;     // 1 while the band still iterates
  int status;     // llp_status of the band
  int pad;
};

// Reduction slots in the per-band result array (doubles [N][kResultSlots]).
enum ResultSlot { kSlotTrueRes = 0, kSlotObjData = 1, kSlotObjLlp = 2, kResultSlots = 4 };

// LDS layout of the tiled operator kernel.  All sizes in floats; computed on the host from the tile shape.
struct ApplyLayout {
  int TH, TW;         // output tile
  int E;              // halo of the staged input region: max(2R, 2r+2)
  int PH, PW;         // staged input region (TH+2E) x (TW+2E)
  int YHm, YWm;       // capacity of the low-resolution intermediate D B p of the tile
  int LH, LW;         // l = L p region: (TH + 2(2r+1)) x (TW + 2(2r+1))
  int AH, AW;         // window-coefficient region: (TH + 2(r+1)) x (TW + 2(r+1))
  int offP, offL, offX, offY, offU;
  int total;          // floats
};

ApplyLayout apply_layout(int TH, int TW, int R, int r, int c, int n);

struct Workspace;  // defined in llp_api.hip

// Tile shapes the operator kernel is built for (index = variant id).
struct TileShape { int TH, TW; };
constexpr int kNumTileVariants = 5;
extern const TileShape kTileVariants[kNumTileVariants];

// Kernel launchers (llp_kernels.hip).  All enqueue on `s` and return the launch status.
hipError_t launch_pan_stats(const Geom& g, const float* Y, float* G, float* mu, float* dinv, int* flag,
                            hipStream_t s);
hipError_t launch_check_finite(const float* a, size_t count, int* flag, hipStream_t s);
hipError_t launch_rhs(const Geom& g, const float* X, const float* u, float* b, double* partials,
                      unsigned* counters, ChanState* st, hipStream_t s);
// mode 0: q = A z.  mode 1: CG direction update p_new = r + beta p_old, q = A p_new, gamma = p_new^T q.
hipError_t launch_apply(const Geom& g, int variant, int mode, const float* zr, const float* p_old, float* p_new,
                        const float* u, const float* G, const float* mu, const float* dinv, float* q,
                        double* partials, unsigned* counters, ChanState* st, hipStream_t s);
hipError_t launch_init_residual(const Geom& g, int from_init, const float* b, const float* q, float* r,
                                float* x, double* partials, unsigned* counters, ChanState* st, int max_iters,
                                float tol, hipStream_t s);
hipError_t launch_cg_update(const Geom& g, float* x, float* r, const float* p, const float* q, double* partials,
                            unsigned* counters, ChanState* st, int max_iters, float tol, hipStream_t s);
hipError_t launch_residual_norm(const Geom& g, const float* b, const float* q, double* partials,
                                unsigned* counters, double* results, hipStream_t s);
hipError_t launch_objective(const Geom& g, const float* z, const float* X, const float* u, const float* G,
                            const float* mu, const float* dinv, double* partials, unsigned* counters,
                            double* results, hipStream_t s);

// Maximum number of reduction partials per band any launcher needs for geometry g.
size_t max_partials_per_band(const Geom& g);

}  // namespace llp
