// Internal declarations shared by the kernels (llp_kernels.hip, llp_operator.hip) and the C ABI (llp_api.hip).
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
  double rho;     // r_k^T r_k (summed directly)
  double bnorm2;  // ||b||^2
  double alpha;   // rho_k / (p_k^T A p_k)
  double beta;    // ||r_k - alpha q_k||^2 / rho_k
  double gamma;   // p_k^T A p_k
  int iters;      // index of the current iterate x_k
  int active;     // 1 while the band still iterates
  int status;     // llp_status of the band
  int init;       // how the band started: kInitZero, kInitUser, kInitNet, kInitNetRejected
};

enum InitKind { kInitZero = 0, kInitUser = 1, kInitNet = 2, kInitNetRejected = 3 };

// What k_finalize does with a band's summed partials.
enum FinOp { kFinBnorm = 0, kFinResult = 1, kFinDir = 2, kFinApply = 3 };

// Reduction slots in the per-band result array (doubles [N][kResultSlots]).
enum ResultSlot { kSlotTrueRes = 0, kSlotObjData = 1, kSlotObjLlp = 2, kResultSlots = 4 };

// Launch configuration of the two iteration kernels (chosen per geometry, see the autotuner).
struct OpConfig {
  int fast;           // 1: kernels specialised on (c, R, r) (fast_path_available), 0: generic kernels
  int dir_rows;       // generic k_dir: LR rows per tile, 4 or 8 (64 LR columns)
  int apply_variant;  // k_apply tile shape index: generic 0 .. kApplyVariants-1 (apply_tile()); fast 0: 32x64,
                      // 1: 16x64, 2: the column sweep k_llp (llp_sweep.hip)
  int seg_rows;       // column sweep: rows per segment
};
constexpr int kSweepVariant = 2;
constexpr int kMinSegRows = 32;  // shortest sweep segment the partial-sum buffers are sized for
bool fast_path_available(int C, int R, int r);
bool fast_path_fits(const Geom& g, int dir_rows, int apply_variant);
int fast_apply_lds_floats(int C, int R, int r, int variant);
constexpr int kApplyVariants = 3;
constexpr int kMaxScale = 4;  // scale factors with built kernels: 1..4

// LDS sizes (floats) of the two iteration kernels; outputs their layout parameters.
int dir_lds_floats(int C, int TYL, int R, int* PS_out);
int apply_lds_floats(int C, int TH, int TW, int R, int r, int* offL, int* offX, int* offY, int* QPS_out);
int apply_tile(int C, int variant, int* TH, int* TW);

// Kernel launchers.  All enqueue on `s` and return the launch status.  Reductions leave their partial sums in
// `partials` and finish with a k_finalize launch.
// G = L Y, the window means mu of G and dinv = 1 / (var + eps / |w|), as planes.
hipError_t launch_pan_stats(const Geom& g, const float* Y, float* G, float* mu, float* dinv, hipStream_t s);
hipError_t launch_check_finite(const float* a, size_t count, int* flag, hipStream_t s);
hipError_t launch_finalize(const Geom& g, int op, const double* partials, int nblk, ChanState* st,
                           double* results, int slot, int k_iter, int max_iters, float tol, hipStream_t s);
// b = B^T D^T X and ||b||^2 (into the band states).
hipError_t launch_rhs(const Geom& g, const float* X, const float* u, float* b, double* partials, ChanState* st,
                      hipStream_t s);
// r_0 = b (Z = 0, x set to 0) or r_0 = b - q (q = A Z0, x already Z0); resets the band states.
hipError_t launch_init(const Geom& g, int from_init, const float* b, const float* q, float* r, float* x,
                       ChanState* st, hipStream_t s);
// mode 0: y = D B z (z = rin).  mode 1: p_0 = r_0 (rin), y = D B p_0, partials of rho_0.  mode 2: the update
// of iteration k (x, r from alpha; p from beta), y = D B p_k, partials of rho_k; final_step skips p and y.
// Modes 1 and 2 are followed by launch_finalize(kFinDir, nblk = dir_ntiles) for the stopping rule of x_k.
hipError_t launch_dir(const Geom& g, const OpConfig& cfg, int mode, int final_step, int k_iter, const float* rin,
                      const float* qin, const float* pin, float* rout, float* pout, float* x, float* y,
                      const float* u, double* partials, ChanState* st, int max_iters, float tol, hipStream_t s);
// mode 0: q = A z (z = p, y = D B z).  mode 1: q = A p_k and partials of the dot products; followed by
// launch_finalize(kFinApply, nblk = apply_ntiles) for alpha_k, beta_k.
hipError_t launch_apply(const Geom& g, const OpConfig& cfg, int mode, const float* p, const float* r,
                        const float* y, const float* u, const float* G, const float* mu, const float* dinv,
                        float* q, double* partials, ChanState* st, hipStream_t s);
int dir_ntiles(const Geom& g, const OpConfig& cfg);
int apply_ntiles(const Geom& g, const OpConfig& cfg);
// After a network start: bands whose start is no better than zero restart from zero (see k_fallback).
hipError_t launch_fallback(const Geom& g, const double* results, ChanState* st, const float* b, float* r, float* x,
                           hipStream_t s);
hipError_t launch_residual_norm(const Geom& g, const float* b, const float* q, double* partials, ChanState* st,
                                double* results, hipStream_t s);
hipError_t launch_objective(const Geom& g, const float* z, const float* X, const float* u, const float* G,
                            const float* mu, const float* dinv, double* partials, ChanState* st, double* results,
                            hipStream_t s);

// Reduction partials per band (each up to 3 doubles) any launcher needs for geometry g.
size_t max_partials_per_band(const Geom& g);

// One scene of a batch (llp_pansharpen_batch): geometry, the caller's arrays, the scene's workspace, and the
// scene's place in the batched launches of its kernel class.
struct SceneDesc {
  Geom g;
  const float* X;  // LRMS [N][h][w]
  const float* Y;  // PAN [H][W]
  const float* u;  // kernel [n][n]
  float* x;        // HRMS [N][H][W] (the iterate)
  float *G, *MU, *DI, *b, *q, *y;
  float* r[2];
  float* p[2];
  double* partials;  // [N][pstride][3]
  int pstride;
  int band0;                  // first band of the scene in the batch's band-state array
  int dir_ntiles, apply_ntiles;
  int dir_block0, apply_block0;  // first workgroup of the scene in its class's k_dir / k_apply launch
  int data_block0;               // column sweep, c = 2: first workgroup of the scene in its class's k_data launch
  int seg_rows;                  // column sweep: rows per segment
  // The same device buffers as byte offsets from the batch workspace base: the batched kernels form their
  // pointers from the workspace base (a kernel argument, hence known to be global memory) and these offsets.
  size_t o_x, o_r[2], o_p[2], o_q, o_y, o_G, o_MU, o_DI, o_partials;
  int taps_index;                // the scene's kernel taps: taps table + taps_index * kTapStride
};
constexpr int kTapStride = 1024;  // floats per scene in the batch's kernel-tap table (n <= 31)

// Column-sweep variant of q = A p (llp_sweep.hip): q_D = B^T D^T y (k_data), then q = q_D + lambda L^T M L p
// and, in mode 1, the dot products (k_llp); apply_ntiles() partials per band.  For the classes of sweep_fused()
// the sweep forms q_D itself and there is no k_data launch.  Segments are multiples of 4 rows.
bool sweep_fused(int C, int R);
bool sweep_fits(const Geom& g, int seg_rows);
int sweep_ntiles(const Geom& g, int seg_rows);
int sweep_data_blocks(const Geom& g);
int sweep_out_width(int r);
hipError_t launch_apply_sweep(const Geom& g, int seg_rows, int mode, const float* p, const float* rres,
                              const float* y, const float* u, const float* G, const float* mu, const float* dinv,
                              float* q, double* partials, ChanState* st, hipStream_t s);
hipError_t launch_apply_sweep_batch(const SceneDesc* table, int count, int data_blocks, int llp_blocks, int C,
                                    int R, int r, int parity, ChanState* st, char* ws, const float* taps,
                                    hipStream_t s);

// k_finalize (kFinDir / kFinApply) for all `bands` bands of the `count` scenes of a table; kFinDir advances each
// active band's iteration count on the device.
hipError_t launch_finalize_batch(int op, const SceneDesc* table, int count, int bands, ChanState* st,
                                 const char* ws, int max_iters, float tol, hipStream_t s);
// Batched CG launches over the scenes [first, first+count) of a class table (all of one (c, R, r) class and one
// launch configuration): every workgroup finds its scene by binary search on the block offsets.  parity selects
// the residual/direction buffers: iteration k reads r[parity], p[parity] and writes r[1-parity], p[1-parity].
// total_blocks == 0 only prepares the kernel (its LDS limit) without launching it.
hipError_t launch_dir_fast_batch(const SceneDesc* table, int count, int total_blocks, int C, int R, int tyl,
                                 int parity, ChanState* st, char* ws, const float* taps, hipStream_t s);
hipError_t launch_apply_fast_batch(const SceneDesc* table, int count, int total_blocks, int C, int R, int r,
                                   int variant, int parity, ChanState* st, char* ws, const float* taps,
                                   hipStream_t s);

}  // namespace llp
