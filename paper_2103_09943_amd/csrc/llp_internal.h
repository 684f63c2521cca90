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
  int pending;    // 1: the recursive residual met the tolerance; the band waits for its true residual
  int last_rep;   // iteration of the band's last residual replacement
  int ref_iter;   // iteration whose FP64 residual the results hold (its part z flushed); -1: none yet
  double rr;      // preconditioned iteration: r_k^T r_k (rho holds r_k^T P^{-1} r_k)
};

// Residual replacement (llp_refine.hip): every kRepEvery iterations, and whenever a band's recursive residual
// meets the tolerance, the band's iterate is flushed into its FP64 accumulator and its residual is recomputed as
// b - A x in FP64.
constexpr int kRepEvery = 64;

enum InitKind { kInitZero = 0, kInitUser = 1, kInitNet = 2, kInitNetRejected = 3 };

// What k_finalize does with a band's summed partials.  The kFinPcg* ops are the preconditioned iteration's:
// start (rho_0 = r_0^T s_0), alpha from p^T A p, beta from the new r^T s, and the end-of-iteration stopping rule.
enum FinOp {
  kFinBnorm = 0, kFinResult = 1, kFinDir = 2, kFinApply = 3,
  kFinPcgStart = 4, kFinPcgAlpha = 5, kFinPcgBeta = 6, kFinPcgStop = 7
};

// Reduction slots in the per-band result array (doubles [N][kResultSlots]): the squared FP64 residual of the
// iterate, the two objective parts, the squared FP64 residual of the float32 output.
enum ResultSlot { kSlotTrueRes = 0, kSlotObjData = 1, kSlotObjLlp = 2, kSlotOutRes = 3, kResultSlots = 4 };

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
// Resets the band states; r_0 = b for a start from Z = 0 (a given start gets its r_0 from the FP64 residual
// pass).
hipError_t launch_init(const Geom& g, int from_init, const float* b, float* r, ChanState* st, hipStream_t s);
// mode 0: y = D B z (z = rin).  mode 1: p_0 = r_0 (rin), y = D B p_0, partials of rho_0.  mode 2: the update
// of iteration k (x, r from alpha; p from beta), y = D B p_k, partials of rho_k; final_step skips p and y.
// mode 3 (preconditioned iteration): p_k = s_k (rin) + beta p_{k-1} (pin), x += alpha p_{k-1}, y = D B p_k; no
// partials.
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
// After a network start: bands whose start is no better than zero restart from zero (see k_fallback); xacc is the
// FP64 iterate.
hipError_t launch_fallback(const Geom& g, const double* results, ChanState* st, const float* b, float* r,
                           double* xacc, hipStream_t s);
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
  size_t o_s;                    // preconditioned residual (batched preconditioned solves)
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

// ---- Residual replacement (llp_refine.hip) ----------------------------------------------------------------------
// One scene of a replacement pass: its geometry, inputs, the two parts of the iterate and the CG buffers.  The
// same table-driven launches serve single-scene solves (a table of one) and batches.
struct RefDesc {
  Geom g;
  const float* Y;     // PAN [H][W]
  const float* u;     // kernel [n][n]
  const float* b;     // right-hand sides [N][H][W]
  float* z;           // float32 part of the iterate, advanced by the CG kernels between replacements [N][H][W]
  double* xacc;       // FP64 part of the iterate [N][H][W]
  float* r[2];        // residual buffers (iteration k writes r[k & 1])
  float* p[2];        // direction buffers
  double* y64;        // D B x in FP64 [N][h][w]
  double* partials;   // [N][pstride][3]: one double per residual tile
  int pstride;
  int band0;          // first band of the scene in the band-state array
  int e_block0;       // first workgroup of the scene in the elementwise launches
  int y_block0;       // ... in the D B x launch
  int r_block0;       // ... in the residual launch
};
// Elementwise operations (k_ref_elem).
enum RefElem {
  kRefFlush = 0,      // selected bands: xacc += z, z = 0
  kRefStartZero = 1,  // all bands: xacc = 0, z = 0
  kRefStartFrom = 2,  // all bands: xacc = z, z = 0 (z holds the start)
  kRefOutput = 3,     // all bands: z = float(xacc + z)
  kRefOutputBack = 4  // all bands: z = float(xacc + z), xacc = z (to evaluate the residual of the float32 output)
};
// What k_ref_fin does with a band's summed squared residual.
enum RefFin {
  kRefStep = 0,   // replacement in the iteration: records it, verifies a pending band, may finish a band
  kRefStart = 1,  // residual of the start: into kSlotTrueRes (the network-start check reads it)
  kRefFinal = 2,  // residual of the returned iterate: into kSlotTrueRes
  kRefOut = 3     // residual of the float32 output: into kSlotOutRes
};
// Blocks of the three launch kinds per band of geometry g.
int ref_elem_blocks(const Geom& g);
int ref_y_blocks(const Geom& g);
int ref_res_blocks(const Geom& g);
// Dynamic LDS of the D B x and residual launches for geometry g (bytes); the launches take the maximum over
// their table.
size_t ref_y_lds(const Geom& g);
size_t ref_res_lds(const Geom& g);
constexpr size_t kRefMaxLds = 160 * 1024 - 256;  // dynamic LDS limit of the two tiled launches (all built sizes fit)
// Raises the dynamic-LDS limit of the tiled launches (once per device, outside any graph capture).
hipError_t ref_prepare();
// force = 0: bands selected for a replacement (pending, or active and kRepEvery iterations past the last one);
// force = 1: every band.  rpar: the residual/direction buffer the next iteration reads; write_r = 0 computes
// the norm only.  `blocks` are the totals over the table; lds the per-launch maxima.
hipError_t launch_ref_elem(int op, const RefDesc* t, int count, int blocks, const ChanState* st, int force,
                           hipStream_t s);
hipError_t launch_ref_y(const RefDesc* t, int count, int blocks, size_t lds, const ChanState* st, int force,
                        hipStream_t s);
hipError_t launch_ref_res(const RefDesc* t, int count, int blocks, size_t lds, const ChanState* st, int force,
                          int rpar, int write_r, hipStream_t s);
hipError_t launch_ref_fin(int op, const RefDesc* t, int count, int bands, ChanState* st, double* results,
                          int force, int plain_cg, int max_iters, float tol, hipStream_t s);

// ---- Fourier-domain preconditioner (llp_precond.hip) -------------------------------------------------------------
constexpr int kPcThreads = 1024;   // threads per workgroup of the row transform passes
constexpr int kPcColThreads = 512; // threads per workgroup of the column pass
constexpr int kPcSmallRowThreads = 256;  // row passes of tables whose rows hold at most kPcSmallElems values
constexpr int kPcMaxElems = 16384; // complex values a workgroup holds in LDS: c W and c H at most this
constexpr int kPcColBudget = 16384; // column pass: pairs of one column are grouped up to this many values
constexpr int kPcSmallElems = 4096; // the same where a transform needs radix 2, 3, 5 or 7
constexpr int kPcMaxRad = 16;      // radix passes per transform length
constexpr int kPcMaxLds = 160 * 1024 - 512;  // dynamic LDS of a transform pass (sequences and twiddles)
constexpr int kPcMbarBlocks = 64;  // workgroups per scene of the mbar reduction
// One scene of the preconditioner's launches.
struct PcDesc {
  Geom g;
  int npair;            // band pairs (N + 1) / 2: band 2i in the real part, band 2i + 1 in the imaginary part
  float2* spec;         // spectra [npair][h][w][c^2]
  float2* uhat;         // kernel DFT at the group members [h][w][c^2]: U[k1 + s h][k2 + t w] at s c + t
  const float2* twh;    // pass-major twiddles of the length-h transform (h values); likewise tww (length w)
  const float2* tww;
  const float2* twH;    // e^{-2 pi i m / H}, m < H (FP64 evaluated, rounded once); likewise twW
  const float2* twW;
  const float* u;       // kernel taps [n][n]
  const float* DI;      // dinv plane of the PAN statistics [H][W]
  double* mbar;         // mean of diag(M_LY), device scalar
  float* r[2];          // residual buffers (iteration k writes r[k & 1])
  float* p[2];          // direction buffers
  const float* q;       // A p of the current iteration
  float* s;             // preconditioned residual P^{-1} r [N][H][W]
  double* partials;     // [N][pstride][3]: slot 0 |r|^2, slot 1 r^T s, one per LR row
  int pstride;
  int band0;
  int row_block0;             // first workgroup of the scene in the row launches
  int col_block0;             // first LR column of the scene among the table's columns (the column pass)
  int nrw, nrh;                // radix passes of the length-w and length-h transforms
  int mixed_w, mixed_h;        // the length-w (length-h) transform needs a radix other than 8 and 4
  int rw[kPcMaxRad], rh[kPcMaxRad];
};
struct PcPlan {
  int count = 0, bands = 0, row_blocks = 0, col_blocks = 0;
  size_t row_lds = 0, col_lds = 0;
  int col_budget = 0;  // column pass: elements of one group of columns (band pairs of one LR column)
  int cus = 256;       // compute units of the device (persistent column workgroups)
  bool mixed = false;  // some transform length needs radix 2, 3, 5 or 7 (the kernels for short transforms)
  bool small_rows = false;  // every scene's c^2 w <= kPcSmallElems: row passes of kPcSmallRowThreads threads
};
enum PcRowsOp { kPcRowsStart = 0, kPcRowsUpdate = 1, kPcRowsKernel = 2 };
enum PcColsOp { kPcColsSolve = 0, kPcColsKernel = 1, kPcColsData = 2 };
// Radices of a transform length (8, 4, 2, 7, 5, 3 in that order) into rad; -1 if L has another prime factor.
int pc_radices(int L, int* rad);
// Whether geometry g can be preconditioned: c <= 4, r >= 1, lambda > 0, h and w with prime factors 2, 3, 5, 7
// only, c W, c H <= kPcMaxElems, and the c^2 padded sequences with their twiddle table within kPcMaxLds.
bool pc_supported(const Geom& g);
size_t pc_spec_floats(const Geom& g);
size_t pc_uhat_floats(const Geom& g);
size_t pc_tw_floats(const Geom& g);
void pc_twiddles(const Geom& g, float* out);  // the twiddle tables of g (host, FP64 evaluated)
void pc_fill(PcDesc& d, const Geom& g, float* tw_dev);  // geometry, radices and twiddle pointers
void pc_plan(PcDesc* h_tab, int count, PcPlan* plan);   // block offsets and launch sizes
hipError_t pc_prepare();  // dynamic-LDS limits of the transform launches (once per device)
hipError_t launch_pc_rows(int op, const PcDesc* t, const PcPlan& P, const ChanState* st, int prev, int cur,
                          hipStream_t s);
hipError_t launch_pc_cols(int op, const PcDesc* t, const PcPlan& P, const ChanState* st, hipStream_t s);
hipError_t launch_pc_rows_inv(const PcDesc* t, const PcPlan& P, const ChanState* st, int cur, hipStream_t s);
// mbar of every scene of the table (part: count * kPcMbarBlocks doubles of scratch).
// out = a + sb * b (n floats); the solve's scalar weight mbar set to v for every scene of the table.
hipError_t launch_pc_axpy(const float* a, const float* b, float* out, float sb, size_t n, hipStream_t s);
hipError_t launch_pc_set_mbar(const PcDesc* t, int count, double v, hipStream_t s);
hipError_t launch_pc_mbar(const PcDesc* t, int count, double* part, hipStream_t s);

// k_finalize (kFinDir / kFinApply) for all `bands` bands of the `count` scenes of a table; kFinDir advances each
// active band's iteration count on the device.
hipError_t launch_finalize_batch(int op, const SceneDesc* table, int count, int bands, ChanState* st,
                                 const char* ws, int max_iters, float tol, hipStream_t s);
// Batched CG launches over the scenes [first, first+count) of a class table (all of one (c, R, r) class and one
// launch configuration): every workgroup finds its scene by binary search on the block offsets.  parity selects
// the residual/direction buffers: iteration k reads r[parity], p[parity] and writes r[1-parity], p[1-parity].
// total_blocks == 0 only prepares the kernel (its LDS limit) without launching it.
hipError_t launch_dir_fast_batch(const SceneDesc* table, int count, int total_blocks, int C, int R, int tyl,
                                 int parity, ChanState* st, char* ws, const float* taps, int mode, hipStream_t s);
hipError_t launch_apply_fast_batch(const SceneDesc* table, int count, int total_blocks, int C, int R, int r,
                                   int variant, int parity, ChanState* st, char* ws, const float* taps,
                                   hipStream_t s);

}  // namespace llp
