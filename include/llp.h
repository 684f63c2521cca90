/*
 * llp.h -- C ABI of libllp, the MI355X (gfx950) solver for the per-band HRMS reconstruction under the local
 * Laplacian prior (LLP) of "Fast and High-Quality Blind Multi-Spectral Image Pansharpening" (Sec. III-B).
 *
 * For every band i of a scene the library computes Z_i, the minimiser of eq. (initialize_z_fast)
 *     1/2 || D B(u) Z_i - X_i ||^2 + lambda/2 (L Z_i)^T M_LY (L Z_i),
 * i.e. the solution of eq. (Z_ini_matting)
 *     (B^T D^T D B + lambda L^T M_LY L) Z_i = B^T D^T X_i,
 * by conjugate gradients, as the paper prescribes for that equation.
 *
 * Notation (Sec. II-A): X is the LRMS image (N bands, h x w each), Y the PAN image (H x W), Z the HRMS image
 * (N bands, H x W), u the n x n blur kernel, c = H/h = W/w.  B(u) is circular convolution (the true
 * convolution, with the kernel's centre tap u[(n-1)/2][(n-1)/2] at offset 0), D keeps pixels (c*m, c*k),
 * L is periodic convolution with the 5-point stencil S of eq. (reg2), and M_LY is the matting matrix of
 * eq. (matting_matrix) built from the Laplacian of the PAN image, with periodic (2r+1) x (2r+1) windows,
 * population variances and eps/|w| + sigma_k^2 in its denominator (a window with eps/|w| + sigma_k^2 == 0
 * contributes no slope term).
 *
 * Memory: every image argument is a DEVICE pointer to C-contiguous float32 data, planar and row-major:
 * LRMS [N][h][w], PAN [H][W], kernel [n][n], HRMS [N][H][W]; HRMS-sized buffers (hrms, init, z, Az) must be
 * 16-byte aligned (LLP_E_ARG otherwise).  The caller owns all of them; the library
 * neither frees nor retains them after a call returns.  The context owns its workspaces (grown on demand,
 * released by llp_destroy).  A context is not thread-safe: calls on one context must not overlap.
 *
 * Streams: all device work of a call is enqueued on `stream` (0 = the null stream).  llp_pansharpen and
 * llp_objective synchronise that stream before returning; the other operator entry points are asynchronous.
 *
 * Errors: every entry point returns an llp_status; no exception crosses the ABI.  Negative values are errors
 * (the output buffers are then unspecified), positive values are warnings with valid outputs.
 */
#ifndef LLP_H
#define LLP_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LLP_OK = 0,
  LLP_NOT_CONVERGED = 1,  /* tolerance not reached within max_iters; output is the last iterate */
  LLP_E_ARG = -1,         /* NULL pointer or parameter out of range */
  LLP_E_SHAPE = -2,       /* inconsistent sizes (n even, n > min(H, W), 2r+1 > min(H, W), ...) */
  LLP_E_UNSUPPORTED = -3, /* valid but beyond the library's limits (see LLP_MAX_*) */
  LLP_E_HIP = -4,         /* a HIP runtime call failed */
  LLP_E_OOM = -5,         /* workspace allocation failed */
  LLP_E_BREAKDOWN = -6,   /* p^T A p <= 0 or not finite in some band: A is not positive definite */
  LLP_E_NONFINITE = -7    /* an input (LRMS, PAN or kernel) holds NaN or Inf */
} llp_status;

/* Build limits. */
#define LLP_MAX_KERNEL 33 /* n <= 33 */
#define LLP_MAX_RADIUS 4  /* r <= 4 */
#define LLP_MAX_SCALE 4   /* c <= 4 */

typedef struct {
  int N; /* bands, >= 1 */
  int h; /* LRMS rows, >= 1 */
  int w; /* LRMS columns, >= 1 */
  int c; /* resolution gap: H = c*h, W = c*w; the paper has c >= 2, c = 1 is accepted */
  int n; /* blur kernel size, odd, n <= min(H, W) */
} llp_shape;

typedef struct {
  int r;         /* LLP window radius (eq. reg2), 0 <= r, 2r+1 <= min(H, W) */
  float lambda;  /* LLP weight, >= 0 */
  float eps;     /* matting regulariser epsilon, >= 0 (enters as eps/|w| + sigma^2) */
  int max_iters; /* CG iteration cap, >= 0 */
  float tol;     /* > 0: stop a band when ||b - A Z|| <= tol * ||b|| (b = B^T D^T X_i) for its iterate Z: when the
                    CG residual r_k meets the bound, r_k is recomputed as b - A Z in FP64 from Z (carried as FP64
                    plus a float32 part) and the band stops only if that meets it too, else it iterates on from
                    the recomputed residual; the same replacement runs every 64 iterations.  The returned HRMS is
                    float(Z).  <= 0: run exactly max_iters iterations (with the same replacements) */
  int init_mode; /* 0: start from Z = 0; 1: start from the caller's `init`; 2: start from the warm-start
                    network's estimate (llp_cnn_set_weights first), band by band only where it is closer
                    than Z = 0 (||b - A Z0|| < ||b||), else from Z = 0 */
  int precond;   /* 0: plain conjugate gradients; 1: preconditioned by P = B^T D^T D B + lambda mbar L^T L,
                    mbar the mean of diag(M_LY), applied exactly in the Fourier domain (not in the paper; the
                    same minimiser, fewer iterations).  Needs r >= 1, lambda > 0, h and w with prime factors in
                    {2, 3, 5, 7}, c W, c H <= 16384 and, at c <= 2, W, H <= 7776 (c = 2) or 9898 (c = 1)
                    (LLP_E_UNSUPPORTED otherwise; a workgroup holds c^2 transforms and their twiddles in LDS),
                    and a kernel with nonzero sum (LLP_E_BREAKDOWN otherwise) */
} llp_params;

typedef struct {
  int iters;                /* CG iterations run for this band */
  int status;               /* llp_status of this band (LLP_OK, LLP_NOT_CONVERGED, LLP_E_BREAKDOWN) */
  double rel_residual;      /* ||r_k|| / ||b|| of the CG residual at exit (the last replaced one, see below) */
  double true_rel_residual; /* ||b - A Z|| / ||b|| of the solver's iterate Z, evaluated in FP64 (the quantity the
                               tolerance is checked on) */
  double objective;         /* eq. (initialize_z_fast) at the returned float32 HRMS */
  int init;                 /* how the band started: 0 Z = 0, 1 the caller's init, 2 the network's estimate,
                               3 the network's estimate was rejected (no better than Z = 0) and Z = 0 used */
  double out_rel_residual;  /* ||b - A Z32|| / ||b|| of the returned float32 HRMS Z32 = float(Z), in FP64: at
                               least the residual that rounding Z to float32 causes */
} llp_report;

typedef struct llp_ctx llp_ctx;

/* Create a context bound to HIP device `device`.  *out receives the handle.  If the environment variable
 * LLP_FORCE_GENERIC is set (and not "0") at creation, the context uses only the generic kernels (no
 * specialisation on kernel size, scale and window radius); results agree to rounding.  LLP_DIR_ROWS (4, 8),
 * LLP_APPLY_VARIANT (0: 32x64 tiles, 1: 16x64 tiles, 2: column sweep) and LLP_SEG_ROWS
 * (rows per sweep segment, >= 32, rounded down to a multiple of 4) force a launch configuration of the
 * specialised kernels instead of the tuned or default one. */
llp_status llp_create(llp_ctx** out, int device);

/* Release a context and all its workspaces.  NULL is accepted. */
void llp_destroy(llp_ctx* ctx);

/* Static description of a status code. */
const char* llp_status_str(int status);

/* Host-only check of a problem description against the rules above and the library's limits (no device
 * work, no context needed).  `params` may be NULL to check the shape alone.  Returns LLP_OK or the error that
 * llp_pansharpen would return for these arguments. */
llp_status llp_validate(const llp_shape* shape, const llp_params* params);

/* Solve eq. (Z_ini_matting) for all N bands of one scene (Sec. III-B; Algorithm "Fast Pansharpening": the
 * matting matrix is formed once from the PAN image, then every band is solved).
 *   lrms  [N][h][w] device, pan [H][W] device, kernel [n][n] device,
 *   init  [N][H][W] device or NULL (read only when params->init_mode == 1),
 *   hrms  [N][H][W] device, written,
 *   rep   host array of N reports, or NULL.
 * Returns the worst band status (errors before warnings).  Inputs are checked for NaN/Inf (LLP_E_NONFINITE). */
llp_status llp_pansharpen(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* lrms,
                          const float* pan, const float* kernel, const float* init, float* hrms,
                          llp_report* rep, hipStream_t stream);

/* ---- Batched solve ---------------------------------------------------------------------------------------- */

/* Flags of llp_pansharpen_batch. */
#define LLP_BATCH_NO_GRAPH 1 /* enqueue the batched iteration kernels directly instead of replaying a graph */
#define LLP_BATCH_SERIAL 2   /* solve the scenes one after another with llp_pansharpen (for comparison) */
#define LLP_BATCH_AUTOTUNE 4 /* first tune every class without a tuned entry: llp_autotune_batch on one of its
                                scenes (llp_autotune if S == 1 or the class has no specialised kernels) */

/* Solve eq. (Z_ini_matting) for every band of S scenes of any sizes at once.  The paper solves the bands of a
 * scene independently (the parallel loop over bands of Algorithm "Fast Pansharpening", Sec. III-B); here all
 * bands of all scenes advance together: each CG iteration is one launch of the operator kernel and one of
 * the update kernel per class of scenes that share (c, n, r) and a tile shape, plus two launches that finish
 * the per-band reductions, and a band that meets its stopping rule stops while the others go on.  Chunks of
 * iterations are captured once in a HIP graph and replayed (cached in the context while the classes and the
 * workspace stay the same).  Scenes whose (c, n, r) has no specialised kernels (llp_validate accepts them)
 * are solved after the batch with llp_pansharpen.
 *   S        number of scenes, >= 0 (0: nothing to do, LLP_OK)
 *   shapes   host array [S]; params: ONE llp_params for all scenes (host)
 *   lrms, pan, kernel, hrms   host arrays [S] of device pointers, laid out as for llp_pansharpen
 *   init     host array [S] of device pointers, read when params->init_mode == 1 (may be NULL otherwise)
 *   rep      host array of sum(shapes[i].N) reports in scene order, band order within a scene, or NULL
 *   flags    0 or LLP_BATCH_* bits
 * Device work runs on a stream owned by the context that first waits for the work already enqueued on
 * `stream`; the call returns after all of it has finished.  Returns the worst status over all bands
 * (errors before warnings); LLP_E_NONFINITE if any scene's inputs hold NaN or Inf (the other scenes' outputs
 * and reports are still valid).  Argument errors are detected before any device work. */
llp_status llp_pansharpen_batch(llp_ctx* ctx, int S, const llp_shape* shapes, const llp_params* params,
                                const float* const* lrms, const float* const* pan, const float* const* kernel,
                                const float* const* init, float* const* hrms, llp_report* rep, int flags,
                                hipStream_t stream);

/* ---- Autotuner ------------------------------------------------------------------------------------------- */

typedef struct {
  int fast;                   /* 1: kernels specialised on (c, n, r); 0: generic kernels */
  int dir_rows;               /* LR rows per tile of the update kernel (4 or 8) */
  int apply_variant;          /* operator kernel: 0 32x64 tiles, 1 16x64 tiles, 2 column sweep */
  int seg_rows;               /* rows per sweep segment (apply_variant 2) */
  double us_per_iter;         /* measured time of one CG iteration (both kernels, all bands) with that choice */
  double default_us_per_iter; /* the same for the untuned default choice */
  int candidates;             /* configurations timed */
} llp_tune_result;
/* (For llp_autotune_batch the times are per CG iteration of one scene of the batch.) */

/* Time every launch configuration the build has for this geometry (iters CG iterations of the given scene per
 * candidate, HIP events around the kernels, the fastest of three runs after an untimed one) and keep the
 * fastest (the default unless another is at least 3% faster) for the geometry's class: (c, n, r) and the
 * image area H*W in half-octaves.  Later single-scene solves of that class on this context use it, and so do
 * batched ones unless the class has a batched entry (llp_autotune_batch); LLP_DIR_ROWS / LLP_APPLY_VARIANT /
 * LLP_SEG_ROWS override both.  Inputs as for
 * llp_pansharpen; scratch: device [N][H][W] float32 written during tuning, or NULL (allocated and freed by the
 * call);
 * 1 <= iters <= 1000; out: host, or NULL.  Synchronises `stream`. */
llp_status llp_autotune(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* lrms,
                        const float* pan, const float* kernel, float* scratch, int iters, llp_tune_result* out,
                        hipStream_t stream);

/* The same for batched solves (llp_pansharpen_batch with S >= 2): there each launch carries the workgroups of
 * many scenes, which favours other shapes than a lone scene does.  Every specialised configuration is timed on
 * a batch of `copies` copies of the given scene (0: enough copies for about 32 M pixel-bands, 2..64), as the
 * difference of the wall time of batched solves of 2 iters and of iters iterations (the fastest of three each,
 * after an untimed solve), and the fastest is kept as the class's batched entry, unless it is less than 3%
 * faster than the common batched shape (column sweep, 4-row update tiles, 64-row segments at r = 1), which
 * keeps scenes of different sizes in shared launches.  LLP_E_UNSUPPORTED if no specialised kernel fits the
 * geometry (no specialised kernels for (c, n, r), or an image narrower or lower than their tiles): such scenes
 * are never batched.  0 <= copies <= 256; 1 <= iters <= 1000, rounded up to a multiple of 8 (batched solves
 * iterate in chunks of 8).  A candidate whose two timings do not differ by a positive amount (timing noise) is
 * skipped; if no candidate gives a valid time, nothing is stored and the call returns the warning
 * LLP_NOT_CONVERGED.  Allocates and frees copies * N*H*W floats of output scratch.  Synchronises `stream`. */
llp_status llp_autotune_batch(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* lrms,
                              const float* pan, const float* kernel, int copies, int iters, llp_tune_result* out,
                              hipStream_t stream);

/* The tuned table: save it as JSON tagged with the device architecture (e.g. "gfx950"), merge a saved table
 * into the context (LLP_E_UNSUPPORTED if it was made for another architecture, LLP_E_ARG if unreadable),
 * clear it, count its entries. */
llp_status llp_tune_save(llp_ctx* ctx, const char* path);
llp_status llp_tune_load(llp_ctx* ctx, const char* path);
llp_status llp_tune_clear(llp_ctx* ctx);
int llp_tune_count(llp_ctx* ctx);

/* ---- Warm-start network -------------------------------------------------------------------------------- */
/* Not in the paper, which leaves the initial guess of the CG solve open (Sec. III-B).  For band i:
 *     z0 = x_up + s * net([(x_up - m)/s, (Y - m_Y)/s_Y])
 * x_up the periodic bicubic upsampling of X_i (Keys, a = -1/2; HR pixel c*m on LR pixel m), m and s the mean
 * and population std of X_i (s = 1 if 0), m_Y and s_Y those of Y; net: five 3x3 convolutions
 * (2 -> 32 -> 32 -> 32 -> 32 -> 1 channels, cross-correlation, periodic padding), ReLU after the first four.
 * Layer inputs and weights are rounded to bfloat16, products accumulate in FP32 (matrix cores); biases FP32.
 * Parameters: LLP_CNN_PARAMS floats, per layer W [cout][cin][3][3] then b [cout]. */
#define LLP_CNN_PARAMS 28641

/* Load the network's parameters (host FP32 array of `count` == LLP_CNN_PARAMS) into the context; resets the
 * optimiser state.  LLP_E_NONFINITE if any parameter is NaN or Inf.  Synchronises the device. */
llp_status llp_cnn_set_weights(llp_ctx* ctx, const float* params, int count);
/* Copy the current (possibly trained) parameters to a host array.  Synchronises the device. */
llp_status llp_cnn_get_weights(llp_ctx* ctx, float* params, int count);
/* The network's estimate for every band of a scene: z0 [N][H][W] device (may be NULL), and the raw network
 * output [N][H][W] device (may be NULL; not both NULL).  Asynchronous on `stream`. */
llp_status llp_cnn_warm_start(llp_ctx* ctx, const llp_shape* shape, const float* lrms, const float* pan,
                              float* z0, float* net_out, hipStream_t stream);
/* Training loss of one scene against the plain solver's HRMS `target` [N][H][W] (device): the mean over all
 * pixels of all bands of (net - t)^2, t = (target - x_up)/s, into *loss (host, may be NULL), and its gradient
 * with respect to every parameter into `grads` (host array of LLP_CNN_PARAMS, may be NULL).  In the backward
 * pass each layer's output gradient is rounded to bfloat16 before its products.  Synchronises `stream`. */
llp_status llp_cnn_loss_grad(llp_ctx* ctx, const llp_shape* shape, const float* lrms, const float* pan,
                             const float* target, double* loss, float* grads, hipStream_t stream);
/* One training step on one scene: the gradient above, then an Adam update (beta1 0.9, beta2 0.999, eps 1e-8,
 * step size lr > 0) of the FP32 parameters.  *loss (host, may be NULL) receives the loss before the update;
 * with loss == NULL the call is asynchronous on `stream`. */
llp_status llp_cnn_train_step(llp_ctx* ctx, const llp_shape* shape, const float* lrms, const float* pan,
                              const float* target, float lr, double* loss, hipStream_t stream);

/* ---- Operator entry points (the steps of the solve, exposed for parity checks) ------------------------ */

/* PAN statistics that define M_LY (eq. matting_matrix with I = L Y): G = L Y [H][W], and per window centre
 * mu [H][W] (window mean of G) and dinv [H][W] = 1/(eps/|w| + sigma^2) (0 where that is 0).
 * Accumulation in FP64, results rounded once to float32.  All pointers device. */
llp_status llp_pan_stats(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* pan,
                         float* G, float* mu, float* dinv, hipStream_t stream);

/* Right-hand side of eq. (Z_ini_matting): b = B^T D^T X_i for every band.  b [N][H][W] device. */
llp_status llp_rhs(llp_ctx* ctx, const llp_shape* shape, const float* lrms, const float* kernel, float* b,
                   hipStream_t stream);

/* Apply the matrix of eq. (Z_ini_matting): Az = (B^T D^T D B + lambda L^T M_LY L) z for every band.
 * z, Az [N][H][W] device (must not alias). */
llp_status llp_apply_A(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* pan,
                       const float* kernel, const float* z, float* Az, hipStream_t stream);

/* The two terms of that matrix separately, with the solve's own kernels and launch configuration:
 *   llp_apply_data: out = B^T D^T D B z, the data term of eq. (Z_ini_matting) (Sec. II-A: B circular
 *                   convolution by the kernel, D decimation by c).  params selects the launch configuration only
 *                   (its r; lambda and eps are not used); no PAN image is needed.
 *   llp_apply_llp:  out = lambda L^T M_LY L z, the LLP term of eq. (Z_ini_matting) with M_LY of
 *                   eq. (matting_matrix); the kernel is read (the operator kernel is shared with the data term)
 *                   but contributes nothing.
 * z, out [N][H][W] device, 16-byte aligned, must not alias.  Asynchronous on `stream`. */
llp_status llp_apply_data(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* kernel,
                          const float* z, float* out, hipStream_t stream);
llp_status llp_apply_llp(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* pan,
                         const float* kernel, const float* z, float* out, hipStream_t stream);

/* The Fourier-domain passes on their own (the transforms of the preconditioned solve, precond = 1):
 *   llp_precond_apply:      out = P^{-1} r, P = B^T D^T D B + lambda mbar L^T L with mbar the mean of diag(M_LY)
 *                           (eq. matting_matrix); not in the paper: the preconditioner of the solve of
 *                           eq. (Z_ini_matting).
 *   llp_apply_data_fourier: out = B^T D^T D B z, the data term of eq. (Z_ini_matting), applied in the Fourier
 *                           domain (Sec. II-A: B circular, so DFT(B z) = DFT(u) DFT(z); D aliases the c^2
 *                           frequencies (k1 + s h, k2 + t w) onto one); params selects nothing but is validated.
 * Both need the sizes that precond = 1 needs (llp_params) (LLP_E_UNSUPPORTED otherwise);
 * llp_precond_apply also r >= 1 and lambda > 0.  r, z, out [N][H][W] device, must not alias.  Asynchronous. */
llp_status llp_precond_apply(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* pan,
                             const float* kernel, const float* r, float* out, hipStream_t stream);
llp_status llp_apply_data_fourier(llp_ctx* ctx, const llp_shape* shape, const llp_params* params,
                                  const float* kernel, const float* z, float* out, hipStream_t stream);

/* The last two steps of Algorithm "Fast Pansharpening" (Sec. III-B) on a given Z0 (normally llp_pansharpen's
 * output): the A, C step of eq. (ac_h_compute) (guided filtering of L Z0 with L Y as the guide, slope denominator
 * sigma^2 + eps/|w|) and the Z step of eq. (Z_solution), solved exactly in the Fourier domain (per aliasing group)
 * with the LLP weight lambda |w|: eq. (pansharp) counts every pixel in |w| = (2r+1)^2 windows, and with this weight
 * the two steps are one round of exact alternating minimisation of eq. (pansharp), whose minimiser (the solution
 * of eq. Z_ini_matting) is a fixed point.  Computed as z = z0 + P1^{-1} (b - A z0), P1 = B^T D^T D B +
 * lambda |w| L^T L (the same values; A, C are not stored).  Needs the sizes that precond = 1 needs (llp_params)
 * (LLP_E_UNSUPPORTED otherwise); lrms [N][h][w], pan [H][W], kernel [n][n], z0, z [N][H][W] device, z0 and z
 * 16-byte aligned, must not alias.  Asynchronous on `stream`. */
llp_status llp_polish(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* lrms,
                      const float* pan, const float* kernel, const float* z0, float* z, hipStream_t stream);

/* The product of llp_apply_A for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): no context, no allocation.  The PAN statistics and
 * y = D B z live in a library-owned device array of LLP_NOALLOC_SCRATCH_FLOATS floats per device (64 MiB), held
 * until the process ends: 3 H W + N h w must fit (LLP_E_UNSUPPORTED otherwise).  Every call on a device shares
 * that device's array, so calls that overlap on one device (on different streams or threads) race.  The untuned
 * default launch configuration is used (the same kernels as a fresh context's llp_apply_A).  Runs on the current
 * device; asynchronous on `stream`.  z, Az [N][H][W] device, 16-byte aligned, must not alias. */
#define LLP_NOALLOC_SCRATCH_FLOATS (16u << 20)
llp_status llp_apply_A_noalloc(const llp_shape* shape, const llp_params* params, const float* pan,
                               const float* kernel, const float* z, float* Az, hipStream_t stream);

/* Objective of eq. (initialize_z_fast) for every band of z: obj host [N] (FP64).  The LLP part is summed
 * window by window in the form of eq. (pansharp) with the optimal (a, c) of each window. */
llp_status llp_objective(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* lrms,
                         const float* pan, const float* kernel, const float* z, double* obj,
                         hipStream_t stream);

/* ---- Filter priors of the cross-channel prior comparison ---------------------------------------------- */

/* The priors Sec. IV compares with LLP (Table "cross_channel_prior"): the window penalty of eq. (reg2) on F Z
 * and F Y for other filters F in place of the Laplacian.  LLP: the 5-point Laplacian of eq. (reg2); LGC: the
 * horizontal and vertical gradients of eq. (reg2_lgc), two filters (forward differences; the orientation does
 * not change the operator); LPP: the identity (the pixels); LPF: the blur kernel u; HPF: delta - u.  Each
 * filter d contributes lambda F_d^T M_{F_d Y} F_d, M the matting matrix of eq. (matting_matrix) with the guide
 * F_d Y, so every band solves (B^T D^T D B + lambda sum_d F_d^T M_{F_d Y} F_d) Z = B^T D^T X. */
typedef enum { LLP_PRIOR_LLP = 0, LLP_PRIOR_LGC = 1, LLP_PRIOR_LPP = 2, LLP_PRIOR_LPF = 3, LLP_PRIOR_HPF = 4 } llp_prior;

/* out = lambda sum_d F_d^T M_{F_d Y} F_d z (+ B^T D^T D B z if data_term != 0) for every band of z.
 * pan [H][W], kernel [n][n], z, out [N][H][W] device, 16-byte aligned, must not alias.  The filter side (n for
 * LPF and HPF) must be <= 31 and the operator's tile must fit in LDS with it (LLP_E_UNSUPPORTED otherwise:
 * n <= 17 at r = 2).  Asynchronous on `stream`. */
llp_status llp_apply_prior(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, int prior,
                           const float* pan, const float* kernel, const float* z, float* out, int data_term,
                           hipStream_t stream);

/* llp_pansharpen with the prior `prior`: plain conjugate gradients (precond must be 0; init_mode 0 or 1, else
 * LLP_E_UNSUPPORTED) on float32 vectors with FP64 dot products.  With tol > 0 a band whose CG residual meets
 * tol ||b|| has its residual recomputed as b - A Z (the float32 operator, FP64 sum); it stops if that meets the
 * tolerance too, else CG restarts from that residual.  The report's true_rel_residual (and out_rel_residual)
 * is that recomputed residual of the returned Z; objective is NaN.  Same buffers and rules as llp_pansharpen;
 * synchronizes the stream. */
llp_status llp_prior_pansharpen(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, int prior,
                                const float* lrms, const float* pan, const float* kernel, const float* init,
                                float* hrms, llp_report* rep, hipStream_t stream);

/* ---- Blur-kernel estimation ------------------------------------------------------------------------------ */

/* Parameters of Algorithm "Blur Kernel Estimation" (Sec. III-A): the kernel side n (odd, <= 29), the box sizes
 * of eq. (objective3) (u_1 the (2l+1)^2 box on the LR grid, u_2 the (c l + 1)^2 box on the HR grid; c l + 1 must
 * be odd), lam_w of eq. (objective3), the TGV weights alpha_1, alpha_2 of eq. (reg1), the penalties mu_1..mu_3
 * and the step rho of the generalized ADMM (eq. Lagrangian, eq. subproblems), the iteration cap and the
 * threshold on ||u^{t+1} - u^t|| / ||u^{t+1}||. */
typedef struct {
  int n, l;
  double lam_w, alpha1, alpha2, mu1, mu2, mu3, rho;
  int t_max;
  double th;
} llp_kernel_est_params;

typedef struct {
  int iters;     /* GADMM iterations run */
  double change; /* relative change of u at the last iteration */
} llp_kernel_est_report;

/* Estimate the blur kernel from the LRMS bands that overlap PAN (Algorithm "Blur Kernel Estimation", App. A):
 * the spectral weights omega of eq. (objective3), then the generalized ADMM on eq. (u_solve) with the TGV^2
 * prior of eq. (reg1) and the simplex constraint of eq. (simplex), from the uniform kernel, in FP64 on the GPU.
 * Readings: periodic forward differences on the kernel grid; the (u, p) step keeps the mu_3 coupling; the
 * returned kernel is z (the simplex-projected copy).  lrms [Np][h][w] (Np <= 16) and pan [c h][c w] device
 * float32; kernel [n][n] device float32 (output, unit gain, >= 0); omega_out device [Np] doubles or NULL; rep
 * host or NULL (then the call is asynchronous on `stream`, else it synchronizes it).  LLP_E_UNSUPPORTED for
 * n > 29, n > c h or c w, or an even c l + 1. */
llp_status llp_estimate_kernel(llp_ctx* ctx, const llp_kernel_est_params* prm, int Np, int h, int w, int c,
                               const float* lrms, const float* pan, float* kernel, double* omega_out,
                               llp_kernel_est_report* rep, hipStream_t stream);

/* ---- Kernel timing -------------------------------------------------------------------------------------- */

typedef struct {
  double apply_ms;          /* summed device time of the operator launches (q = A p and its dot products) */
  long long apply_launches;
  double dir_ms;            /* summed device time of the direction launches (plain: x, r, p, D B p, r^T r;
                               preconditioned: p = s + beta p, D B p) */
  long long dir_launches;
  double pc_rows_ms;        /* preconditioned: forward row transforms with the update of x and r */
  long long pc_rows_launches;
  double pc_cols_ms;        /* preconditioned: column transforms with the group solve */
  long long pc_cols_launches;
  double pc_rows_inv_ms;    /* preconditioned: inverse row transforms, s = P^{-1} r and r^T s */
  long long pc_rows_inv_launches;
  double ref_ms;            /* FP64 residual replacement passes (all launches of a pass, also passes that find
                               no band due) */
  long long ref_passes;
} llp_kernel_times;

/* Enable (1) or disable (0) timing of the CG kernels of later llp_pansharpen and llp_pansharpen_batch calls on
 * this context.  Timing brackets each launch with HIP events on the call's stream; it adds two event records
 * per launch.  A timed llp_pansharpen_batch enqueues its iteration kernels directly (no graph); each class
 * launch counts as one launch. */
llp_status llp_set_profiling(llp_ctx* ctx, int enable);

/* Accumulated kernel times since the last reset (host struct); reset != 0 clears them afterwards. */
llp_status llp_get_kernel_times(llp_ctx* ctx, llp_kernel_times* out, int reset);

#ifdef __cplusplus
}
#endif

#endif /* LLP_H */
