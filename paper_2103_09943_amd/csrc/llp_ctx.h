// Host-side state of a libllp context and the helpers shared by the C-ABI sources (llp_api.hip: single-scene
// entry points; llp_batch.hip: the batched solve; llp_tune.hip: the autotuner).
#pragma once

#include <stdint.h>

#include <vector>

#include "llp.h"
#include "llp_cnn.h"
#include "llp_internal.h"

namespace llp {
namespace host {

constexpr int kCheckEvery = 8;  // CG iterations between convergence polls in tolerance mode (even)
constexpr int kMaxLdsFloats = 160 * 1024 / 4;

#define HIP_TRY(expr)                       \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return LLP_E_HIP; \
  } while (0)

// Tuned launch configuration of one geometry class: (c, R, r) and the image area in half-octaves, for solves
// of one scene (batched = 0) or for batched solves, whose launches carry the workgroups of many scenes
// (batched = 1).
struct TuneEntry {
  int c, R, r, bucket;
  OpConfig cfg;
  double us_per_iter;  // measured time of one CG iteration (operator + update kernels) of one scene
  int batched;
};
int area_bucket(const Geom& g);

size_t align_up(size_t v, size_t a);
bool aligned16(const void* p);  // image buffers are read and written with 16-byte vector accesses
llp_status validate(const llp_shape* s, const llp_params* p, Geom* g);
// Default launch configuration: the first shapes (in preference order) whose LDS fits.
bool pick_config(const Geom& g, OpConfig* cfg, bool allow_fast = true, int want_dir_rows = 0,
                 int want_apply_variant = -1);
// The configuration a context uses for g: environment overrides, else a tuned entry (for batched solves the
// batched entry of the class if there is one, then the single-scene entry), else the default.
bool ctx_config(llp_ctx* ctx, const Geom& g, OpConfig* cfg, bool batched = false);
llp_status ensure_workspace(llp_ctx* ctx, const Geom& g, bool precond = false);
// Kernel timing (llp_set_profiling): timing_begin records a start event on s and returns its pair's index (or
// -1 when not profiling or on failure), timing_end records the end event and the pair's slot.
enum TimeSlot { kTApply = 0, kTDir = 1, kTPcRows = 2, kTPcCols = 3, kTPcRowsInv = 4, kTRef = 5, kTSlots = 6 };
int timing_begin(llp_ctx* ctx, hipStream_t s);
void timing_end(llp_ctx* ctx, hipStream_t s, int pair, int slot);
llp_status collect_times(llp_ctx* ctx);
llp_status check_inputs(llp_ctx* ctx, const Geom& g, const float* lrms, const float* pan, const float* kernel,
                        hipStream_t s);
llp_status apply_A_into(llp_ctx* ctx, const Geom& g, const OpConfig& cfg, const float* z, const float* kernel,
                        float* q, hipStream_t s);
// Warm-start network state of a context (llp_cnn_set_weights).
struct CnnState {
  void* mem = nullptr;  // one allocation: master weights, Adam moments, gradient, MFMA weight operands
  float *master = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
  void* fwd[kCnnLayers] = {};  // forward operands of each layer
  void* bwd[kCnnLayers] = {};  // transposed, flipped operands (input gradients)
  int steps = 0;               // Adam steps taken
  void* ws = nullptr;          // activations and scratch, grown on demand
  size_t ws_bytes = 0;
  double* h_loss = nullptr;    // pinned
};
void cnn_free(CnnState* c);
// z0 (and the raw network output, if netout) for every band of a scene; the context must hold weights.
llp_status cnn_warm_start(llp_ctx* ctx, const Geom& g, const float* X, const float* Y, float* z0, float* netout,
                          hipStream_t s);

// Launch sizes of a residual-replacement pass over a RefDesc table (blocks and LDS over all its scenes).
struct RefPlan {
  int count = 0, bands = 0;
  int eblocks = 0, yblocks = 0, rblocks = 0;
  size_t ylds = 0, rlds = 0;
};
// Assigns the table's block offsets (e_block0, y_block0, r_block0) in order and sums the plan.
void ref_plan(RefDesc* tab, int count, RefPlan* plan);
// One replacement pass over the table: flush (except for kRefOut), D B x, residual, finalisation fin_op.
llp_status ref_pass(const RefDesc* d_tab, const RefPlan& P, ChanState* st, double* results, int fin_op, int force,
                    int rpar, int write_r, int max_iters, float tol, int plain_cg, hipStream_t s);

llp_status pc_setup(llp_ctx* ctx, const Geom& g, const float* kernel, float* sout, PcPlan* PP,
                    hipStream_t s);

// The whole single-scene solve with launch configuration cfg (the body of llp_pansharpen).
llp_status solve_scene(llp_ctx* ctx, const Geom& g, const OpConfig& cfg, const llp_params* params,
                       const float* lrms, const float* pan, const float* kernel, const float* init, float* hrms,
                       llp_report* rep, hipStream_t s);

}  // namespace host
}  // namespace llp

struct llp_ctx {
  int device = 0;
  bool allow_fast = true;  // false when LLP_FORCE_GENERIC is set at creation: generic kernels only
  int want_dir_rows = 0;   // launch-shape overrides (0: default), from LLP_DIR_ROWS / LLP_APPLY_VARIANT
  int want_apply_variant = -1;
  int want_seg_rows = 0;  // LLP_SEG_ROWS: rows per segment of the column sweep (>= kMinSegRows)
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // views into ws
  float *G = nullptr, *MU = nullptr, *DI = nullptr, *b = nullptr, *q = nullptr, *y = nullptr;
  float* r[2] = {nullptr, nullptr};  // residual, alternating between iterations
  float* p[2] = {nullptr, nullptr};  // direction, alternating between iterations
  double* partials = nullptr;
  double* xacc = nullptr;  // FP64 part of the iterate [N][H][W]
  double* y64 = nullptr;   // D B x of the FP64 residual pass [N][h][w]
  llp::RefDesc* d_ref = nullptr;  // the scene's residual-pass table (one entry)
  llp::RefDesc* h_ref = nullptr;  // pinned host copy
  // preconditioner (solves with precond = 1)
  float* s = nullptr;      // P^{-1} r [N][H][W]
  float* spec = nullptr;   // spectra of the band pairs
  float* uhat = nullptr;   // kernel DFT at the group members
  float* tw = nullptr;     // twiddle tables
  double* mbar = nullptr;  // mbar, then kPcMbarBlocks partials
  llp::PcDesc* d_pc = nullptr;
  llp::PcDesc* h_pc = nullptr;  // pinned
  float* h_tw = nullptr;        // pinned twiddle staging
  size_t h_tw_cap = 0;
  llp::ChanState* st = nullptr;
  double* results = nullptr;
  int* flags = nullptr;
  // pinned host mirrors
  llp::ChanState* h_st = nullptr;
  double* h_results = nullptr;
  int* h_flags = nullptr;
  int h_cap = 0;  // bands the mirrors hold
  hipEvent_t ev[2] = {nullptr, nullptr};
  // kernel timing (llp_set_profiling)
  bool profiling = false;
  std::vector<hipEvent_t> tev;  // timing events, in start/end pairs
  std::vector<int> tslot;       // slot of every pair
  size_t tev_used = 0;          // pairs in use
  llp_kernel_times times = {};
  // llp_pansharpen_batch: own stream, workspace, pinned mirrors and the cached graph of an iteration chunk
  hipStream_t bstream = nullptr;
  hipEvent_t bev_in = nullptr;
  void* bws = nullptr;
  size_t bws_bytes = 0;
  llp::ChanState* h_bst[2] = {nullptr, nullptr};
  double* h_bres = nullptr;
  int* h_bflags = nullptr;
  llp::SceneDesc* h_table = nullptr;
  llp::RefDesc* h_rtable = nullptr;
  llp::PcDesc* h_ptable = nullptr;  // preconditioned batches: the transform table
  int hb_bands = 0, hb_scenes = 0;  // capacities of the batch mirrors
  float* h_btw = nullptr;           // preconditioned batches: pinned twiddle staging of all scenes
  size_t h_btw_cap = 0;
  hipGraphExec_t gexec = nullptr;
  std::vector<long long> gkey;  // what the cached graph was captured for
  // launch configurations chosen by the autotuner (llp_autotune), by geometry class
  std::vector<llp::host::TuneEntry> tuned;
  llp::host::CnnState* cnn = nullptr;  // warm-start network (llp_cnn_set_weights)
  // filter priors (llp_prior_pansharpen, llp_apply_prior): guides, statistics, taps, restart flags
  void* prior_ws = nullptr;
  size_t prior_bytes = 0;
  // blur-kernel estimation (llp_estimate_kernel): omega terms, f, E^T f, correlations, E^T E and its inverse
  void* ke_ws = nullptr;
  size_t ke_bytes = 0;
};
