// Autotuner of the launch configuration of the two CG iteration kernels (tile shapes of k_apply, rows per tile
// of k_dir, specialised or generic kernels), per geometry class: (c, R, r) and the image area in half-octaves.
// Every candidate runs a few CG iterations of the caller's scene under HIP-event timing; the fastest is kept in
// the context and used by later solves of that class.  Batched solves have their own entries: there every
// launch carries the workgroups of many scenes, so a shape that leaves a lone small scene's launch short of
// workgroups can still be the fastest, and the batched tuner times candidates on a batch of copies of the
// scene.  The table can be saved to and loaded from a small JSON file tagged with the device architecture.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <string>
#include <vector>

#include "llp_ctx.h"

using namespace llp;
using namespace llp::host;

namespace llp {
namespace host {

int area_bucket(const Geom& g) { return (int)floor(2.0 * log2((double)g.H * (double)g.W)); }

}  // namespace host
}  // namespace llp

namespace {

constexpr int kRuns = 3;            // timed runs per candidate
constexpr double kMargin = 0.97;    // a candidate replaces the default only if at least 3% faster

// Every launch configuration that fits the library's kernels and the LDS: the specialised kernels' shapes when
// (c, R, r) has them, otherwise the generic kernels' shapes.
std::vector<OpConfig> candidates(const Geom& g, bool allow_fast) {
  std::vector<OpConfig> out;
  if (allow_fast && fast_path_available(g.c, g.R, g.r)) {
    for (int v : {kSweepVariant, 1, 0})
      for (int rows : {4, 8}) {
        const int f = fast_apply_lds_floats(g.c, g.R, g.r, v);
        if (!(f > 0 && f <= kMaxLdsFloats && fast_path_fits(g, rows, v))) continue;
        if (v == kSweepVariant) {
          for (int seg : {32, 64, 128, 256})
            if (seg >= kMinSegRows) out.push_back(OpConfig{1, rows, v, seg});
        } else {
          out.push_back(OpConfig{1, rows, v, 2 * kMinSegRows});
        }
      }
    if (!out.empty()) return out;
  }
  for (int rows : {8, 4}) {
    if (dir_lds_floats(g.c, rows, g.R, nullptr) > kMaxLdsFloats) continue;
    for (int v = 0; v < kApplyVariants; ++v) {
      int TH = 0, TW = 0;
      if (apply_tile(g.c, v, &TH, &TW) != 0) continue;
      if (apply_lds_floats(g.c, TH, TW, g.R, g.r, nullptr, nullptr, nullptr, nullptr) > kMaxLdsFloats) continue;
      out.push_back(OpConfig{0, rows, v, 2 * kMinSegRows});
    }
  }
  return out;
}

bool same(const OpConfig& a, const OpConfig& b) {
  return a.fast == b.fast && a.dir_rows == b.dir_rows && a.apply_variant == b.apply_variant &&
         (a.apply_variant != kSweepVariant || a.seg_rows == b.seg_rows);
}

// Microseconds per CG iteration of the scene with configuration cfg (the fastest of kRuns timed runs after
// one untimed run).
llp_status time_config(llp_ctx* ctx, const Geom& g, const OpConfig& cfg, const llp_params* params,
                       const float* lrms, const float* pan, const float* kernel, float* scratch, int iters,
                       hipStream_t s, double* us) {
  llp_params p = *params;
  p.max_iters = iters;
  p.tol = 0.0f;
  p.init_mode = 0;
  double best = 0.0;
  for (int run = 0; run <= kRuns; ++run) {
    ctx->times = llp_kernel_times{0.0, 0, 0.0, 0};
    const llp_status st = solve_scene(ctx, g, cfg, &p, lrms, pan, kernel, nullptr, scratch, nullptr, s);
    if (st < 0 && st != LLP_E_BREAKDOWN && st != LLP_E_NONFINITE) return st;
    const long long n = ctx->times.apply_launches;
    const double us = n > 0 ? (ctx->times.apply_ms + ctx->times.dir_ms) * 1e3 / (double)n : 0.0;
    if (run > 0 && (best == 0.0 || us < best)) best = us;
  }
  *us = best;
  return LLP_OK;
}

// Keeps e in the context's table, replacing the entry of the same class and mode.
void keep_entry(llp_ctx* ctx, const TuneEntry& e) {
  for (TuneEntry& t : ctx->tuned)
    if (t.c == e.c && t.R == e.R && t.r == e.r && t.bucket == e.bucket && t.batched == e.batched) {
      t = e;
      return;
    }
  ctx->tuned.push_back(e);
}

// Wall-clock seconds of one batched solve (the call is synchronous) of `copies` copies of a scene with the
// launch configuration forced to cfg.
llp_status time_batch(llp_ctx* ctx, const OpConfig& cfg, const llp_shape* shape, const llp_params* params,
                      int max_iters, const float* lrms, const float* pan, const float* kernel, float* out,
                      int copies, hipStream_t s, double* secs) {
  llp_params p = *params;
  p.max_iters = max_iters;
  p.tol = 0.0f;
  p.init_mode = 0;
  const size_t nhw = (size_t)shape->N * shape->c * shape->h * shape->c * shape->w;
  std::vector<llp_shape> shapes(copies, *shape);
  std::vector<const float*> L(copies, lrms), P(copies, pan), K(copies, kernel);
  std::vector<float*> O(copies);
  for (int i = 0; i < copies; ++i) O[i] = out + (size_t)i * nhw;
  const int saved[3] = {ctx->want_dir_rows, ctx->want_apply_variant, ctx->want_seg_rows};
  ctx->want_dir_rows = cfg.dir_rows;
  ctx->want_apply_variant = cfg.apply_variant;
  ctx->want_seg_rows = cfg.seg_rows;
  HIP_TRY(hipStreamSynchronize(s));
  const auto t0 = std::chrono::steady_clock::now();
  llp_status v = llp_pansharpen_batch(ctx, copies, shapes.data(), &p, L.data(), P.data(), K.data(), nullptr,
                                      O.data(), nullptr, 0, s);
  const auto t1 = std::chrono::steady_clock::now();
  ctx->want_dir_rows = saved[0];
  ctx->want_apply_variant = saved[1];
  ctx->want_seg_rows = saved[2];
  if (v == LLP_E_BREAKDOWN || v == LLP_E_NONFINITE || v > 0) v = LLP_OK;
  *secs = std::chrono::duration<double>(t1 - t0).count();
  return v;
}

std::string device_arch(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

// Value of "key": <number> inside [b, e) of a JSON text, or false.
bool json_number(const std::string& t, size_t b, size_t e, const char* key, double* out) {
  const std::string k = std::string("\"") + key + "\"";
  const size_t at = t.find(k, b);
  if (at == std::string::npos || at >= e) return false;
  size_t c = t.find(':', at + k.size());
  if (c == std::string::npos || c >= e) return false;
  const char* s = t.c_str() + c + 1;
  char* end = nullptr;
  const double v = strtod(s, &end);
  if (end == s) return false;
  *out = v;
  return true;
}

}  // namespace

extern "C" {

llp_status llp_autotune(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* lrms,
                        const float* pan, const float* kernel, float* scratch, int iters, llp_tune_result* out,
                        hipStream_t stream) {
  if (!ctx || !params || !lrms || !pan || !kernel || iters < 1 || iters > 1000) return LLP_E_ARG;
  if (scratch && !aligned16(scratch)) return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, params, &g);
  if (v != LLP_OK) return v;
  HIP_TRY(hipSetDevice(ctx->device));
  const std::vector<OpConfig> cands = candidates(g, ctx->allow_fast);
  if (cands.empty()) return LLP_E_UNSUPPORTED;
  OpConfig def;
  if (!pick_config(g, &def, ctx->allow_fast)) return LLP_E_UNSUPPORTED;
  float* own = nullptr;
  if (!scratch) {
    if (hipMalloc((void**)&own, sizeof(float) * (size_t)g.N * g.H * g.W) != hipSuccess) return LLP_E_OOM;
    scratch = own;
  }
  // Timing uses the context's event machinery; its accumulated kernel times are kept aside meanwhile.
  const bool prof = ctx->profiling;
  const llp_kernel_times saved = ctx->times;
  ctx->profiling = true;
  double best_us = 0.0, def_us = 0.0;
  bool have_best = false;
  OpConfig best = cands[0];
  for (const OpConfig& c : cands) {
    double us = 0.0;
    v = time_config(ctx, g, c, params, lrms, pan, kernel, scratch, iters, stream, &us);
    if (v != LLP_OK) break;
    if (!(us > 0.0)) continue;  // no valid measurement for this candidate
    if (same(c, def)) def_us = us;
    if (!have_best || us < best_us) {
      have_best = true;
      best_us = us;
      best = c;
    }
  }
  if (v == LLP_OK && !have_best) {  // nothing measured: the default, no table entry
    best = def;
    best_us = 0.0;
  }
  if (v == LLP_OK && def_us > 0.0 && !(best_us < kMargin * def_us)) {  // measured gain within noise: default
    best = def;
    best_us = def_us;
  }
  ctx->profiling = prof;
  ctx->times = saved;
  if (own) {
    (void)hipStreamSynchronize(stream);
    (void)hipFree(own);
  }
  if (v != LLP_OK) return v;
  if (have_best) keep_entry(ctx, TuneEntry{g.c, g.R, g.r, area_bucket(g), best, best_us, 0});
  if (out) {
    out->fast = best.fast;
    out->dir_rows = best.dir_rows;
    out->apply_variant = best.apply_variant;
    out->seg_rows = best.seg_rows;
    out->us_per_iter = best_us;
    out->default_us_per_iter = def_us;
    out->candidates = (int)cands.size();
  }
  return LLP_OK;
}

llp_status llp_autotune_batch(llp_ctx* ctx, const llp_shape* shape, const llp_params* params, const float* lrms,
                              const float* pan, const float* kernel, int copies, int iters, llp_tune_result* out,
                              hipStream_t stream) {
  if (!ctx || !params || !lrms || !pan || !kernel || iters < 1 || iters > 1000 || copies < 0 || copies > 256)
    return LLP_E_ARG;
  Geom g;
  llp_status v = validate(shape, params, &g);
  if (v != LLP_OK) return v;
  if (!ctx->allow_fast || !fast_path_available(g.c, g.R, g.r)) return LLP_E_UNSUPPORTED;  // never batched
  HIP_TRY(hipSetDevice(ctx->device));
  std::vector<OpConfig> cands;
  for (const OpConfig& c : candidates(g, true))
    if (c.fast) cands.push_back(c);
  OpConfig def;
  if (cands.empty() || !pick_config(g, &def, true)) return LLP_E_UNSUPPORTED;
  // Reference of the batched choice: one shape for every class where it fits (the sweep, 4-row update tiles,
  // 64-row segments for r = 1), so that scenes of different sizes share launches unless a class gains at least
  // the margin from another shape.
  if (def.fast && sweep_fits(g, 2 * kMinSegRows) && fast_path_fits(g, 4, kSweepVariant)) {
    def.dir_rows = 4;
    def.apply_variant = kSweepVariant;
    if (g.r == 1) def.seg_rows = 2 * kMinSegRows;
  }
  const size_t nhw = (size_t)g.N * g.H * g.W;
  if (copies == 0) {  // about 32 M pixel-bands in the batch
    const size_t want = ((size_t)32 << 20) / nhw;
    copies = (int)(want < 2 ? 2 : (want > 64 ? 64 : want));
  }
  float* outbuf = nullptr;
  if (hipMalloc((void**)&outbuf, sizeof(float) * nhw * copies) != hipSuccess) return LLP_E_OOM;
  // Batched solves run their iterations in graph-captured chunks of 8: whole chunks only.
  iters = (iters + 7) / 8 * 8;
  // Per candidate and iteration count (iters, 2 iters): one untimed solve (graph capture, workspace), then the
  // fastest of kRuns solves; the difference of the two is the time of iters iterations without the set-up work.
  double best_us = 0.0, def_us = 0.0;
  bool have_best = false;
  OpConfig best = cands[0];
  for (const OpConfig& c : cands) {
    double t[2] = {0.0, 0.0};
    for (int j = 0; j < 2 && v == LLP_OK; ++j) {
      const int it = (j + 1) * iters;
      double secs = 0.0;
      v = time_batch(ctx, c, shape, params, it, lrms, pan, kernel, outbuf, copies, stream, &secs);
      for (int run = 0; run < kRuns && v == LLP_OK; ++run) {
        v = time_batch(ctx, c, shape, params, it, lrms, pan, kernel, outbuf, copies, stream, &secs);
        if (run == 0 || secs < t[j]) t[j] = secs;
      }
    }
    if (v != LLP_OK) break;
    const double t1 = t[0], t2 = t[1];
    if (!(t2 > t1)) continue;  // noise swamped the difference: no valid measurement for this candidate
    const double us = (t2 - t1) * 1e6 / (double)iters / (double)copies;
    if (same(c, def)) def_us = us;
    if (!have_best || us < best_us) {
      have_best = true;
      best_us = us;
      best = c;
    }
  }
  (void)hipFree(outbuf);
  if (v != LLP_OK) return v;
  if (!have_best) {  // nothing measured: keep the table as it is
    if (out) {
      *out = llp_tune_result{def.fast, def.dir_rows, def.apply_variant, def.seg_rows, 0.0, 0.0, (int)cands.size()};
    }
    return LLP_NOT_CONVERGED;
  }
  if (def_us > 0.0 && !(best_us < kMargin * def_us)) {
    best = def;
    best_us = def_us;
  }
  keep_entry(ctx, TuneEntry{g.c, g.R, g.r, area_bucket(g), best, best_us, 1});
  if (out) {
    out->fast = best.fast;
    out->dir_rows = best.dir_rows;
    out->apply_variant = best.apply_variant;
    out->seg_rows = best.seg_rows;
    out->us_per_iter = best_us;
    out->default_us_per_iter = def_us;
    out->candidates = (int)cands.size();
  }
  return LLP_OK;
}

llp_status llp_tune_clear(llp_ctx* ctx) {
  if (!ctx) return LLP_E_ARG;
  ctx->tuned.clear();
  return LLP_OK;
}

int llp_tune_count(llp_ctx* ctx) { return ctx ? (int)ctx->tuned.size() : 0; }

llp_status llp_tune_save(llp_ctx* ctx, const char* path) {
  if (!ctx || !path) return LLP_E_ARG;
  FILE* f = fopen(path, "w");
  if (!f) return LLP_E_ARG;
  fprintf(f, "{\n  \"arch\": \"%s\",\n  \"entries\": [", device_arch(ctx->device).c_str());
  for (size_t i = 0; i < ctx->tuned.size(); ++i) {
    const TuneEntry& t = ctx->tuned[i];
    fprintf(f,
            "%s\n    {\"c\": %d, \"R\": %d, \"r\": %d, \"bucket\": %d, \"batched\": %d, \"fast\": %d, "
            "\"dir_rows\": %d, \"apply_variant\": %d, \"seg_rows\": %d, \"us_per_iter\": %.2f}",
            i ? "," : "", t.c, t.R, t.r, t.bucket, t.batched, t.cfg.fast, t.cfg.dir_rows, t.cfg.apply_variant,
            t.cfg.seg_rows, t.us_per_iter);
  }
  fprintf(f, "\n  ]\n}\n");
  return fclose(f) == 0 ? LLP_OK : LLP_E_ARG;
}

llp_status llp_tune_load(llp_ctx* ctx, const char* path) {
  if (!ctx || !path) return LLP_E_ARG;
  FILE* f = fopen(path, "r");
  if (!f) return LLP_E_ARG;
  std::string t;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof(buf), f)) > 0) t.append(buf, n);
  fclose(f);
  // "arch": "<name>" must name this device's architecture.
  const size_t a = t.find("\"arch\"");
  if (a == std::string::npos) return LLP_E_ARG;
  const size_t q0 = t.find('"', t.find(':', a) + 1);
  const size_t q1 = q0 == std::string::npos ? q0 : t.find('"', q0 + 1);
  if (q1 == std::string::npos) return LLP_E_ARG;
  if (t.substr(q0 + 1, q1 - q0 - 1) != device_arch(ctx->device)) return LLP_E_UNSUPPORTED;
  std::vector<TuneEntry> entries;
  size_t pos = t.find("\"entries\"");
  if (pos == std::string::npos) return LLP_E_ARG;
  while (true) {
    const size_t b = t.find('{', pos);
    if (b == std::string::npos) break;
    const size_t e = t.find('}', b);
    if (e == std::string::npos) return LLP_E_ARG;
    double c, R, r, bucket, fast, rows, var, us = 0.0;
    if (!json_number(t, b, e, "c", &c) || !json_number(t, b, e, "R", &R) || !json_number(t, b, e, "r", &r) ||
        !json_number(t, b, e, "bucket", &bucket) || !json_number(t, b, e, "fast", &fast) ||
        !json_number(t, b, e, "dir_rows", &rows) || !json_number(t, b, e, "apply_variant", &var))
      return LLP_E_ARG;
    json_number(t, b, e, "us_per_iter", &us);
    double seg = 2 * kMinSegRows, batched = 0.0;
    json_number(t, b, e, "seg_rows", &seg);
    json_number(t, b, e, "batched", &batched);
    const OpConfig cfg{(int)fast, (int)rows, (int)var, (int)seg};
    if ((cfg.fast != 0 && cfg.fast != 1) || (cfg.dir_rows != 4 && cfg.dir_rows != 8) || cfg.apply_variant < 0 ||
        cfg.apply_variant >= kApplyVariants || cfg.seg_rows < kMinSegRows || cfg.seg_rows > 4096 ||
        (batched != 0.0 && batched != 1.0))
      return LLP_E_ARG;
    entries.push_back(TuneEntry{(int)c, (int)R, (int)r, (int)bucket, cfg, us, (int)batched});
    pos = e + 1;
  }
  for (const TuneEntry& e : entries) keep_entry(ctx, e);
  return LLP_OK;
}

}  // extern "C"
