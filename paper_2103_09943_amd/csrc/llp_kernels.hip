// Per-scene and once-per-solve kernels of the LLP HRMS solve (Sec. III-B): input checks, PAN statistics, the
// right-hand side, the CG start, the true residual, the objective, and the finalisation of every reduction.
//
// Layout: planar float32, row-major, band-major ([N][H][W]); all convolutions and windows are periodic.
// Reductions are two-step and deterministic: every workgroup stores its partial sums (FP64, fixed order within
// the workgroup), then k_finalize -- one workgroup per band -- adds a band's partials in a fixed order and
// applies the result (to the band's CG state or to a result slot).  No atomics and no device-wide fences.
#include "llp_device.h"

#include <math.h>

namespace llp {
using namespace dev;

constexpr int kChunk = kBlock * 16;  // elements per workgroup in the flat kernels

// Periodic index: one conditional add or subtract for -n <= i < 2n (the usual case), a true modulo otherwise.
__device__ __forceinline__ int wrapc(int i, int n) {
  if (i >= -n && i < 2 * n) return i < 0 ? i + n : (i >= n ? i - n : i);
  return wrapi(i, n);
}

// ---------------------------------------------------------------------------------- input checks ---

__global__ __launch_bounds__(kBlock) void k_check_finite(const float* __restrict__ a, size_t count,
                                                         int* __restrict__ flag) {
  int bad = 0;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (size_t)gridDim.x * kBlock)
    bad |= !isfinite(a[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

hipError_t launch_check_finite(const float* a, size_t count, int* flag, hipStream_t s) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + kBlock * 8 - 1) / (kBlock * 8);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)blocks), dim3(kBlock), 0, s, a, count, flag);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------ PAN statistics (a2) ---
// G = L Y, and for every window centre k: mu_k = mean of G over w_k, var_k its population variance,
// dinv_k = 1/(eps/|w| + var_k) (0 where that vanishes).  eq. (matting_matrix) with I = L Y.

__device__ __forceinline__ double lap64(const float* __restrict__ Y, int i, int j, int H, int W) {
  const int im = i == 0 ? H - 1 : i - 1, ip = i == H - 1 ? 0 : i + 1;
  const int jm = j == 0 ? W - 1 : j - 1, jp = j == W - 1 ? 0 : j + 1;
  return 4.0 * (double)Y[(size_t)i * W + j] - (double)Y[(size_t)im * W + j] - (double)Y[(size_t)ip * W + j] -
         (double)Y[(size_t)i * W + jm] - (double)Y[(size_t)i * W + jp];
}

__global__ __launch_bounds__(kBlock) void k_pan_stats(Geom g, const float* __restrict__ Y, float* __restrict__ G,
                                                      float* __restrict__ MU, float* __restrict__ DI) {
  const size_t HW = (size_t)g.H * g.W;
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= HW) return;
  const int ki = (int)idx / g.W, kj = (int)idx - ki * g.W;  // H W < 2^31
  const int r = g.r;
  const double nw = (double)((2 * r + 1) * (2 * r + 1));
  double s1 = 0.0, s2 = 0.0;
  for (int dy = -r; dy <= r; ++dy) {
    const int i = wrapc(ki + dy, g.H);
    for (int dx = -r; dx <= r; ++dx) {
      const double v = lap64(Y, i, wrapc(kj + dx, g.W), g.H, g.W);
      s1 += v;
      s2 += v * v;
    }
  }
  const double mu = s1 / nw;
  const double var = s2 / nw - mu * mu;
  const double den = (double)g.eps / nw + var;
  const float gv = (float)lap64(Y, ki, kj, g.H, g.W), mv = (float)mu;
  const float dv = den != 0.0 ? (float)(1.0 / den) : 0.0f;
  G[idx] = gv;
  MU[idx] = mv;
  DI[idx] = dv;
}

hipError_t launch_pan_stats(const Geom& g, const float* Y, float* G, float* mu, float* dinv, hipStream_t s) {
  const size_t HW = (size_t)g.H * g.W;
  hipLaunchKernelGGL(k_pan_stats, dim3((unsigned)((HW + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, g, Y, G, mu,
                     dinv);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------- reduction finalisation ---

// The stopping rule after iterate x_k, from rr = |r_k|^2 of the recursion.
__device__ __forceinline__ void stop_rule(ChanState& c, double rr, int k_iter, int max_iters, float tol) {
  c.iters = k_iter;
  if (!isfinite(rr)) {
    c.status = -6;
    c.active = 0;
  } else if (rr == 0.0 || (tol > 0.0f && sqrt(rr) <= (double)tol * sqrt(c.bnorm2))) {
    c.active = 0;
    if (tol > 0.0f) c.pending = 1;  // stops only once the residual recomputed from the iterate agrees
    else c.status = 0;
  } else if (k_iter >= max_iters) {
    c.status = tol > 0.0f ? 1 : 0;
    c.active = 0;
  }
}

// Applies a band's summed partials s[] to its CG state.  kFinDir: rho of x_k; kFinApply: gamma, sigma, tau.
// Preconditioned iteration: kFinPcgStart and kFinPcgBeta: |r|^2, r^T s; kFinPcgAlpha: gamma; kFinPcgStop: none.
__device__ void finish_band(int op, const double (&s)[3], ChanState& c, int k_iter, int max_iters, float tol) {
  if (op == kFinDir) {  // rho_k of the iterate x_k, and the stopping rule
    c.rho = s[0];
    stop_rule(c, s[0], k_iter, max_iters, tol);
  } else if (op == kFinPcgStart) {  // r_0^T r_0, rho_0 = r_0^T P^{-1} r_0
    c.rr = s[0];
    c.rho = s[1];
    if (!isfinite(s[1]) || s[1] < 0.0) {
      c.status = -6;
      c.active = 0;
    } else {
      stop_rule(c, s[0], 0, max_iters, tol);
    }
  } else if (op == kFinPcgAlpha) {  // alpha_k = rho / p^T A p
    const double gam = s[0];
    c.gamma = gam;
    if (!(gam > 0.0) || !isfinite(gam)) {
      c.status = -6;
      c.active = 0;
    } else {
      c.alpha = c.rho / gam;
    }
  } else if (op == kFinPcgBeta) {  // |r_k|^2 and rho_k = r_k^T P^{-1} r_k -> beta_k
    if (!isfinite(s[0]) || !isfinite(s[1]) || s[1] < 0.0) {
      c.status = -6;
      c.active = 0;
    } else {
      c.beta = c.rho > 0.0 ? s[1] / c.rho : 0.0;
      c.rho = s[1];
      c.rr = s[0];
    }
  } else if (op == kFinPcgStop) {  // end of iteration k: the stopping rule on |r_k|
    stop_rule(c, c.rr, k_iter, max_iters, tol);
  } else if (op == kFinApply) {  // gamma = p^T A p, sigma = r^T A p, tau = |A p|^2 -> alpha, beta
    const double gam = s[0], sig = s[1], tau = s[2];
    c.gamma = gam;
    if (!(gam > 0.0) || !isfinite(gam) || !isfinite(sig) || !isfinite(tau)) {
      c.status = -6;
      c.active = 0;
    } else {
      const double al = c.rho / gam;
      double rt = c.rho - 2.0 * al * sig + al * al * tau;
      if (rt < 0.0) rt = 0.0;
      c.alpha = al;
      c.beta = rt / c.rho;
    }
  }
}

// Doubles per workgroup partial of each finalisation.
__device__ __forceinline__ int fin_values(int op) {
  return (op == kFinApply || op == kFinPcgStart || op == kFinPcgAlpha || op == kFinPcgBeta) ? 3 : 1;
}

// Sum, in a fixed order, of nblk partials of K doubles each (result in thread 0).
__device__ __forceinline__ void sum_partials(const double* __restrict__ base, int nblk, int K, double (&s)[3],
                                             double* red) {
  s[0] = s[1] = s[2] = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kBlock)
    for (int k = 0; k < K; ++k) s[k] += base[(size_t)i * K + k];
  block_sums<3>(s, red);
}

// One workgroup per band: adds the band's nblk partials (K doubles each) in a fixed order and applies them.
__global__ __launch_bounds__(kBlock) void k_finalize(int op, const double* __restrict__ partials, int pstride,
                                                     int nblk, ChanState* __restrict__ st,
                                                     double* __restrict__ results, int slot, int k_iter,
                                                     int max_iters, float tol) {
  __shared__ double red[3 * kWaves];
  const int ch = blockIdx.x;
  if (op != kFinBnorm && op != kFinResult && !st[ch].active) return;
  double s[3];
  sum_partials(partials + (size_t)ch * pstride * 3, nblk, fin_values(op), s, red);
  if (threadIdx.x != 0) return;
  ChanState& c = st[ch];
  if (op == kFinBnorm) c.bnorm2 = s[0];
  else if (op == kFinResult) results[ch * kResultSlots + slot] = s[0];
  else finish_band(op, s, c, k_iter < 0 ? c.iters + 1 : k_iter, max_iters, tol);  // k_iter < 0: the band's next
}

// Batched finalisation (kFinDir / kFinApply) over every band of a scene table; one workgroup per band.  The
// iteration index lives on the device: kFinDir advances a band from x_{k-1} to x_k.
__global__ __launch_bounds__(kBlock) void k_finalize_batch(int op, const SceneDesc* __restrict__ t, int count,
                                                           ChanState* __restrict__ st, const char* __restrict__ ws,
                                                           int max_iters, float tol) {
  __shared__ double red[3 * kWaves];
  const int band = blockIdx.x;
  if (!st[band].active) return;
  int lo = 0, hi = count - 1;  // scene of the band: the last entry whose band0 <= band
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (t[mid].band0 <= band) lo = mid;
    else hi = mid - 1;
  }
  const SceneDesc& d = t[lo];
  const int ch = band - d.band0;
  const int nblk = (op == kFinApply || op == kFinPcgAlpha) ? d.apply_ntiles
                   : op == kFinDir                          ? d.dir_ntiles
                   : op == kFinPcgStop                      ? 0
                                                            : d.g.h;  // the preconditioner's rows
  double s[3];
  sum_partials((const double*)(ws + d.o_partials) + (size_t)ch * d.pstride * 3, nblk, fin_values(op), s, red);
  if (threadIdx.x != 0) return;
  ChanState& c = st[band];
  finish_band(op, s, c, op == kFinPcgStart ? 0 : c.iters + 1, max_iters, tol);
}

hipError_t launch_finalize_batch(int op, const SceneDesc* table, int count, int bands, ChanState* st,
                                 const char* ws, int max_iters, float tol, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_batch, dim3(bands), dim3(kBlock), 0, s, op, table, count, st, ws, max_iters, tol);
  return hipGetLastError();
}

hipError_t launch_finalize(const Geom& g, int op, const double* partials, int nblk, ChanState* st,
                           double* results, int slot, int k_iter, int max_iters, float tol, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(g.N), dim3(kBlock), 0, s, op, partials, (int)max_partials_per_band(g), nblk,
                     st, results, slot, k_iter, max_iters, tol);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------ RHS (a3) ---
// b = B^T D^T X: the low-resolution sample X[m][k] sits at (c m, c k); B^T correlates with u, so
// b[i][j] = sum over taps (a, b') with (i + a - R) = c m and (j + b' - R) = c k of u[a][b'] X[m][k].

// b = B^T D^T X and the partial sums of |b|^2.  One workgroup per 32 x 128 block of HR pixels; the LR region of X
// its taps reach is staged in LDS once.  Per pixel the taps run in the same order as in a direct loop.
constexpr int kRhsTH = 32, kRhsTW = 128;

__host__ __device__ __forceinline__ int rhs_lr_count(int t, int R, int c) {  // LR rows (columns) t rows reach
  return (t - 1 + 2 * R) / c + 2;
}

__global__ __launch_bounds__(kBlock) void k_rhs(Geom g, const float* __restrict__ X, const float* __restrict__ u,
                                                float* __restrict__ b, double* __restrict__ partials,
                                                int pstride) {
  extern __shared__ float rhs_sh[];
  __shared__ double red[kWaves];
  const int ch = blockIdx.y;
  const int c = g.c, n = g.n, R = g.R;
  const size_t HW = (size_t)g.H * g.W;
  const float* Xc = X + (size_t)ch * g.h * g.w;
  float* bc = b + (size_t)ch * HW;
  const int tiles_x = (g.W + kRhsTW - 1) / kRhsTW;
  const int i0 = (int)(blockIdx.x / tiles_x) * kRhsTH, j0 = (int)(blockIdx.x % tiles_x) * kRhsTW;
  // LR rows floor((i0 - R) / c) ..; LR columns likewise
  const int mlo = floor_div(i0 - R, c), klo = floor_div(j0 - R, c);
  const int LH = rhs_lr_count(kRhsTH, R, c), LW = rhs_lr_count(kRhsTW, R, c);
  for (int idx = threadIdx.x; idx < LH * LW; idx += kBlock) {
    const int li = idx / LW, lj = idx - li * LW;
    rhs_sh[idx] = Xc[(size_t)wrapc(mlo + li, g.h) * g.w + wrapc(klo + lj, g.w)];
  }
  __syncthreads();
  double acc = 0.0;
  for (int p = threadIdx.x; p < kRhsTH * kRhsTW; p += kBlock) {
    const int pi = p / kRhsTW, pj = p - pi * kRhsTW;
    const int i = i0 + pi, j = j0 + pj;
    if (i >= g.H || j >= g.W) continue;
    const int a0 = wrapi(R - i, c), b0 = wrapi(R - j, c);
    // i + a - R and j + b - R are multiples of c on the taps visited: the LR indices step by one per tap
    const int m0 = (i + a0 - R) / c - mlo, k0 = (j + b0 - R) / c - klo;
    double v = 0.0;
    for (int a = a0, m = m0; a < n; a += c, ++m) {
      const float* xrow = rhs_sh + m * LW;
      for (int bb = b0, k = k0; bb < n; bb += c, ++k) v += (double)u[a * n + bb] * (double)xrow[k];
    }
    const float vf = (float)v;
    bc[(size_t)i * g.W + j] = vf;
    acc += (double)vf * (double)vf;
  }
  double v[1] = {acc};
  block_partials<1>(v, red, partials + (size_t)ch * pstride * 3 + blockIdx.x);
}

hipError_t launch_rhs(const Geom& g, const float* X, const float* u, float* b, double* partials, ChanState* st,
                      hipStream_t s) {
  // blocks of 32 x 128 pixels: no more than the operator's 16 x 64 tiles, so within the partials per band
  const int nblk = ((g.H + kRhsTH - 1) / kRhsTH) * ((g.W + kRhsTW - 1) / kRhsTW);
  const int pstride = (int)max_partials_per_band(g);
  const size_t lds = (size_t)rhs_lr_count(kRhsTH, g.R, g.c) * rhs_lr_count(kRhsTW, g.R, g.c) * sizeof(float);
  hipLaunchKernelGGL(k_rhs, dim3(nblk, g.N), dim3(kBlock), lds, s, g, X, u, b, partials, pstride);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(g, kFinBnorm, partials, nblk, st, nullptr, 0, 0, 0, 0.0f, s);
}

// ------------------------------------------------------------------------------ CG start (a4, a7) ---
// Resets the band states (first workgroup of each band) and, for a start from Z = 0, sets r_0 = b.  A start
// from a given Z0 gets r_0 = b - A Z0 from the FP64 residual pass instead.  rho_0 is summed by the first k_dir
// launch.
__global__ __launch_bounds__(kBlock) void k_init(Geom g, int from_init, const float* __restrict__ b,
                                                 float* __restrict__ r, ChanState* __restrict__ st) {
  const int ch = blockIdx.y;
  const size_t HW = (size_t)g.H * g.W;
  const size_t base = (size_t)ch * HW;
  const size_t e0 = (size_t)blockIdx.x * kChunk;
  const size_t e1 = e0 + kChunk < HW ? e0 + kChunk : HW;
  if (!from_init)
    for (size_t e = e0 + threadIdx.x; e < e1; e += kBlock) r[base + e] = b[base + e];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ChanState& s = st[ch];
    s.rho = 0.0;
    s.alpha = 0.0;
    s.beta = 0.0;
    s.gamma = 0.0;
    s.iters = 0;
    s.active = 1;
    s.status = 0;
    s.init = from_init ? kInitUser : kInitZero;
    s.pending = 0;
    s.last_rep = 0;
    s.ref_iter = -1;
  }
}

hipError_t launch_init(const Geom& g, int from_init, const float* b, float* r, ChanState* st, hipStream_t s) {
  const size_t HW = (size_t)g.H * g.W;
  const int nblk = (int)((HW + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_init, dim3(nblk, g.N), dim3(kBlock), 0, s, g, from_init, b, r, st);
  return hipGetLastError();
}

// Check of a network start z0 (xacc = z0, r = b - A z0, results[kSlotTrueRes] = ||r||^2): a band whose start is
// no better than Z = 0 (||r||^2 >= ||b||^2) restarts from Z = 0.  Records the band's start in its state.
__global__ __launch_bounds__(kBlock) void k_fallback(Geom g, const double* __restrict__ results,
                                                     ChanState* __restrict__ st, const float* __restrict__ b,
                                                     float* __restrict__ r, double* __restrict__ x) {
  const int ch = blockIdx.y;
  const bool reject = !(results[ch * kResultSlots + kSlotTrueRes] < st[ch].bnorm2);
  const size_t HW = (size_t)g.H * g.W;
  const size_t base = (size_t)ch * HW;
  const size_t e0 = (size_t)blockIdx.x * kChunk;
  const size_t e1 = e0 + kChunk < HW ? e0 + kChunk : HW;
  if (reject) {
    for (size_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
      x[base + e] = 0.0;
      r[base + e] = b[base + e];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st[ch].init = reject ? kInitNetRejected : kInitNet;
    if (reject) st[ch].ref_iter = -1;  // the residual in the results is the rejected start's
  }
}

hipError_t launch_fallback(const Geom& g, const double* results, ChanState* st, const float* b, float* r,
                           double* x, hipStream_t s) {
  const size_t HW = (size_t)g.H * g.W;
  const int nblk = (int)((HW + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_fallback, dim3(nblk, g.N), dim3(kBlock), 0, s, g, results, st, b, r, x);
  return hipGetLastError();
}

// ||b - q||^2 per band (q = A Z): the true residual of the returned iterate.
__global__ __launch_bounds__(kBlock) void k_residual_norm(Geom g, const float* __restrict__ b,
                                                          const float* __restrict__ q, double* __restrict__ partials,
                                                          int pstride) {
  __shared__ double red[kWaves];
  const int ch = blockIdx.y;
  const size_t HW = (size_t)g.H * g.W;
  const size_t base = (size_t)ch * HW;
  double acc = 0.0;
  const size_t e0 = (size_t)blockIdx.x * kChunk;
  const size_t e1 = e0 + kChunk < HW ? e0 + kChunk : HW;
  for (size_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
    const double d = (double)b[base + e] - (double)q[base + e];
    acc += d * d;
  }
  double v[1] = {acc};
  block_partials<1>(v, red, partials + (size_t)ch * pstride * 3 + blockIdx.x);
}

hipError_t launch_residual_norm(const Geom& g, const float* b, const float* q, double* partials, ChanState* st,
                                double* results, hipStream_t s) {
  const size_t HW = (size_t)g.H * g.W;
  const int nblk = (int)((HW + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_residual_norm, dim3(nblk, g.N), dim3(kBlock), 0, s, g, b, q, partials,
                     (int)max_partials_per_band(g));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(g, kFinResult, partials, nblk, st, results, kSlotTrueRes, 0, 0, 0.0f, s);
}

// ----------------------------------------------------------------------------------- objective (a8) ---
// 1/2 ||D B z - X||^2 (on the low-resolution lattice) + lambda/2 sum_k min_{a,c} [sum_{i in w_k}
// (l_i - a G_i - c)^2 + eps a^2] with l = L z (eq. pansharp with the per-window optimum; equal to
// (L z)^T M_LY (L z) of eq. initialize_z_fast).  Every term is a sum of squares accumulated in FP64.

// Data part of the objective: sum over LR cells of (D B z - X)^2.  One workgroup per block of LR cells covering
// about 32 x 128 HR pixels (32/c x 128/c cells); the z region the block's taps reach is staged in LDS once.
__global__ __launch_bounds__(kBlock) void k_obj_data(Geom g, const float* __restrict__ z, const float* __restrict__ X,
                                                     const float* __restrict__ u, double* __restrict__ partials,
                                                     int pstride) {
  extern __shared__ float objd_sh[];
  __shared__ double red[kWaves];
  const int ch = blockIdx.y;
  const int c = g.c, n = g.n, R = g.R;
  const int TM = 32 / c, TK = 128 / c;
  const int RH = c * TM + n - 1, RW = c * TK + n - 1;
  const int tiles_x = (g.w + TK - 1) / TK;
  const int m0 = (int)(blockIdx.x / tiles_x) * TM, k0 = (int)(blockIdx.x % tiles_x) * TK;
  const float* zc = z + (size_t)ch * g.H * g.W;
  // region rows c m0 - R .. c (m0 + TM - 1) + R, columns likewise
  const int r0 = c * m0 - R, q0 = c * k0 - R;
  for (int idx = threadIdx.x; idx < RH * RW; idx += kBlock) {
    const int li = idx / RW, lj = idx - li * RW;
    objd_sh[idx] = zc[(size_t)wrapc(r0 + li, g.H) * g.W + wrapc(q0 + lj, g.W)];
  }
  __syncthreads();
  double acc = 0.0;
  for (int p = threadIdx.x; p < TM * TK; p += kBlock) {
    const int pm = p / TK, pk = p - pm * TK;
    const int m = m0 + pm, k = k0 + pk;
    if (m >= g.h || k >= g.w) continue;
    double v = 0.0;
    for (int a = 0; a < n; ++a) {
      const float* zrow = objd_sh + (c * pm + 2 * R - a) * RW + c * pk + 2 * R;  // row c m + R - a, column c k + R
      for (int b = 0; b < n; ++b) v += (double)u[a * n + b] * (double)zrow[-b];
    }
    const double d = v - (double)X[(size_t)ch * g.h * g.w + (size_t)m * g.w + k];
    acc += d * d;
  }
  double v[1] = {acc};
  block_partials<1>(v, red, partials + (size_t)ch * pstride * 3 + blockIdx.x);
}

__device__ __forceinline__ double lapz(const float* __restrict__ z, int i, int j, int H, int W) {
  const int im = i == 0 ? H - 1 : i - 1, ip = i == H - 1 ? 0 : i + 1;
  const int jm = j == 0 ? W - 1 : j - 1, jp = j == W - 1 ? 0 : j + 1;
  return 4.0 * (double)z[(size_t)i * W + j] - (double)z[(size_t)im * W + j] - (double)z[(size_t)ip * W + j] -
         (double)z[(size_t)i * W + jm] - (double)z[(size_t)i * W + jp];
}

// LLP part of the objective per window k (Levin's form): sum over the window of (l_i - a_k G_i - c_k)^2 plus
// eps a_k^2, with l = L z and (a_k, c_k) the window's least-squares coefficients.  One workgroup per tile of
// kObjTH x kObjTW windows: l (FP64) and G over the tile and its r-halo are staged in LDS once.
constexpr int kObjTH = 32, kObjTW = 64;

__global__ __launch_bounds__(kBlock) void k_obj_llp(Geom g, const float* __restrict__ z, const float* __restrict__ G,
                                                    const float* __restrict__ MU, const float* __restrict__ DI,
                                                    double* __restrict__ partials, int pstride) {
  extern __shared__ double obj_sh[];
  __shared__ double red[kWaves];
  const int ch = blockIdx.y;
  const int H = g.H, W = g.W, r = g.r;
  const size_t HW = (size_t)H * W;
  const float* zc = z + (size_t)ch * HW;
  const int EH = kObjTH + 2 * r, EW = kObjTW + 2 * r;
  double* Ls = obj_sh;
  float* Gs = (float*)(obj_sh + EH * EW);
  const int tiles_x = (W + kObjTW - 1) / kObjTW;
  const int i0 = (int)(blockIdx.x / tiles_x) * kObjTH, j0 = (int)(blockIdx.x % tiles_x) * kObjTW;
  for (int idx = threadIdx.x; idx < EH * EW; idx += kBlock) {
    const int li = idx / EW, lj = idx - li * EW;
    const int i = wrapc(i0 - r + li, H), j = wrapc(j0 - r + lj, W);
    Ls[idx] = lapz(zc, i, j, H, W);
    Gs[idx] = G[(size_t)i * W + j];
  }
  __syncthreads();
  const double nw = (double)((2 * r + 1) * (2 * r + 1));
  double acc = 0.0;
  for (int p = threadIdx.x; p < kObjTH * kObjTW; p += kBlock) {
    const int pi = p / kObjTW, pj = p - pi * kObjTW;
    const int ki = i0 + pi, kj = j0 + pj;
    if (ki >= H || kj >= W) continue;
    double sl = 0.0, sgl = 0.0;
    for (int dy = -r; dy <= r; ++dy) {
      const int rowo = (pi + r + dy) * EW + pj + r;
      for (int dx = -r; dx <= r; ++dx) {
        const double l = Ls[rowo + dx];
        sl += l;
        sgl += (double)Gs[rowo + dx] * l;
      }
    }
    const size_t e = (size_t)ki * W + kj;
    const double mu = MU[e], di = DI[e];
    const double m1 = sl / nw, m2 = sgl / nw;
    const double a = (m2 - mu * m1) * di;
    const double cc = m1 - a * mu;
    double pen = (double)g.eps * a * a;
    for (int dy = -r; dy <= r; ++dy) {
      const int rowo = (pi + r + dy) * EW + pj + r;
      for (int dx = -r; dx <= r; ++dx) {
        const double res = Ls[rowo + dx] - a * (double)Gs[rowo + dx] - cc;
        pen += res * res;
      }
    }
    acc += pen;
  }
  double v[1] = {acc};
  block_partials<1>(v, red, partials + (size_t)ch * pstride * 3 + blockIdx.x);
}

hipError_t launch_objective(const Geom& g, const float* z, const float* X, const float* u, const float* G,
                            const float* mu, const float* dinv, double* partials, ChanState* st, double* results,
                            hipStream_t s) {
  const int pstride = (int)max_partials_per_band(g);
  // blocks of about 32 x 128 HR pixels: no more than the operator's 16 x 64 tiles, so within the partials
  const int TM = 32 / g.c, TK = 128 / g.c;
  const int nb1 = ((g.h + TM - 1) / TM) * ((g.w + TK - 1) / TK);
  const size_t lds1 = (size_t)(g.c * TM + g.n - 1) * (g.c * TK + g.n - 1) * sizeof(float);
  hipLaunchKernelGGL(k_obj_data, dim3(nb1, g.N), dim3(kBlock), lds1, s, g, z, X, u, partials, pstride);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_finalize(g, kFinResult, partials, nb1, st, results, kSlotObjData, 0, 0, 0.0f, s);
  if (e != hipSuccess) return e;
  // tiles of 32 x 64 windows: no more than the operator's 16 x 64 tiles, so within the partials per band
  const int nb2 = ((g.H + kObjTH - 1) / kObjTH) * ((g.W + kObjTW - 1) / kObjTW);
  const size_t lds = (size_t)(kObjTH + 2 * g.r) * (kObjTW + 2 * g.r) * (sizeof(double) + sizeof(float));
  hipLaunchKernelGGL(k_obj_llp, dim3(nb2, g.N), dim3(kBlock), lds, s, g, z, G, mu, dinv, partials, pstride);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(g, kFinResult, partials, nb2, st, results, kSlotObjLlp, 0, 0, 0.0f, s);
}

}  // namespace llp
