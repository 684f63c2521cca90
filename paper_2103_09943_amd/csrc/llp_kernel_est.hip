// Blur-kernel estimation, Algorithm "Blur Kernel Estimation" (Sec. III-A, App. A), on the GPU in FP64:
//
//   k_ke_omega_terms / k_ke_omega_solve   the spectral weights omega of eq. (objective3) from its normal
//                                          equations (box-blurred LRMS bands against the decimated box-blurred
//                                          PAN, plus the first-difference regulariser), solved on the device;
//   k_ke_f                                 f = sum_i omega_i X'_i on the LR grid;
//   k_ke_etf                               E^T f, E = D C(Y) the matrix of eq. (z_solution);
//   k_ke_corr / k_ke_ete                   E^T E from the phase-restricted correlations of PAN: entry
//                                          ((a,b),(a',b')) is sum over the pixels (i, j) of phase (-a, -b) mod c of
//                                          Y[i][j] Y[i+a-a'][j+b-b'], so c^2 (2n-1)^2 sums replace the n^2 x n^2
//                                          Gram matrix over all LR pixels;
//   k_ke_gj                                (E^T E + mu_3 I)^-1 by Gauss-Jordan elimination, one launch per pivot
//                                          (the matrix is symmetric positive definite: no pivoting);
//   k_ke_gadmm                             the generalized ADMM of eq. (subproblems) to convergence in one
//                                          persistent workgroup with every iterate in LDS: the shrinkages of
//                                          eq. (x_update) / (y_update), the z step of eq. (z_solution) (a product
//                                          with the inverse, then the projection onto the simplex of eq. (simplex)
//                                          by Michelot's exact finite method), the (u, p) step of eq.
//                                          (u_p_solution) by Cramer's rule per frequency of the n x n DFT (App. A),
//                                          the multiplier updates and the stopping rule on the relative change of u.
//
// The readings are the oracle's: periodic forward differences on the kernel grid, the mu_3 coupling in the
// (u, p) step, the mean of the two equal middle columns of E(p), the uniform start, z returned.
#include <math.h>
#include <string.h>

#include "llp_ctx.h"
#include "llp_device.h"

namespace llp {

using namespace dev;

namespace {

constexpr int kKeMaxSide = 29;           // longest kernel side the iteration's LDS holds
constexpr int kKeMaxBands = 16;          // overlapping LRMS bands
constexpr int kKeThreads = 512;          // the iteration workgroup (2 waves per SIMD: room for the FP64 Cramer temporaries)
constexpr int kKeFlat = kBlock * 16;     // LR pixels per workgroup of the flat reductions
constexpr int kKeOmegaVals = kKeMaxBands * (kKeMaxBands + 1) / 2 + kKeMaxBands;

struct KeArgs {
  int Np, h, w, c, H, W, n, l;
  double lam_w, a1m1, a2m2, mu1, mu2, mu3, rho, th;
  int t_max;
};

__device__ __forceinline__ int wrapd(int i, int m) {
  int r = i % m;
  return r < 0 ? r + m : r;
}

}  // namespace

// Per LR pixel: m_i = (box_{2l+1} * X'_i)[m][k] (circular on the LR grid) and v = (box_{cl+1} * Y)[c m][c k];
// the partial sums of m_i m_j (i <= j) and m_i v over the block.
__global__ __launch_bounds__(kBlock) void k_ke_omega_terms(KeArgs K, const float* __restrict__ X,
                                                           const float* __restrict__ Y,
                                                           double* __restrict__ partials) {
  __shared__ double acc[kKeOmegaVals];
  for (int e = threadIdx.x; e < kKeOmegaVals; e += kBlock) acc[e] = 0.0;
  __syncthreads();
  const int hw = K.h * K.w;
  const int Np = K.Np;
  const int l = K.l, sb = K.c * K.l + 1, Rb = (sb - 1) / 2;
  const double inv_lr = 1.0 / (double)((2 * l + 1) * (2 * l + 1)), inv_hr = 1.0 / (double)(sb * sb);
  double mloc[kKeMaxBands];
  double t[kKeOmegaVals];
  const int nv = Np * (Np + 1) / 2 + Np;
  for (int e = 0; e < nv; ++e) t[e] = 0.0;
  const int e0 = blockIdx.x * kKeFlat, e1 = min(e0 + kKeFlat, hw);
  for (int e = e0 + threadIdx.x; e < e1; e += kBlock) {
    const int m = e / K.w, k = e - m * K.w;
    for (int i = 0; i < Np; ++i) {
      const float* Xi = X + (size_t)i * hw;
      double s = 0.0;
      for (int a = -l; a <= l; ++a) {
        const int mm = wrapd(m - a, K.h);
        for (int b = -l; b <= l; ++b) s += (double)Xi[mm * K.w + wrapd(k - b, K.w)];
      }
      mloc[i] = s * inv_lr;
    }
    double v = 0.0;
    for (int a = -Rb; a <= Rb; ++a) {
      const size_t row = (size_t)wrapd(K.c * m - a, K.H) * K.W;
      for (int b = -Rb; b <= Rb; ++b) v += (double)Y[row + wrapd(K.c * k - b, K.W)];
    }
    v *= inv_hr;
    int o = 0;
    for (int i = 0; i < Np; ++i)
      for (int j = i; j < Np; ++j) t[o++] += mloc[i] * mloc[j];
    for (int i = 0; i < Np; ++i) t[o++] += mloc[i] * v;
  }
  // block sums in a fixed order: lane sums by wave, then waves one after another
  for (int e = 0; e < nv; ++e) {
    double s = wave_sum(t[e]);
    if ((threadIdx.x & 63) == 0) t[e] = s;
  }
  for (int wv = 0; wv < kWaves; ++wv) {
    if ((threadIdx.x >> 6) == wv && (threadIdx.x & 63) == 0)
      for (int e = 0; e < nv; ++e) acc[e] += t[e];
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nv; e += kBlock) partials[(size_t)blockIdx.x * kKeOmegaVals + e] = acc[e];
}

// Sums the partials in order and solves (M^T M + lam_w G^T G) omega = M^T v (Gaussian elimination with partial
// pivoting, one thread: Np <= 16).
__global__ void k_ke_omega_solve(KeArgs K, const double* __restrict__ partials, int nblk,
                                 double* __restrict__ omega) {
  __shared__ double S[kKeOmegaVals];
  const int Np = K.Np, nv = Np * (Np + 1) / 2 + Np;
  for (int e = threadIdx.x; e < nv; e += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partials[(size_t)b * kKeOmegaVals + e];
    S[e] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double A[kKeMaxBands][kKeMaxBands + 1];
  int o = 0;
  for (int i = 0; i < Np; ++i)
    for (int j = i; j < Np; ++j) {
      A[i][j] = S[o];
      A[j][i] = S[o];
      ++o;
    }
  for (int i = 0; i < Np; ++i) A[i][Np] = S[o++];
  // + lam_w G^T G, G the (Np-1) x Np first-difference matrix: a tridiagonal with 1, 2, ..., 2, 1 and -1
  for (int i = 0; i + 1 < Np; ++i) {
    A[i][i] += K.lam_w;
    A[i + 1][i + 1] += K.lam_w;
    A[i][i + 1] -= K.lam_w;
    A[i + 1][i] -= K.lam_w;
  }
  for (int col = 0; col < Np; ++col) {
    int piv = col;
    for (int r = col + 1; r < Np; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (piv != col)
      for (int j = 0; j <= Np; ++j) {
        const double tmp = A[col][j];
        A[col][j] = A[piv][j];
        A[piv][j] = tmp;
      }
    for (int r = col + 1; r < Np; ++r) {
      const double f = A[r][col] / A[col][col];
      for (int j = col; j <= Np; ++j) A[r][j] -= f * A[col][j];
    }
  }
  for (int i = Np - 1; i >= 0; --i) {
    double s = A[i][Np];
    for (int j = i + 1; j < Np; ++j) s -= A[i][j] * omega[j];
    omega[i] = s / A[i][i];
  }
}

// f = sum_i omega_i X'_i (LR grid, FP64).
__global__ __launch_bounds__(kBlock) void k_ke_f(KeArgs K, const float* __restrict__ X,
                                                 const double* __restrict__ omega, double* __restrict__ f) {
  const int hw = K.h * K.w;
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= hw) return;
  double s = 0.0;
  for (int i = 0; i < K.Np; ++i) s += omega[i] * (double)X[(size_t)i * hw + e];
  f[e] = s;
}

// (E^T f)[(a+R) n + (b+R)] = sum_{m,k} Y[(c m - a) mod H][(c k - b) mod W] f[m][k]: one workgroup per tap.
__global__ __launch_bounds__(kBlock) void k_ke_etf(KeArgs K, const float* __restrict__ Y,
                                                   const double* __restrict__ f, double* __restrict__ etf) {
  __shared__ double red[kWaves];
  const int tap = blockIdx.x, R = (K.n - 1) / 2;
  const int a = tap / K.n - R, b = tap % K.n - R;
  double s = 0.0;
  const int hw = K.h * K.w;
  for (int e = threadIdx.x; e < hw; e += kBlock) {
    const int m = e / K.w, k = e - m * K.w;
    s += (double)Y[(size_t)wrapd(K.c * m - a, K.H) * K.W + wrapd(K.c * k - b, K.W)] * f[e];
  }
  double v[1] = {s};
  block_sums<1>(v, red);
  if (threadIdx.x == 0) etf[tap] = v[0];
}

// S[pa][pb][da + n - 1][db + n - 1] = sum_{m,k} Y[pa + c m][pb + c k] Y[pa + c m + da][pb + c k + db] (periodic),
// for |da|, |db| <= n - 1.  One workgroup per (pa, pb, da); lane j of each wave owns the lag db = j - (n - 1); the
// four waves split the LR columns.  Per LR row the HR row pa + c m + da is staged in LDS with a periodic halo of
// n - 1 on both sides, so lane j reads position pb + c k + j: consecutive lanes, consecutive words, no wrap.
__global__ __launch_bounds__(kBlock) void k_ke_corr(KeArgs K, const float* __restrict__ Y, double* __restrict__ S) {
  extern __shared__ float ke_row[];
  __shared__ double red[kWaves][64];
  const int n = K.n, L = 2 * n - 1, W = K.W;
  const int da = (int)(blockIdx.x % L) - (n - 1);
  const int ph = blockIdx.x / L, pa = ph / K.c, pb = ph % K.c;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool live = lane < L;
  const int RW = W + 2 * (n - 1);
  float* row = ke_row;         // RW floats: row[t] = Y[pa + c m + da][(t - (n - 1)) mod W]
  float* dec = ke_row + RW;    // w floats: Y[pa + c m][pb + c k]
  double acc = 0.0;
  for (int m = 0; m < K.h; ++m) {
    const int i = pa + K.c * m;
    const float* yr = Y + (size_t)wrapd(i + da, K.H) * W;
    const float* y0 = Y + (size_t)i * W;
    __syncthreads();
    for (int t = threadIdx.x; t < RW; t += kBlock) {
      int j = t - (n - 1);
      j += j < 0 ? W : 0;
      j -= j >= W ? W : 0;
      row[t] = yr[j];
    }
    for (int k = threadIdx.x; k < K.w; k += kBlock) dec[k] = y0[pb + K.c * k];
    __syncthreads();
    if (live) {
      const float* rl = row + pb + lane;
      for (int k = wave; k < K.w; k += kWaves) acc += (double)dec[k] * (double)rl[K.c * k];
    }
  }
  red[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && live) {
    double s = 0.0;
    for (int wv = 0; wv < kWaves; ++wv) s += red[wv][lane];
    S[((size_t)ph * L + (da + n - 1)) * L + lane] = s;
  }
}

// A = E^T E + mu_3 I from the correlations: A[(a+R)n+(b+R)][(a'+R)n+(b'+R)] = S[(-a) mod c][(-b) mod c][a-a'][b-b'].
__global__ __launch_bounds__(kBlock) void k_ke_ete(KeArgs K, const double* __restrict__ S, double* __restrict__ A) {
  const int n = K.n, n2 = n * n, L = 2 * n - 1, R = (n - 1) / 2;
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= n2 * n2) return;
  const int r = e / n2, q = e - r * n2;
  const int a = r / n - R, b = r % n - R, a2 = q / n - R, b2 = q % n - R;
  const int ph = wrapd(-a, K.c) * K.c + wrapd(-b, K.c);
  double v = S[((size_t)ph * L + (a - a2 + n - 1)) * L + (b - b2 + n - 1)];
  if (r == q) v += K.mu3;
  A[e] = v;
}

// One Gauss-Jordan step on the N x N matrix A (in place, becomes its inverse after N steps).  rin/cin hold row k
// and column k of A before this step; the step writes row k+1 and column k+1 of its result to rout/cout.
__global__ __launch_bounds__(kBlock) void k_ke_gj(int N, int k, double* __restrict__ A, const double* __restrict__ rin,
                                                  const double* __restrict__ cin, double* __restrict__ rout,
                                                  double* __restrict__ cout) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= N * N) return;
  const int i = e / N, j = e - i * N;
  const double p = rin[k];
  double v;
  if (i == k && j == k) v = 1.0 / p;
  else if (i == k) v = rin[j] / p;
  else if (j == k) v = -cin[i] / p;
  else v = A[e] - cin[i] * rin[j] / p;
  A[e] = v;
  if (i == k + 1) rout[j] = v;
  if (j == k + 1) cout[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_ke_gj_init(int N, const double* __restrict__ A, double* __restrict__ r,
                                                       double* __restrict__ c) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= N) return;
  r[e] = A[e];
  c[e] = A[(size_t)e * N];
}

// ----------------------------------------------------------------------------------- the GADMM iteration ---

namespace {

struct KeLds {
  // real n x n planes (doubles)
  double *u, *z, *L3, *p0, *p1, *x0, *x1, *L10, *L11, *y0, *y1, *y3, *L20, *L21, *L23;
  // complex n x n planes (re, im interleaved)
  double *F1, *F2, *F3, *T;
  double* roots;  // n complex roots exp(-2 pi i m / n)
  double* red;    // reduction scratch
};

// Block sums of two values (red: 2 kKeThreads / 64 doubles); every thread gets both.
__device__ __forceinline__ void blk_sum2(double& a, double& b, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  __syncthreads();
  if (lane == 0) {
    red[wave] = a;
    red[kKeThreads / 64 + wave] = b;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
  for (int i = 0; i < kKeThreads / 64; ++i) {
    sa += red[i];
    sb += red[kKeThreads / 64 + i];
  }
  a = sa;
  b = sb;
}

// dst (complex n x n, rows j, columns k) = src W (along_cols: transform along the column index) or W src (along
// the row index), W the DFT matrix (forward, exp(-2 pi i jk/n)) or its conjugate (inverse).
__device__ void dft_pass(const double* F, double* T, const double* roots, int n, bool along_cols, bool inverse) {
  const int n2 = n * n;
  for (int e = threadIdx.x; e < n2; e += kKeThreads) {
    const int j = e / n, k = e - j * n;
    double sr = 0.0, si = 0.0;
    const int step = along_cols ? k : j;  // the root index advances by the output index per term
    int idx = 0;
    for (int m = 0; m < n; ++m, idx = (idx + step >= n ? idx + step - n : idx + step)) {
      const int src = along_cols ? j * n + m : m * n + k;
      const double wr = roots[2 * idx], wi = inverse ? -roots[2 * idx + 1] : roots[2 * idx + 1];
      const double fr = F[2 * src], fi = F[2 * src + 1];
      sr += fr * wr - fi * wi;
      si += fr * wi + fi * wr;
    }
    T[2 * e] = sr;
    T[2 * e + 1] = si;
  }
  __syncthreads();
}

}  // namespace

__global__ __launch_bounds__(kKeThreads) void k_ke_gadmm(KeArgs K, const double* __restrict__ Kinv,
                                                         const double* __restrict__ etf, float* __restrict__ kout,
                                                         double* __restrict__ info) {
  extern __shared__ double ke_lds[];
  const int n = K.n, n2 = n * n;
  KeLds S;
  double* q = ke_lds;
  double** reals[] = {&S.u, &S.z, &S.L3, &S.p0, &S.p1, &S.x0, &S.x1, &S.L10, &S.L11, &S.y0, &S.y1, &S.y3,
                      &S.L20, &S.L21, &S.L23};
  for (double** r : reals) {
    *r = q;
    q += n2;
  }
  S.F1 = q;
  q += 2 * n2;
  S.F2 = q;
  q += 2 * n2;
  S.F3 = q;
  q += 2 * n2;
  S.T = q;
  q += 2 * n2;
  S.roots = q;
  q += 2 * n;
  S.red = q;
  const int tid = threadIdx.x;
  const double PI = 3.14159265358979323846;
  for (int m = tid; m < n; m += kKeThreads) {
    double sn, cs;
    sincos(-2.0 * PI * (double)m / (double)n, &sn, &cs);
    S.roots[2 * m] = cs;
    S.roots[2 * m + 1] = sn;
  }
  // start: u = z = 1/n^2, p = grad u = 0, x = y = 0, multipliers 0
  const double u0 = 1.0 / (double)n2;
  for (int e = tid; e < n2; e += kKeThreads) {
    S.u[e] = u0;
    S.z[e] = u0;
    S.L3[e] = 0.0;
    S.p0[e] = S.p1[e] = 0.0;
    S.x0[e] = S.x1[e] = 0.0;
    S.L10[e] = S.L11[e] = 0.0;
    S.y0[e] = S.y1[e] = S.y3[e] = 0.0;
    S.L20[e] = S.L21[e] = S.L23[e] = 0.0;
  }
  __syncthreads();
  // periodic forward differences on the n x n grid
  auto dh = [&](const double* a, int e) { const int i = e / n, j = e - i * n; return a[i * n + (j + 1 == n ? 0 : j + 1)] - a[e]; };
  auto dv = [&](const double* a, int e) { const int i = e / n; return a[(i + 1 == n ? e - i * n : e + n)] - a[e]; };

  const double a1m1 = K.a1m1, a2m2 = K.a2m2, mu3 = K.mu3, rho = K.rho;
  const double t1 = 1.0 / K.mu1, t2 = 1.0 / K.mu2;
  int t = 0;
  double change = 0.0;
  for (t = 0; t < K.t_max; ++t) {
    // x = shrink2(grad u - p + L1, 1/mu1);  y = shrink2(E(p) + L2, 1/mu2) (the middle columns stored once)
    for (int e = tid; e < n2; e += kKeThreads) {
      const double g0 = dh(S.u, e) - S.p0[e] + S.L10[e];
      const double g1 = dv(S.u, e) - S.p1[e] + S.L11[e];
      const double nx = sqrt(g0 * g0 + g1 * g1);
      const double sx = nx > 0.0 ? fmax(nx - t1, 0.0) / nx : 0.0;
      const double e0 = dh(S.p0, e) + S.L20[e];
      const double e1 = 0.5 * (dv(S.p0, e) + dh(S.p1, e)) + S.L21[e];
      const double e3 = dv(S.p1, e) + S.L23[e];
      const double ny = sqrt(e0 * e0 + 2.0 * e1 * e1 + e3 * e3);
      const double sy = ny > 0.0 ? fmax(ny - t2, 0.0) / ny : 0.0;
      S.x0[e] = g0 * sx;
      S.x1[e] = g1 * sx;
      S.y0[e] = e0 * sy;
      S.y1[e] = e1 * sy;
      S.y3[e] = e3 * sy;
      S.F1[e] = etf[e] + mu3 * (S.u[e] + S.L3[e]);  // the z step's right-hand side (real, in F1's first n^2)
    }
    __syncthreads();
    // z = (E^T E + mu3 I)^{-1} rhs: one wave per row, lanes along the row (coalesced)
    {
      // four rows per wave step, so that each lane has four independent streams of loads in flight
      const int lane = tid & 63, wave = tid >> 6;
      constexpr int kRows = 4;
      for (int r0 = wave * kRows; r0 < n2; r0 += (kKeThreads / 64) * kRows) {
        double s[kRows];
#pragma unroll
        for (int q = 0; q < kRows; ++q) s[q] = 0.0;
        for (int j = lane; j < n2; j += 64) {
          const double rv = S.F1[j];
#pragma unroll
          for (int q = 0; q < kRows; ++q) {
            const int rr = min(r0 + q, n2 - 1);
            s[q] += Kinv[(size_t)rr * n2 + j] * rv;
          }
        }
#pragma unroll
        for (int q = 0; q < kRows; ++q) {
          const double t = wave_sum(s[q]);
          if (lane == 0 && r0 + q < n2) S.z[r0 + q] = t;
        }
      }
    }
    __syncthreads();
    // projection onto the simplex (Michelot): theta = (sum over the support - 1) / |support|, support = {z > theta},
    // repeated until the support stops shrinking
    {
      double theta = -INFINITY;
      double prev_cnt = -1.0;
      for (int it = 0; it < n2 + 1; ++it) {
        double s = 0.0, cnt = 0.0;
        for (int e = tid; e < n2; e += kKeThreads)
          if (S.z[e] > theta) {
            s += S.z[e];
            cnt += 1.0;
          }
        double ssum = s, csum = cnt;
        blk_sum2(ssum, csum, S.red);
        if (csum == prev_cnt) break;
        prev_cnt = csum;
        theta = (ssum - 1.0) / csum;
      }
      __syncthreads();
      for (int e = tid; e < n2; e += kKeThreads) S.z[e] = fmax(S.z[e] - theta, 0.0);
    }
    __syncthreads();
    // B1, B2, B3 (App. A, with the mu3 coupling; y_3 and Lambda_23 the shared middle columns) into F1..F3
    for (int e = tid; e < n2; e += kKeThreads) {
      // differences of (x - L1) and (y - L2) need neighbours: formed from the planes directly
      const int i = e / n, j = e - i * n;
      const int jm = i * n + (j == 0 ? n - 1 : j - 1), im = (i == 0 ? e + (n - 1) * n : e - n);
      const double xl0 = S.x0[e] - S.L10[e], xl0m = S.x0[jm] - S.L10[jm];
      const double xl1 = S.x1[e] - S.L11[e], xl1m = S.x1[im] - S.L11[im];
      const double yl0 = S.y0[e] - S.L20[e], yl0m = S.y0[jm] - S.L20[jm];
      const double yl1 = S.y1[e] - S.L21[e], yl1h = S.y1[jm] - S.L21[jm], yl1v = S.y1[im] - S.L21[im];
      const double yl3 = S.y3[e] - S.L23[e], yl3m = S.y3[im] - S.L23[im];
      const double b1 = a1m1 * ((xl0m - xl0) + (xl1m - xl1)) + mu3 * (S.z[e] - S.L3[e]);
      const double b2 = a1m1 * (S.L10[e] - S.x0[e]) + a2m2 * ((yl0m - yl0) + (yl1v - yl1));
      const double b3 = a1m1 * (S.L11[e] - S.x1[e]) + a2m2 * ((yl3m - yl3) + (yl1h - yl1));
      S.F1[2 * e] = b1;
      S.F1[2 * e + 1] = 0.0;
      S.F2[2 * e] = b2;
      S.F2[2 * e + 1] = 0.0;
      S.F3[2 * e] = b3;
      S.F3[2 * e + 1] = 0.0;
    }
    __syncthreads();
    // each 2-D transform goes F -> T (rows) -> F (columns)
    dft_pass(S.F1, S.T, S.roots, n, true, false);
    dft_pass(S.T, S.F1, S.roots, n, false, false);
    dft_pass(S.F2, S.T, S.roots, n, true, false);
    dft_pass(S.T, S.F2, S.roots, n, false, false);
    dft_pass(S.F3, S.T, S.roots, n, true, false);
    dft_pass(S.T, S.F3, S.roots, n, false, false);
    // Cramer's rule per frequency (k1 row, k2 column): symbols sh = e^{2 pi i k2/n} - 1, sv = e^{2 pi i k1/n} - 1
    for (int e = tid; e < n2; e += kKeThreads) {
      const int k1 = e / n, k2 = e - k1 * n;
      const double shr = S.roots[2 * k2] - 1.0, shi = -S.roots[2 * k2 + 1];
      const double svr = S.roots[2 * k1] - 1.0, svi = -S.roots[2 * k1 + 1];
      const double ah = shr * shr + shi * shi, av = svr * svr + svi * svi;
      // complex helpers
      struct cd { double r, i; };
      auto mul = [](cd a, cd b) { return cd{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; };
      auto add = [](cd a, cd b) { return cd{a.r + b.r, a.i + b.i}; };
      auto sub = [](cd a, cd b) { return cd{a.r - b.r, a.i - b.i}; };
      auto cj = [](cd a) { return cd{a.r, -a.i}; };
      const cd d1{a1m1 * (ah + av) + mu3, 0.0};
      const cd d2{a1m1 + a2m2 * ah + 0.5 * a2m2 * av, 0.0};
      const cd d3{a1m1 + 0.5 * a2m2 * ah + a2m2 * av, 0.0};
      const cd d4{-a1m1 * shr, -a1m1 * shi};
      const cd d5{-a1m1 * svr, -a1m1 * svi};
      const cd d6 = mul(cd{0.5 * a2m2 * shr, -0.5 * a2m2 * shi}, cd{svr, svi});
      cd M[3][3] = {{d1, cj(d4), cj(d5)}, {d4, d2, cj(d6)}, {d5, d6, d3}};
      const cd rhs[3] = {{S.F1[2 * e], S.F1[2 * e + 1]}, {S.F2[2 * e], S.F2[2 * e + 1]}, {S.F3[2 * e], S.F3[2 * e + 1]}};
      auto det = [&](const cd (&a)[3][3]) {
        cd s = mul(mul(a[0][0], a[1][1]), a[2][2]);
        s = add(s, mul(mul(a[0][1], a[1][2]), a[2][0]));
        s = add(s, mul(mul(a[0][2], a[1][0]), a[2][1]));
        s = sub(s, mul(mul(a[0][2], a[1][1]), a[2][0]));
        s = sub(s, mul(mul(a[0][1], a[1][0]), a[2][2]));
        s = sub(s, mul(mul(a[0][0], a[2][1]), a[1][2]));
        return s;
      };
      const cd den = det(M);
      const double dd = den.r * den.r + den.i * den.i;
      cd sol[3];
      for (int col = 0; col < 3; ++col) {
        cd Mc[3][3];
        for (int r = 0; r < 3; ++r)
          for (int cc = 0; cc < 3; ++cc) Mc[r][cc] = cc == col ? rhs[r] : M[r][cc];
        const cd nu = det(Mc);
        sol[col] = cd{(nu.r * den.r + nu.i * den.i) / dd, (nu.i * den.r - nu.r * den.i) / dd};
      }
      S.F1[2 * e] = sol[0].r;
      S.F1[2 * e + 1] = sol[0].i;
      S.F2[2 * e] = sol[1].r;
      S.F2[2 * e + 1] = sol[1].i;
      S.F3[2 * e] = sol[2].r;
      S.F3[2 * e + 1] = sol[2].i;
    }
    __syncthreads();
    dft_pass(S.F1, S.T, S.roots, n, true, true);
    dft_pass(S.T, S.F1, S.roots, n, false, true);
    dft_pass(S.F2, S.T, S.roots, n, true, true);
    dft_pass(S.T, S.F2, S.roots, n, false, true);
    dft_pass(S.F3, S.T, S.roots, n, true, true);
    dft_pass(S.T, S.F3, S.roots, n, false, true);
    // u_new (real part / n^2, kept in F1's real slots), p; the multipliers; the change of u
    const double inv = 1.0 / (double)n2;
    double dsq = 0.0, nsq = 0.0;
    for (int e = tid; e < n2; e += kKeThreads) {
      const double un = S.F1[2 * e] * inv;
      S.T[e] = un;
      S.p0[e] = S.F2[2 * e] * inv;
      S.p1[e] = S.F3[2 * e] * inv;
      const double d = S.u[e] - un;
      dsq += d * d;
      nsq += un * un;
    }
    __syncthreads();
    for (int e = tid; e < n2; e += kKeThreads) {
      const double un = S.T[e];
      S.L10[e] += rho * (dh(S.T, e) - S.p0[e] - S.x0[e]);
      S.L11[e] += rho * (dv(S.T, e) - S.p1[e] - S.x1[e]);
      S.L20[e] += rho * (dh(S.p0, e) - S.y0[e]);
      S.L21[e] += rho * (0.5 * (dv(S.p0, e) + dh(S.p1, e)) - S.y1[e]);
      S.L23[e] += rho * (dv(S.p1, e) - S.y3[e]);
      S.L3[e] += rho * (un - S.z[e]);
    }
    double dtot = dsq, ntot = nsq;
    blk_sum2(dtot, ntot, S.red);
    for (int e = tid; e < n2; e += kKeThreads) S.u[e] = S.T[e];
    __syncthreads();
    change = sqrt(dtot) / fmax(sqrt(ntot), 1e-300);
    if (change < K.th) {
      ++t;
      break;
    }
  }
  for (int e = tid; e < n2; e += kKeThreads) kout[e] = (float)S.z[e];
  if (tid == 0) {
    info[0] = (double)(t < K.t_max ? t : K.t_max);
    info[1] = change;
  }
}

namespace host {
namespace {

size_t ke_lds_bytes(int n) { return ((size_t)15 * n * n + 8 * n * n + 2 * n + 2 * kKeThreads / 64) * sizeof(double); }

}  // namespace
}  // namespace host
}  // namespace llp

using namespace llp;
using namespace llp::host;

extern "C" {

llp_status llp_estimate_kernel(llp_ctx* ctx, const llp_kernel_est_params* prm, int Np, int h, int w, int c,
                               const float* lrms, const float* pan, float* kernel, double* omega_out,
                               llp_kernel_est_report* rep, hipStream_t stream) {
  if (!ctx || !prm || !lrms || !pan || !kernel) return LLP_E_ARG;
  const int n = prm->n;
  if (Np < 1 || Np > kKeMaxBands || h < 1 || w < 1 || c < 1 || n < 1 || n % 2 == 0 || prm->l < 0 ||
      prm->t_max < 0 || !(prm->mu1 > 0) || !(prm->mu2 > 0) || !(prm->mu3 > 0) || prm->lam_w < 0)
    return LLP_E_ARG;
  const int H = c * h, W = c * w;
  if (n > kKeMaxSide || n > H || n > W || ((c * prm->l + 1) % 2) == 0 || 2 * n - 1 > 64)
    return LLP_E_UNSUPPORTED;
  if ((size_t)h * w > (size_t)1 << 30) return LLP_E_SHAPE;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = stream;
  KeArgs K;
  K.Np = Np;
  K.h = h;
  K.w = w;
  K.c = c;
  K.H = H;
  K.W = W;
  K.n = n;
  K.l = prm->l;
  K.lam_w = prm->lam_w;
  K.a1m1 = prm->alpha1 * prm->mu1;
  K.a2m2 = prm->alpha2 * prm->mu2;
  K.mu1 = prm->mu1;
  K.mu2 = prm->mu2;
  K.mu3 = prm->mu3;
  K.rho = prm->rho;
  K.th = prm->th;
  K.t_max = prm->t_max;
  const int n2 = n * n, L = 2 * n - 1;
  const size_t hw = (size_t)h * w;
  const int nblk = (int)((hw + kKeFlat - 1) / kKeFlat);
  // workspace (doubles): omega partials, omega, f, E^T f, S, A, the two Gauss-Jordan row/column buffers, info
  size_t off = 0;
  auto take = [&](size_t count) {
    const size_t o = off;
    off = align_up(off + count * sizeof(double), 256);
    return o;
  };
  const size_t o_part = take((size_t)nblk * kKeOmegaVals), o_om = take(kKeMaxBands), o_f = take(hw),
               o_etf = take(n2), o_S = take((size_t)c * c * L * L), o_A = take((size_t)n2 * n2),
               o_gj = take(4 * (size_t)n2), o_info = take(2);
  if (off > ctx->ke_bytes) {
    if (ctx->ke_ws) {
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(ctx->ke_ws));
      ctx->ke_ws = nullptr;
      ctx->ke_bytes = 0;
    }
    if (hipMalloc(&ctx->ke_ws, off) != hipSuccess) {
      ctx->ke_ws = nullptr;
      return LLP_E_OOM;
    }
    ctx->ke_bytes = off;
  }
  char* base = (char*)ctx->ke_ws;
  double* part = (double*)(base + o_part);
  double* om = (double*)(base + o_om);
  double* f = (double*)(base + o_f);
  double* etf = (double*)(base + o_etf);
  double* Sc = (double*)(base + o_S);
  double* A = (double*)(base + o_A);
  double* gj = (double*)(base + o_gj);
  double* info = (double*)(base + o_info);

  hipLaunchKernelGGL(k_ke_omega_terms, dim3(nblk), dim3(kBlock), 0, s, K, lrms, pan, part);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_ke_omega_solve, dim3(1), dim3(kBlock), 0, s, K, (const double*)part, nblk, om);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_ke_f, dim3((unsigned)((hw + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, K, lrms,
                     (const double*)om, f);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_ke_etf, dim3(n2), dim3(kBlock), 0, s, K, pan, (const double*)f, etf);
  HIP_TRY(hipGetLastError());
  const size_t corr_lds = ((size_t)W + 2 * (n - 1) + w) * sizeof(float);
  if (corr_lds > 64 * 1024)
    HIP_TRY(hipFuncSetAttribute((const void*)k_ke_corr, hipFuncAttributeMaxDynamicSharedMemorySize, (int)corr_lds));
  hipLaunchKernelGGL(k_ke_corr, dim3((unsigned)(c * c * L)), dim3(kBlock), corr_lds, s, K, pan, Sc);
  HIP_TRY(hipGetLastError());
  const unsigned nA = (unsigned)(((size_t)n2 * n2 + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_ke_ete, dim3(nA), dim3(kBlock), 0, s, K, (const double*)Sc, A);
  HIP_TRY(hipGetLastError());
  double *r0 = gj, *c0 = gj + n2, *r1 = gj + 2 * n2, *c1 = gj + 3 * n2;
  hipLaunchKernelGGL(k_ke_gj_init, dim3((n2 + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n2, (const double*)A, r0,
                     c0);
  HIP_TRY(hipGetLastError());
  for (int k = 0; k < n2; ++k) {
    const bool even = (k & 1) == 0;
    hipLaunchKernelGGL(k_ke_gj, dim3(nA), dim3(kBlock), 0, s, n2, k, A, even ? r0 : r1, even ? c0 : c1,
                       even ? r1 : r0, even ? c1 : c0);
    HIP_TRY(hipGetLastError());
  }
  const size_t lds = ke_lds_bytes(n);
  HIP_TRY(hipFuncSetAttribute((const void*)k_ke_gadmm, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_ke_gadmm, dim3(1), dim3(kKeThreads), lds, s, K, (const double*)A, (const double*)etf, kernel,
                     info);
  HIP_TRY(hipGetLastError());
  if (omega_out) HIP_TRY(hipMemcpyAsync(omega_out, om, sizeof(double) * Np, hipMemcpyDeviceToDevice, s));
  if (rep) {
    double hinfo[2];
    HIP_TRY(hipMemcpyAsync(hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    rep->iters = (int)hinfo[0];
    rep->change = hinfo[1];
  }
  return LLP_OK;
}

}  // extern "C"
