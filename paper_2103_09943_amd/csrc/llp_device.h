// Device helpers shared by the iteration kernels (llp_operator.hip, llp_fast.hip).
#pragma once

#include "llp_internal.h"

namespace llp {
namespace dev {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ int wrapi(int i, int n) {
  int m = i % n;
  return m < 0 ? m + n : m;
}
__host__ __device__ __forceinline__ int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
__host__ __device__ __forceinline__ int pos_mod(int a, int b) { return a - floor_div(a, b) * b; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sums K values over a block of NW waves (red: K * NW doubles of LDS); results valid in thread 0.
template <int K, int NW = kWaves>
__device__ __forceinline__ void block_sums(double (&v)[K], double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    v[k] = wave_sum(v[k]);
    if (lane == 0) red[k * NW + wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double t = 0.0;
      for (int i = 0; i < NW; ++i) t += red[k * NW + i];
      v[k] = t;
    }
  }
}

// Sums K values over the workgroup and stores them at dst[0..K) (thread 0).
template <int K, int NW = kWaves>
__device__ __forceinline__ void block_partials(double (&v)[K], double* red, double* dst) {
  block_sums<K, NW>(v, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) dst[k] = v[k];
  }
}

// Workgroups are dealt round-robin to the 8 XCDs.  Remap the flat id so that each XCD walks a contiguous run of
// (tile, band) pairs, bands of one tile adjacent: halos and per-scene PAN statistics stay in one XCD's L2.
__device__ __forceinline__ void tile_and_band(int ntiles, int N, int bid, int& tile, int& ch) {
  const int nb = ntiles * N;
  const int b8 = (nb / 8) * 8;
  const int lin = bid < b8 ? (bid % 8) * (b8 / 8) + bid / 8 : bid;
  tile = lin / N;
  ch = lin % N;
}

}  // namespace dev

// Arguments of the iteration kernels (generic and fast paths).
struct DirArgs {
  int mode;        // 0: y = D B z (z = rin);  1: first iteration, p_0 = r_0;  2: iteration k >= 1
  int final_step;  // mode 2: update x and r only (the iteration cap is reached)
  int k_iter;      // iteration index k (the iterate produced is x_k)
  const float* rin;
  const float* qin;
  const float* pin;
  float* rout;
  float* pout;
  float* x;
  float* y;
  double* partials;  // [N][pstride][3]; this kernel writes one double per workgroup of each active band
  ChanState* st;
  int tiles_x, ntiles, pstride;
  int PS;  // floats per polyphase plane (padded)
};

struct ApplyArgs {
  int mode;  // 0: q = A z (z = p);  1: CG: also gamma, sigma, tau -> alpha, beta
  const float* p;
  const float* r;
  const float* y;
  const float* G;
  const float* MU;
  const float* DI;
  float* q;
  double* partials;  // [N][pstride][3]; this kernel writes three doubles per workgroup of each active band
  ChanState* st;
  int tiles_x, ntiles, pstride;
  int offL, offX, offY, QPS;  // LDS layout (floats); the region buffer starts at 0
};


// Fast path (llp_fast.hip): kernels specialised on (C, R, r).
bool fast_path_available(int C, int R, int r);
int fast_apply_lds_floats(int C, int R, int r, int variant);
hipError_t launch_dir_fast(const Geom& g, DirArgs A, int tyl, const float* u, hipStream_t s);
hipError_t launch_apply_fast(const Geom& g, int variant, ApplyArgs A, const float* u, hipStream_t s);
// Batched CG launches over the scenes [first, first+count) of a class table (all of one (c, R, r) class and one
// launch configuration): every workgroup finds its scene by binary search on the block offsets.  parity selects
// the residual/direction buffers: iteration k reads r[parity], p[parity] and writes r[1-parity], p[1-parity].
// total_blocks == 0 only prepares the kernel (its LDS limit) without launching it.

}  // namespace llp
