// Learned warm start of the CG solve (the paper leaves the initial guess open, Sec. III-B): a five-layer 3x3
// convolution network (2 -> 32 -> 32 -> 32 -> 32 -> 1 channels, ReLU after the first four, periodic padding)
// maps a band's bicubic upsampling and the PAN image to an estimate of the HRMS band:
//     z0 = x_up + s * net([(x_up - m)/s, (Y - m_Y)/s_Y]),
// m, s the mean and population standard deviation of the LRMS band, m_Y, s_Y those of the PAN image.
//
// Arithmetic: layer inputs and weights in bfloat16 (round to nearest even), products on the matrix cores
// (v_mfma_f32_16x16x32_bf16) with FP32 accumulation, FP32 biases; training keeps FP32 master weights and Adam
// moments.  The backward pass rounds every layer-output gradient to bfloat16 before its products.
//
// Layout: activations are [band][H][W][32] bfloat16 (channel-fastest, 64 bytes per pixel); the 2-channel input
// and the 1-channel output gradient are stored zero-padded to 32 channels, so that every layer, forward and
// backward, runs the same implicit-GEMM kernels: per 3x3 tap one MFMA K-step of 32 input channels.
//
// MFMA operand layout (16x16x32, one wave): lane l holds A[m = l%16][k = 8(l/16) .. 8(l/16)+7],
// B[k = 8(l/16) .. +7][n = l%16]; the accumulator holds D[m = 4(l/16) + i][n = l%16], i = 0..3.
#include <math.h>
#include <stdint.h>

#include "llp_cnn.h"
#include "llp_device.h"

namespace llp {

// Periodic index for -n <= i < 2n by one conditional add or subtract (no division); pos_mod otherwise.
__device__ __forceinline__ int wrap_p(int i, int n) {
  if (i >= -n && i < 2 * n) return i < 0 ? i + n : (i >= n ? i - n : i);
  return dev::pos_mod(i, n);
}
using namespace dev;

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;

constexpr int kCh = 32;        // padded channel count of every activation
constexpr int kTaps = 9;
constexpr int kTileW = 64;     // conv kernel: pixels per wave (one row segment)
constexpr int kTileRows = 4;   // conv kernel: rows per workgroup (one per wave)

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint32_t pack2(float a, float b) { return (uint32_t)f2bf(a) | ((uint32_t)f2bf(b) << 16); }

__device__ __forceinline__ int wrapc(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// ------------------------------------------------------------------------------------- band statistics ---
// Mean and population standard deviation (1 where it is 0) of each of `count` arrays of `len` floats, array k
// at src + k * stride.  Two steps, deterministic: every workgroup sums a chunk in FP64 (part[k][chunk][2]),
// then one workgroup per array adds the chunks in order.
constexpr int kStatChunk = kBlock * 16;

__global__ __launch_bounds__(kBlock) void k_stats_part(const float* __restrict__ src, size_t stride, size_t len,
                                                       int nchunk, double* __restrict__ part) {
  __shared__ double red[2 * kWaves];
  const float* a = src + (size_t)blockIdx.y * stride;
  const size_t e0 = (size_t)blockIdx.x * kStatChunk;
  const size_t e1 = e0 + kStatChunk < len ? e0 + kStatChunk : len;
  double s[2] = {0.0, 0.0};
  for (size_t i = e0 + threadIdx.x; i < e1; i += kBlock) {
    const double v = a[i];
    s[0] += v;
    s[1] += v * v;
  }
  block_partials<2>(s, red, part + ((size_t)blockIdx.y * nchunk + blockIdx.x) * 2);
}

__global__ __launch_bounds__(kBlock) void k_stats_final(const double* __restrict__ part, int nchunk, size_t len,
                                                        float* __restrict__ out) {
  __shared__ double red[2 * kWaves];
  const double* p = part + (size_t)blockIdx.x * nchunk * 2;
  double s[2] = {0.0, 0.0};
  for (int i = threadIdx.x; i < nchunk; i += kBlock) {
    s[0] += p[2 * i];
    s[1] += p[2 * i + 1];
  }
  block_sums<2>(s, red);
  if (threadIdx.x == 0) {
    const double m = s[0] / (double)len;
    double var = s[1] / (double)len - m * m;
    if (var < 0.0) var = 0.0;
    const double sd = sqrt(var);
    out[2 * blockIdx.x] = (float)m;
    out[2 * blockIdx.x + 1] = sd > 0.0 ? (float)sd : 1.0f;
  }
}

// --------------------------------------------------------------------------------------- network input ---
// Keys' cubic convolution weight (a = -1/2) at offset s.
__device__ __forceinline__ float keys(float s) {
  s = fabsf(s);
  if (s <= 1.0f) return (1.5f * s - 2.5f) * s * s + 1.0f;
  if (s < 2.0f) return ((-0.5f * s + 2.5f) * s - 4.0f) * s + 2.0f;
  return 0.0f;
}

// x_up = bicubic(X_band) (HR pixel i at LR coordinate i / c, periodic) and the input planes of the network.
__global__ __launch_bounds__(kBlock) void k_input(CnnGeom g, const float* __restrict__ X, const float* __restrict__ Y,
                                                  const float* __restrict__ stats, const float* __restrict__ statsY,
                                                  float* __restrict__ xup, uint16_t* __restrict__ in0) {
  const size_t HW = (size_t)g.H * g.W;
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  const int band = blockIdx.y;
  if (idx >= HW) return;
  const int i = (int)idx / g.W, j = (int)idx - i * g.W;  // H W < 2^31
  const int mi = i / g.c, mj = j / g.c;
  const float ti = (float)(i - mi * g.c) / (float)g.c, tj = (float)(j - mj * g.c) / (float)g.c;
  float wy[4], wx[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    wy[k] = keys((float)(k - 1) - ti);
    wx[k] = keys((float)(k - 1) - tj);
  }
  const float* Xb = X + (size_t)band * g.h * g.w;
  float v = 0.0f;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int r = wrap_p(mi + a - 1, g.h);
    float rs = 0.0f;
#pragma unroll
    for (int b = 0; b < 4; ++b) rs = fmaf(wx[b], Xb[(size_t)r * g.w + wrap_p(mj + b - 1, g.w)], rs);
    v = fmaf(wy[a], rs, v);
  }
  xup[(size_t)band * HW + idx] = v;
  const float m = stats[2 * band], s = stats[2 * band + 1];
  const float mY = statsY[0], sY = statsY[1];
  u32x4* dst = (u32x4*)(in0 + ((size_t)band * HW + idx) * kCh);
  const u32x4 z = {0u, 0u, 0u, 0u};
  u32x4 first = z;
  first.x = pack2((v - m) / s, (Y[idx] - mY) / sY);
  dst[0] = first;
  dst[1] = z;
  dst[2] = z;
  dst[3] = z;
}

// ------------------------------------------------------------------------------------------ convolution ---
// out[p][o] = sum_{tap, c} A_tap[o][c] * in[p + off(tap)][c], off(tap) = (tap/3 - 1, tap%3 - 1), p periodic.
// The weights arrive as ready MFMA A operands: wt[(tap * COB + cob) * 64 + lane] holds 8 bfloat16.
// One wave computes one row segment of 64 pixels (4 MFMA column blocks) for COB blocks of 16 outputs.
// Epilogues:
//   kEpiRelu  out = relu(acc + bias), bfloat16, all 32 channels
//   kEpiFinal channel 0 only: net = acc + bias; netout = net (FP32, optional); z0 = x_up + s * net (optional)
//   kEpiMask  out = acc * (mask > 0) (the ReLU derivative of the layer below), bfloat16, all 32 channels
enum { kEpiRelu = 0, kEpiFinal = 1, kEpiMask = 2 };

template <int COB, int EPI>
__global__ __launch_bounds__(kBlock) void k_conv(CnnGeom g, const uint16_t* __restrict__ in,
                                                 const u32x4* __restrict__ wt, const float* __restrict__ bias,
                                                 uint16_t* __restrict__ out, const uint16_t* __restrict__ mask,
                                                 float* __restrict__ netout, float* __restrict__ z0,
                                                 const float* __restrict__ xup, const float* __restrict__ stats) {
  // The workgroup's input tile (its 4 rows and 64 columns plus a 1-pixel periodic halo, all 32 channels) is
  // staged in LDS once; the 9 taps of the 4 waves then read their MFMA B operands from there.
  __shared__ __align__(16) uint16_t tile[kTileRows + 2][kTileW + 2][kCh];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = blockIdx.y * kTileRows, row = row0 + wave;
  const int band = blockIdx.z;
  const int H = g.H, W = g.W;
  const size_t HW = (size_t)H * W;
  const int col0 = blockIdx.x * kTileW;
  const int kq = lane >> 4, n16 = lane & 15;
  const uint16_t* inb = in + (size_t)band * HW * kCh;
  for (int k = threadIdx.x; k < (kTileRows + 2) * (kTileW + 2) * 4; k += kBlock) {
    const int pix = k >> 2, part = k & 3;
    const int lr = pix / (kTileW + 2), lc = pix % (kTileW + 2);
    const int sr = wrap_p(row0 + lr - 1, H), sc = wrap_p(col0 + lc - 1, W);
    *(u32x4*)&tile[lr][lc][part * 8] = *(const u32x4*)(inb + ((size_t)sr * W + sc) * kCh + part * 8);
  }
  __syncthreads();
  if (row >= H) return;  // the only barrier is behind
  f32x4 acc[COB][4];
#pragma unroll
  for (int cb = 0; cb < COB; ++cb)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc[cb][nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int dy = 0; dy < 3; ++dy) {
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const int tap = dy * 3 + dx;
      bf16x8 a[COB];
#pragma unroll
      for (int cb = 0; cb < COB; ++cb) a[cb] = __builtin_bit_cast(bf16x8, wt[(tap * COB + cb) * 64 + lane]);
      bf16x8 b[4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
        b[nb] = __builtin_bit_cast(bf16x8, *(const u32x4*)&tile[wave + dy][nb * 16 + n16 + dx][kq * 8]);
#pragma unroll
      for (int cb = 0; cb < COB; ++cb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
          acc[cb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[cb], b[nb], acc[cb][nb], 0, 0, 0);
    }
  }
  // epilogue: lane holds outputs o = cb*16 + 4*kq + i of pixel col0 + nb*16 + n16
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int col = col0 + nb * 16 + n16;
    if (col >= W) continue;
    const size_t p = (size_t)band * HW + (size_t)row * W + col;
    if (EPI == kEpiFinal) {
      if (kq == 0) {
        const float net = acc[0][nb][0] + bias[0];
        if (netout) netout[p] = net;
        if (z0) z0[p] = fmaf(stats[2 * band + 1], net, xup[p]);
      }
    } else {
#pragma unroll
      for (int cb = 0; cb < COB; ++cb) {
        const int o = cb * 16 + kq * 4;
        float v[4];
        if (EPI == kEpiRelu) {
#pragma unroll
          for (int i = 0; i < 4; ++i) v[i] = fmaxf(acc[cb][nb][i] + bias[o + i], 0.0f);
        } else {
          const uint2 mk = *(const uint2*)(mask + p * kCh + o);
          v[0] = (mk.x & 0xFFFFu) && !(mk.x & 0x8000u) ? acc[cb][nb][0] : 0.0f;
          v[1] = (mk.x >> 16) && !(mk.x & 0x80000000u) ? acc[cb][nb][1] : 0.0f;
          v[2] = (mk.y & 0xFFFFu) && !(mk.y & 0x8000u) ? acc[cb][nb][2] : 0.0f;
          v[3] = (mk.y >> 16) && !(mk.y & 0x80000000u) ? acc[cb][nb][3] : 0.0f;
        }
        uint2 st;
        st.x = pack2(v[0], v[1]);
        st.y = pack2(v[2], v[3]);
        *(uint2*)(out + p * kCh + o) = st;
      }
      if (COB == 1) {  // outputs 16..31 of a one-block layer are zero (padding)
        *(uint2*)(out + p * kCh + 16 + kq * 4) = uint2{0u, 0u};
      }
    }
  }
}

// ------------------------------------------------------------------------------------------ weight grad ---
// dW[o][c][tap] = sum_p gout[p][o] * in[p + off(tap)][c] and db[o] = sum_p gout[p][o] over all pixels of all
// bands, per workgroup (persistent: tiles of 4 rows x 64 columns, strided over the grid); partial sums go to
// part[blockIdx.x][32*32*9 + 32] in the flat order o, c, tap then the biases.
constexpr int kGR = 4, kGC = 64;                 // tile rows, columns
constexpr int kAR = kGR + 2, kAC = kGC + 8;      // staged input rows (halo 1) and padded columns (halo at 0..65)
constexpr int kGradPart = kCh * kCh * kTaps + kCh;

__device__ __forceinline__ bf16x8 lds_row8(const uint16_t* base, int off) {  // 8 bfloat16 at any even/odd offset
  const uint32_t* w = (const uint32_t*)(base + (off & ~1));
  const uint32_t sh = (uint32_t)(off & 1) * 16u;
  u32x4 r;
  const uint32_t w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3], w4 = w[4];
  r.x = __builtin_amdgcn_alignbit(w1, w0, sh);
  r.y = __builtin_amdgcn_alignbit(w2, w1, sh);
  r.z = __builtin_amdgcn_alignbit(w3, w2, sh);
  r.w = __builtin_amdgcn_alignbit(w4, w3, sh);
  return __builtin_bit_cast(bf16x8, r);
}

__global__ __launch_bounds__(kBlock) void k_wgrad(CnnGeom g, const uint16_t* __restrict__ gout,
                                                  const uint16_t* __restrict__ in, float* __restrict__ part) {
  __shared__ __align__(16) uint16_t gT[kCh][kGR * kGC];          // [o][pixel of the tile]
  __shared__ __align__(16) uint16_t aT[kCh][kAR][kAC];           // [c][row][col]: input with a 1-pixel halo
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kq = lane >> 4, n16 = lane & 15;
  const int H = g.H, W = g.W;
  const size_t HW = (size_t)H * W;
  const int tx = (W + kGC - 1) / kGC, ty = (H + kGR - 1) / kGR;
  const int ntiles = tx * ty * g.N;
  // this wave's (tap, output block) pairs: w, w+4, ... < 18
  constexpr int kPairs = (2 * kTaps + 3) / 4;
  f32x4 acc[kPairs][2];
#pragma unroll
  for (int q = 0; q < kPairs; ++q) acc[q][0] = acc[q][1] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  float bsum = 0.0f;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int band = t / (tx * ty), rem = t % (tx * ty);
    const int r0 = (rem / tx) * kGR, c0 = (rem % tx) * kGC;
    const uint16_t* gb = gout + (size_t)band * HW * kCh;
    const uint16_t* ib = in + (size_t)band * HW * kCh;
    __syncthreads();  // the previous tile's LDS reads are done
    // stage gout (zero outside the image) and the input (periodic) transposed to channel-major
    for (int k = threadIdx.x; k < kGR * kGC * 4; k += kBlock) {
      const int pix = k >> 2, part8 = k & 3;
      const int rr = r0 + pix / kGC, cc = c0 + pix % kGC;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (rr < H && cc < W) v = *(const u32x4*)(gb + ((size_t)rr * W + cc) * kCh + part8 * 8);
      const uint32_t vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        gT[part8 * 8 + 2 * e][pix] = (uint16_t)(vv[e] & 0xFFFFu);
        gT[part8 * 8 + 2 * e + 1][pix] = (uint16_t)(vv[e] >> 16);
      }
    }
    for (int k = threadIdx.x; k < kAR * (kGC + 2) * 4; k += kBlock) {
      const int pix = k >> 2, part8 = k & 3;
      const int lr = pix / (kGC + 2), lc = pix % (kGC + 2);
      const int rr = wrap_p(r0 + lr - 1, H), cc = wrap_p(c0 + lc - 1, W);
      const u32x4 v = *(const u32x4*)(ib + ((size_t)rr * W + cc) * kCh + part8 * 8);
      const uint32_t vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        aT[part8 * 8 + 2 * e][lr][lc] = (uint16_t)(vv[e] & 0xFFFFu);
        aT[part8 * 8 + 2 * e + 1][lr][lc] = (uint16_t)(vv[e] >> 16);
      }
    }
    __syncthreads();
    if (threadIdx.x < kCh) {
      float s = 0.0f;
      for (int k = 0; k < kGR * kGC; ++k) s += bf2f(gT[threadIdx.x][k]);
      bsum += s;
    }
    // K-steps: 32 pixels of one tile row (8 steps per tile)
#pragma unroll 1
    for (int ks = 0; ks < kGR * kGC / 32; ++ks) {
      const int rr = ks / (kGC / 32), cs = (ks % (kGC / 32)) * 32;
#pragma unroll
      for (int q = 0; q < kPairs; ++q) {
        const int pair = wave + 4 * q;
        if (pair >= 2 * kTaps) break;
        const int tap = pair >> 1, ob = pair & 1;
        const int dy = tap / 3, dx = tap % 3;
        // A[m = o][k = pixel]: gout of output ob*16 + n16 at 8 consecutive pixels
        const bf16x8 a = __builtin_bit_cast(bf16x8, *(const u32x4*)&gT[ob * 16 + n16][rr * kGC + cs + 8 * kq]);
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          // B[k = pixel][n = c]: input channel cb*16 + n16 at the same pixels shifted by the tap
          const bf16x8 b = lds_row8(&aT[cb * 16 + n16][rr + dy][0], cs + 8 * kq + dx);
          acc[q][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[q][cb], 0, 0, 0);
        }
      }
    }
  }
  float* dst = part + (size_t)blockIdx.x * kGradPart;
#pragma unroll
  for (int q = 0; q < kPairs; ++q) {
    const int pair = wave + 4 * q;
    if (pair >= 2 * kTaps) break;
    const int tap = pair >> 1, ob = pair & 1;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int o = ob * 16 + kq * 4 + i, c = cb * 16 + n16;
        dst[(o * kCh + c) * kTaps + tap] = acc[q][cb][i];
      }
  }
  if (threadIdx.x < kCh) dst[kCh * kCh * kTaps + threadIdx.x] = bsum;
}

// Sum of the per-workgroup partials into the layer's gradient in the flat parameter layout (W [cout][cin][3][3]
// then b [cout]) at grad.  A workgroup takes kRedOut outputs; its kRedSlices slices of threads each sum every
// kRedSlices-th partial (slice s: partials s, s + kRedSlices, ...), then the slices are added in order: a fixed
// order, so training stays deterministic, with the loads of many partials in flight at once.
constexpr int kRedOut = 32, kRedSlices = kBlock / kRedOut;

__global__ __launch_bounds__(kBlock) void k_wgrad_reduce(const float* __restrict__ part, int nparts, int cout,
                                                         int cin, float* __restrict__ grad) {
  __shared__ double red[kRedSlices][kRedOut];
  const int nW = cout * cin * kTaps;
  const int j = threadIdx.x % kRedOut, sl = threadIdx.x / kRedOut;
  const int idx = blockIdx.x * kRedOut + j;
  double acc = 0.0;
  if (idx < nW + cout) {
    int src;
    if (idx < nW) {
      const int o = idx / (cin * kTaps), c = (idx / kTaps) % cin, tap = idx % kTaps;
      src = (o * kCh + c) * kTaps + tap;
    } else {
      src = kCh * kCh * kTaps + (idx - nW);
    }
#pragma unroll 8
    for (int k = sl; k < nparts; k += kRedSlices) acc += (double)part[(size_t)k * kGradPart + src];
  }
  red[sl][j] = acc;
  __syncthreads();
  if (sl == 0 && idx < nW + cout) {
    double s = 0.0;
    for (int q = 0; q < kRedSlices; ++q) s += red[q][j];
    grad[idx] = (float)s;
  }
}

// ------------------------------------------------------------------------------------- loss and output grad ---
// t = (Z - x_up)/s, diff = net - t; loss partials sum diff^2; gout channel 0 = bfloat16(2 diff / P).
__global__ __launch_bounds__(kBlock) void k_loss(CnnGeom g, const float* __restrict__ net,
                                                 const float* __restrict__ Z, const float* __restrict__ xup,
                                                 const float* __restrict__ stats, float inv_count,
                                                 uint16_t* __restrict__ gout, double* __restrict__ part) {
  __shared__ double red[kWaves];
  const size_t HW = (size_t)g.H * g.W;
  const size_t total = HW * g.N;
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  double acc = 0.0;
  if (idx < total) {
    const int band = (int)(idx / HW);
    const float t = (Z[idx] - xup[idx]) / stats[2 * band + 1];
    const float d = net[idx] - t;
    acc = (double)d * d;
    u32x4* dst = (u32x4*)(gout + idx * kCh);
    const u32x4 z = {0u, 0u, 0u, 0u};
    u32x4 first = z;
    first.x = (uint32_t)f2bf(2.0f * d * inv_count);
    dst[0] = first;
    dst[1] = z;
    dst[2] = z;
    dst[3] = z;
  }
  double v[1] = {acc};
  block_partials<1>(v, red, part + blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_sum(const double* __restrict__ part, int n, double scale,
                                                double* __restrict__ out) {
  __shared__ double red[kWaves];
  double s[1] = {0.0};
  for (int i = threadIdx.x; i < n; i += kBlock) s[0] += part[i];
  block_sums<1>(s, red);
  if (threadIdx.x == 0) out[0] = s[0] * scale;
}

// ---------------------------------------------------------------------------------- weights and optimiser ---
// MFMA A operands of one layer from the FP32 master weights W [cout][cin][3][3]:
//   forward  (COB blocks of 16 outputs):  A_tap[m = o][k = c]      = W[o][c][tap]
//   backward (2 blocks of 16 inputs):     A_tap[m = c][k = o]      = W[o][c][8 - tap]   (transposed, flipped)
// Entries outside (cout, cin) are zero.  out[(tap * COB + cob) * 64 + lane] holds the lane's 8 values.
__global__ __launch_bounds__(kBlock) void k_prep(const float* __restrict__ Wm, int cout, int cin, int cob,
                                                 int backward, u32x4* __restrict__ out) {
  const int idx = blockIdx.x * kBlock + threadIdx.x;  // (tap, block, lane)
  if (idx >= kTaps * cob * 64) return;
  const int lane = idx & 63, blk = (idx >> 6) % cob, tap = idx / (64 * cob);
  const int m = blk * 16 + (lane & 15);
  uint32_t w[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float v2[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k = (lane >> 4) * 8 + 2 * e + h;
      const int o = backward ? k : m, c = backward ? m : k;
      const int tp = backward ? kTaps - 1 - tap : tap;
      v2[h] = (o < cout && c < cin) ? Wm[(o * cin + c) * kTaps + tp] : 0.0f;
    }
    w[e] = pack2(v2[0], v2[1]);
  }
  out[idx] = u32x4{w[0], w[1], w[2], w[3]};
}

__global__ __launch_bounds__(kBlock) void k_adam(float* __restrict__ p, const float* __restrict__ grad,
                                                 float* __restrict__ m, float* __restrict__ v, int n, float lr,
                                                 float beta1, float beta2, float eps, float bc1, float bc2) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float gi = grad[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

}  // namespace

// ================================================================================================= host ===

int cnn_layer_cin(int l) { return l == 0 ? 2 : 32; }
int cnn_layer_cout(int l) { return l == kCnnLayers - 1 ? 1 : 32; }
int cnn_layer_offset(int l) {
  int off = 0;
  for (int k = 0; k < l; ++k) off += cnn_layer_cout(k) * cnn_layer_cin(k) * kTaps + cnn_layer_cout(k);
  return off;
}
size_t cnn_tile_bytes(int cob) { return (size_t)kTaps * cob * 64 * 16; }
int cnn_wgrad_parts() { return 512; }
size_t cnn_wgrad_part_floats() { return kGradPart; }

size_t cnn_stats_parts(size_t len) { return (len + kStatChunk - 1) / kStatChunk; }

hipError_t cnn_launch_stats(const float* src, size_t stride, size_t len, int count, double* part, float* out,
                            hipStream_t s) {
  const int nchunk = (int)cnn_stats_parts(len);
  hipLaunchKernelGGL(k_stats_part, dim3(nchunk, count), dim3(kBlock), 0, s, src, stride, len, nchunk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_stats_final, dim3(count), dim3(kBlock), 0, s, part, nchunk, len, out);
  return hipGetLastError();
}

hipError_t cnn_launch_input(const CnnGeom& g, const float* X, const float* Y, const float* stats,
                            const float* statsY, float* xup, uint16_t* in0, hipStream_t s) {
  const size_t HW = (size_t)g.H * g.W;
  hipLaunchKernelGGL(k_input, dim3((unsigned)((HW + kBlock - 1) / kBlock), g.N), dim3(kBlock), 0, s, g, X, Y, stats,
                     statsY, xup, in0);
  return hipGetLastError();
}

hipError_t cnn_launch_conv(const CnnGeom& g, int cob, int epi, const uint16_t* in, const void* wt,
                           const float* bias, uint16_t* out, const uint16_t* mask, float* netout, float* z0,
                           const float* xup, const float* stats, hipStream_t s) {
  const dim3 grid((g.W + kTileW - 1) / kTileW, (g.H + kTileRows - 1) / kTileRows, g.N);
  const u32x4* w = (const u32x4*)wt;
  if (cob == 2 && epi == kEpiRelu)
    hipLaunchKernelGGL((k_conv<2, kEpiRelu>), grid, dim3(kBlock), 0, s, g, in, w, bias, out, mask, netout, z0, xup,
                       stats);
  else if (cob == 2 && epi == kEpiMask)
    hipLaunchKernelGGL((k_conv<2, kEpiMask>), grid, dim3(kBlock), 0, s, g, in, w, bias, out, mask, netout, z0, xup,
                       stats);
  else if (cob == 1 && epi == kEpiFinal)
    hipLaunchKernelGGL((k_conv<1, kEpiFinal>), grid, dim3(kBlock), 0, s, g, in, w, bias, out, mask, netout, z0, xup,
                       stats);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t cnn_launch_wgrad(const CnnGeom& g, const uint16_t* gout, const uint16_t* in, float* part, int cout,
                            int cin, float* grad, hipStream_t s) {
  const int tx = (g.W + kGC - 1) / kGC, ty = (g.H + kGR - 1) / kGR;
  int nparts = tx * ty * g.N;
  if (nparts > cnn_wgrad_parts()) nparts = cnn_wgrad_parts();
  hipLaunchKernelGGL(k_wgrad, dim3(nparts), dim3(kBlock), 0, s, g, gout, in, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n = cout * cin * kTaps + cout;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((n + kRedOut - 1) / kRedOut), dim3(kBlock), 0, s, part, nparts, cout, cin,
                     grad);
  return hipGetLastError();
}

hipError_t cnn_launch_loss(const CnnGeom& g, const float* net, const float* Z, const float* xup,
                           const float* stats, uint16_t* gout, double* part, double* loss, hipStream_t s) {
  const size_t total = (size_t)g.N * g.H * g.W;
  const unsigned blocks = (unsigned)((total + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_loss, dim3(blocks), dim3(kBlock), 0, s, g, net, Z, xup, stats, (float)(1.0 / (double)total),
                     gout, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kBlock), 0, s, part, (int)blocks, 1.0 / (double)total, loss);
  return hipGetLastError();
}

size_t cnn_loss_parts(const CnnGeom& g) { return ((size_t)g.N * g.H * g.W + kBlock - 1) / kBlock; }

hipError_t cnn_launch_prep(const float* Wm, int cout, int cin, int cob, int backward, void* out, hipStream_t s) {
  const int n = kTaps * cob * 64;
  hipLaunchKernelGGL(k_prep, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, Wm, cout, cin, cob, backward,
                     (u32x4*)out);
  return hipGetLastError();
}

hipError_t cnn_launch_adam(float* p, const float* grad, float* m, float* v, int n, float lr, int t, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = (float)(1.0 - pow(0.9, t)), bc2 = (float)(1.0 - pow(0.999, t));
  hipLaunchKernelGGL(k_adam, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, p, grad, m, v, n, lr, b1, b2, 1e-8f,
                     bc1, bc2);
  return hipGetLastError();
}

}  // namespace llp
