// Fourier-domain preconditioner of the conjugate-gradient solve of eq. (Z_ini_matting) (Sec. III-B), and the
// batched mixed-radix FFT it runs on.  Not part of the paper's method: P = B^T D^T D B + lambda mbar L^T L keeps
// the data term of eq. (Z_ini_matting) exactly and replaces the matting matrix of eq. (matting_matrix) by the
// scalar mbar, the mean of its diagonal.
//
// B is circular convolution (Sec. II-A), L circular convolution with the 5-point stencil (eq. reg2) and D
// decimation at phase 0, so in the Fourier domain of an H x W plane P couples only the c^2 frequencies
// (k1 + s h, k2 + t w), s, t < c, that D aliases onto one low-resolution frequency (k1, k2):
//     (P z)^[K] = d_K z^[K] + conj(U_K) / c^2 * sum_{K' in group} U_K' z^[K'],   d_K = lambda mbar Sh_K^2,
// U the DFT of the kernel and Sh the stencil's symbol.  Each group is one c^2 x c^2 block, solved per thread.
//
// Layout.  Two bands go through one complex transform (band a real, band b imaginary: P^{-1} is real, hence
// complex-linear).  The H x W plane is split into its c^2 polyphase components x_{al,be}[m][k] =
// x[c m + al][c k + be], each an h x w plane, so that
//     z^[k1 + s h][k2 + t w] = sum_{al,be} e^{-2 pi i (al k1 / H + be k2 / W)} X_{al,be}[k1][k2] w_c^{al s + be t}
// with X_{al,be} the h x w DFT of x_{al,be} and w_c = e^{-2 pi i / c}: an h x w transform per component, a
// twiddle, and a c x c DFT per low-resolution frequency.  Spectra are stored cell-major, [pair][k1][k2][al c + be]
// (c^2 complex values, 128 bytes at c = 4, per cell), so both passes read and write whole cells:
//   rows    one workgroup per (pair, LR row m): the c HR rows c m .. c m + c - 1 (coalesced) -> c^2 length-w
//           transforms in LDS -> the row of cells;
//   columns one workgroup per (pair, LR column k2): h cells -> c^2 length-h transforms -> per cell the twiddle,
//           c x c DFT, group solve, inverse c x c DFT, conjugate twiddle -> inverse length-h transforms;
//   rows    inverse length-w transforms -> the c HR rows of both bands, scaled by 1/(H W).
//
// FFT.  Stockham autosort passes of radix 8, 4, 2, 7, 5 and 3 on LDS-resident sequences: per pass every thread
// loads its butterflies' inputs into registers, multiplies by twiddles from a table evaluated in FP64 and
// rounded once, transforms, and after a barrier writes its outputs to their sorted positions.  Inverse
// transforms conjugate on the way in and out.
#include "llp_device.h"

#include <math.h>
#include <stdlib.h>

#include <algorithm>
#include <utility>

namespace llp {
using namespace dev;

namespace {

constexpr int T = kPcThreads;      // threads of the row passes (TS for tables whose rows hold <= kPcSmallElems)
constexpr int TS = kPcSmallRowThreads;
constexpr int TC = kPcColThreads;  // threads of the column pass (more registers per thread for the group solve)
// Complex values a row-pass workgroup of TH threads holds at most.
__host__ __device__ constexpr int row_elems(int TH) { return TH == T ? kPcMaxElems : kPcSmallElems; }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }  // -i a

// threadIdx.x behind an optimisation barrier: the persistent column loop would otherwise hoist every address
// derived from it out of the loop and keep them all live, beyond the register budget.
__device__ __forceinline__ int opaque_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Loads and stores through pointers taken from a descriptor: in the global address space, so that they are
// issued as global (not flat) memory instructions and waits on LDS accesses do not wait for them.
#define LLP_G __attribute__((address_space(1)))
typedef float gf2 __attribute__((ext_vector_type(2)));
typedef float gf4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float gld(const float* p) { return *(const LLP_G float*)p; }
__device__ __forceinline__ float2 gld(const float2* p) {
  const gf2 v = *(const LLP_G gf2*)p;
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ float4 gld(const float4* p) {
  const gf4 v = *(const LLP_G gf4*)p;
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gst(float* p, float v) { *(LLP_G float*)p = v; }
__device__ __forceinline__ void gst(double* p, double v) { *(LLP_G double*)p = v; }
__device__ __forceinline__ void gst(float2* p, float2 v) { *(LLP_G gf2*)p = gf2{v.x, v.y}; }
__device__ __forceinline__ void gst(float4* p, float4 v) { *(LLP_G gf4*)p = gf4{v.x, v.y, v.z, v.w}; }
#undef LLP_G

// Forward DFT of R points in registers: X_m = sum_t v_t e^{-2 pi i m t / R}.
template <int R>
struct Dft;

template <>
struct Dft<1> {
  static __device__ __forceinline__ void run(float2 (&)[1]) {}
};

template <>
struct Dft<2> {
  static __device__ __forceinline__ void run(float2 (&v)[2]) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <>
struct Dft<4> {
  static __device__ __forceinline__ void run(float2 (&v)[4]) {
    const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]), t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, mul_mi(t3));
    v[3] = csub(t1, mul_mi(t3));
  }
};

template <>
struct Dft<8> {
  static __device__ __forceinline__ void run(float2 (&v)[8]) {
    float2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4>::run(e);
    Dft<4>::run(o);
    constexpr float h = 0.70710678118654752f;  // cos(pi/4)
    const float2 o1 = make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));    // e^{-i pi/4} o1
    const float2 o2 = mul_mi(o[2]);                                                // e^{-i pi/2} o2
    const float2 o3 = make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));  // e^{-3 i pi/4} o3
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// 16 = 4 x 4 (Cooley-Tukey): v_{4 n1 + n2} -> four 4-point DFTs over n1, the twiddles e^{-2 pi i n2 k1 / 16},
// four 4-point DFTs over n2; output k1 + 4 k2.
template <>
struct Dft<16> {
  static __device__ __forceinline__ void rot(float2& a, float c, float s) {  // a * (c + i s)
    a = make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
  }
  static __device__ __forceinline__ void run(float2 (&v)[16]) {
    constexpr float c1 = 0.92387953251128675613f;  // cos(pi/8)
    constexpr float s1 = 0.38268343236508977173f;  // sin(pi/8)
    constexpr float h = 0.70710678118654752440f;   // cos(pi/4)
    float2 a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      float2 q[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
      Dft<4>::run(q);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) a[n2][k1] = q[k1];
    }
    rot(a[1][1], c1, -s1);  // W^1
    rot(a[1][2], h, -h);    // W^2
    rot(a[1][3], s1, -c1);  // W^3
    rot(a[2][1], h, -h);    // W^2
    a[2][2] = mul_mi(a[2][2]);  // W^4
    rot(a[2][3], -h, -h);   // W^6
    rot(a[3][1], s1, -c1);  // W^3
    rot(a[3][2], -h, -h);   // W^6
    rot(a[3][3], -c1, s1);  // W^9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 q[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      Dft<4>::run(q);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = q[k2];
    }
  }
};

// cos(pi k / 16) for 0 <= k < 32, and a * e^{-i pi m / 16} with m a compile-time constant.
__host__ __device__ constexpr float cos16(int k) {
  return k > 16 ? cos16(32 - k)
       : k > 8  ? -cos16(16 - k)
       : k == 0 ? 1.0f
       : k == 1 ? 0.98078528040323044913f
       : k == 2 ? 0.92387953251128675613f
       : k == 3 ? 0.83146961230254523708f
       : k == 4 ? 0.70710678118654752440f
       : k == 5 ? 0.55557023301960222474f
       : k == 6 ? 0.38268343236508977173f
       : k == 7 ? 0.19509032201612826785f
                : 0.0f;
}
template <int m>
__device__ __forceinline__ void twiddle32(float2& a) {
  if constexpr (m % 32 == 0) {
    return;
  } else if constexpr (m % 32 == 8) {
    a = mul_mi(a);
  } else {
    constexpr float c = cos16(m % 32), s = cos16(m % 32 <= 8 ? 8 - m % 32 : m % 32 - 8);  // sin(pi m / 16)
    a = make_float2(a.x * c + a.y * s, a.y * c - a.x * s);
  }
}
template <int N2, int... K1>
__device__ __forceinline__ void twiddle32_row(float2 (&a)[8], std::integer_sequence<int, K1...>) {
  (twiddle32<N2 * K1>(a[K1]), ...);
}

// 32 = 8 x 4 (Cooley-Tukey): v_{4 n1 + n2} -> four 8-point DFTs over n1, the twiddles e^{-2 pi i n2 k1 / 32},
// eight 4-point DFTs over n2; output k1 + 8 k2.
template <>
struct Dft<32> {
  static __device__ __forceinline__ void run(float2 (&v)[32]) {
    float2 a[4][8];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < 8; ++n1) a[n2][n1] = v[4 * n1 + n2];
      Dft<8>::run(a[n2]);
    }
    twiddle32_row<1>(a[1], std::make_integer_sequence<int, 8>{});
    twiddle32_row<2>(a[2], std::make_integer_sequence<int, 8>{});
    twiddle32_row<3>(a[3], std::make_integer_sequence<int, 8>{});
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) {
      float2 q[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      Dft<4>::run(q);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 8 * k2] = q[k2];
    }
  }
};

// Odd radices by the definition, with cos and sin of 2 pi k / R as constants.
__constant__ float kCos3[3] = {1.0f, -0.5f, -0.5f};
__constant__ float kSin3[3] = {0.0f, 0.86602540378443865f, -0.86602540378443865f};
__constant__ float kCos5[5] = {1.0f, 0.30901699437494745f, -0.80901699437494742f, -0.80901699437494742f,
                               0.30901699437494745f};
__constant__ float kSin5[5] = {0.0f, 0.95105651629515357f, 0.58778525229247313f, -0.58778525229247313f,
                               -0.95105651629515357f};
__constant__ float kCos7[7] = {1.0f, 0.62348980185873353f, -0.22252093395631440f, -0.90096886790241913f,
                               -0.90096886790241913f, -0.22252093395631440f, 0.62348980185873353f};
__constant__ float kSin7[7] = {0.0f, 0.78183148246802981f, 0.97492791218182361f, 0.43388373911755812f,
                               -0.43388373911755812f, -0.97492791218182361f, -0.78183148246802981f};

template <int R>
__device__ __forceinline__ void dft_odd(float2 (&v)[R], const float* cs, const float* sn) {
  float2 out[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    float2 acc = v[0];
#pragma unroll
    for (int t = 1; t < R; ++t) {
      const int k = (m * t) % R;  // e^{-2 pi i k / R} = cos - i sin
      acc.x += v[t].x * cs[k] + v[t].y * sn[k];
      acc.y += v[t].y * cs[k] - v[t].x * sn[k];
    }
    out[m] = acc;
  }
#pragma unroll
  for (int m = 0; m < R; ++m) v[m] = out[m];
}
template <>
struct Dft<3> {
  static __device__ __forceinline__ void run(float2 (&v)[3]) { dft_odd<3>(v, kCos3, kSin3); }
};
template <>
struct Dft<5> {
  static __device__ __forceinline__ void run(float2 (&v)[5]) { dft_odd<5>(v, kCos5, kSin5); }
};
template <>
struct Dft<7> {
  static __device__ __forceinline__ void run(float2 (&v)[7]) { dft_odd<7>(v, kCos7, kSin7); }
};

// LDS slot of element i of sequence seq: one unused slot after every 16 elements and sequences S = L + L/16 + 1
// slots apart, so that the strided accesses of the early passes (stride R Ns) and the accesses across
// sequences (stride S, odd modulo the banks for the lengths used) spread over the banks.
__host__ __device__ __forceinline__ int seq_stride(int L) { return L + (L >> 4) + 1; }
__device__ __forceinline__ int pd(int seq, int S, int i) { return __mul24(seq, S) + i + (i >> 4); }

// One Stockham pass of radix R (any of 2, 3, 4, 5, 7, 8) over nseq sequences of length L stored back to back in
// buf; Ns is the length of the sub-transforms already done.  tw: this pass's twiddles in LDS, tw[(t - 1) Ns + k]
// = e^{-2 pi i t k / (Ns R)} for k < Ns, 0 < t < R (consecutive k, read by consecutive lanes, side by side).
template <int TH, int R, int PER>
__device__ __forceinline__ void fft_pass(float2* buf, int L, int nseq, int Ns, const float2* tw) {
  constexpr int NB = (PER + R - 1) / R;  // butterflies per thread: PER values per thread at most
  const int M = L / R, total = nseq * M, S = seq_stride(L);
  float2 v[NB][R];
  int ob[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = opaque_tid() + b * TH;
    ob[b] = -1;
    if (j < total) {
      const int seq = j / M, jj = j - seq * M, k = jj % Ns;
      const int o = (jj / Ns) * Ns * R + k;
#pragma unroll
      for (int t = 0; t < R; ++t) v[b][t] = buf[pd(seq, S, jj + t * M)];
#pragma unroll
      for (int t = 1; t < R; ++t) v[b][t] = cmul(v[b][t], tw[(t - 1) * Ns + k]);
      Dft<R>::run(v[b]);
      ob[b] = (seq << 16) | o;  // sequence and element offset (L <= 16384)
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (ob[b] >= 0) {
#pragma unroll
      for (int t = 0; t < R; ++t) buf[pd(ob[b] >> 16, S, (ob[b] & 0xffff) + t * Ns)] = v[b][t];
    }
  }
  __syncthreads();
}

// The same pass for L a power of two (R = 32, 16, 8 or 4), with every LDS index an offset from one base per butterfly:
// when M = L / R is a multiple of 16 (LIN) the R inputs jj + t M sit (M + M / 16) slots apart, and the outputs
// o + t Ns always sit t Ns + (t Ns) / 16 slots from o (the padding of a block of R Ns outputs is linear in t, as
// the block starts on a multiple of min(R Ns, 16)).  TW = false for the first pass (Ns = 1: every twiddle is 1).
template <int TH, int R, int PER, bool LIN, bool TW>
__device__ __forceinline__ void fft_pass_p2(float2* gbuf, int L, int nseq, int Ns, const float2* gtw) {
  // LDS-typed pointers (32-bit index arithmetic) to plain two-float vectors
  typedef __attribute__((address_space(3))) gf2 lds_f2;
  lds_f2* buf = (lds_f2*)gbuf;
  const lds_f2* tw = (const lds_f2*)gtw;
  auto ld = [](const lds_f2* p) {
    const gf2 x = *p;
    return make_float2(x.x, x.y);
  };
  constexpr int NB = (PER + R - 1) / R;
  constexpr int LR = R == 32 ? 5 : R == 16 ? 4 : R == 8 ? 3 : 2;
  const int M = L >> LR, total = nseq * M, S = seq_stride(L);
  const int lgM = __builtin_ctz(M), lgNs = __builtin_ctz(Ns);
  const int rstep = M + (M >> 4);
  float2 v[NB][R];
  int wb[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = opaque_tid() + b * TH;
    wb[b] = -1;
    if (j < total) {
      const int seq = j >> lgM, jj = j & (M - 1), k = jj & (Ns - 1);
      const int sb = __mul24(seq, S);
      if (LIN) {
        const int rb = sb + jj + (jj >> 4);
#pragma unroll
        for (int t = 0; t < R; ++t) v[b][t] = ld(buf + rb + t * rstep);
      } else {
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int i = jj + t * M;
          v[b][t] = ld(buf + sb + i + (i >> 4));
        }
      }
      if (TW) {
        const lds_f2* twk = tw + k;
#pragma unroll
        for (int t = 1; t < R; ++t) v[b][t] = cmul(v[b][t], ld(twk + (t - 1) * Ns));
      }
      Dft<R>::run(v[b]);
      const int o = ((jj >> lgNs) << (lgNs + LR)) | k;
      wb[b] = sb + o + (o >> 4);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (wb[b] >= 0) {
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int tn = t * Ns;
        buf[wb[b] + tn + (tn >> 4)] = gf2{v[b][t].x, v[b][t].y};
      }
    }
  }
  __syncthreads();
}

template <int TH, int R, int PER>
__device__ __forceinline__ void fft_pass_p2_any(float2* buf, int L, int nseq, int Ns, const float2* tw) {
  const bool lin = (L / R) % 16 == 0;
  if (Ns == 1) {
    if (lin) fft_pass_p2<TH, R, PER, true, false>(buf, L, nseq, Ns, tw);
    else fft_pass_p2<TH, R, PER, false, false>(buf, L, nseq, Ns, tw);
  } else {
    if (lin) fft_pass_p2<TH, R, PER, true, true>(buf, L, nseq, Ns, tw);
    else fft_pass_p2<TH, R, PER, false, true>(buf, L, nseq, Ns, tw);
  }
}

// Forward DFT of nseq sequences of length L in LDS (radices rad[0..nrad), product L; tw: the pass-major
// twiddle table of the transform in LDS, see pass_twiddles).
// TH threads, at most ELEMS values.  MIXED = false: radices 8 and 4 only (L a power of two), up to ELEMS / TH
// values per thread, and with WIDE radix 16 too and radix 32 in workgroups that hold kPcMaxElems values (the
// plan of pc_wide_radices; the small-row workgroups keep their register budget); MIXED = true: every radix,
// up to min(ELEMS, kPcSmallElems) / TH values per thread (short transforms only, see pc_supported).  Splitting
// them keeps every pass within the register budget.
template <int TH, bool MIXED, int ELEMS = kPcMaxElems, bool WIDE = false>
__device__ __forceinline__ void fft_lds(float2* buf, int L, int nseq, const int* rad, int nrad, const float2* tw) {
  constexpr int PER = (MIXED ? (ELEMS < kPcSmallElems ? ELEMS : kPcSmallElems) : ELEMS) / TH;
  int Ns = 1, off = 0;
  for (int p = 0; p < nrad; ++p) {
    const int R = rad[p];
    if (MIXED) {
      switch (R) {
        case 8: fft_pass<TH, 8, PER>(buf, L, nseq, Ns, tw + off); break;
        case 4: fft_pass<TH, 4, PER>(buf, L, nseq, Ns, tw + off); break;
        case 2: fft_pass<TH, 2, PER>(buf, L, nseq, Ns, tw + off); break;
        case 3: fft_pass<TH, 3, PER>(buf, L, nseq, Ns, tw + off); break;
        case 5: fft_pass<TH, 5, PER>(buf, L, nseq, Ns, tw + off); break;
        default: fft_pass<TH, 7, PER>(buf, L, nseq, Ns, tw + off); break;
      }
    } else if (WIDE && R == 32) {
      if constexpr (WIDE && PER * TH >= kPcMaxElems) fft_pass_p2_any<TH, 32, PER>(buf, L, nseq, Ns, tw + off);
    } else if (WIDE && R == 16) {
      fft_pass_p2_any<TH, 16, PER>(buf, L, nseq, Ns, tw + off);
    } else if (R == 8) {
      fft_pass_p2_any<TH, 8, PER>(buf, L, nseq, Ns, tw + off);
    } else {
      fft_pass_p2_any<TH, 4, PER>(buf, L, nseq, Ns, tw + off);
    }
    off += Ns * (R - 1);
    Ns *= R;
  }
}

// Element e < n (n >= 1) goes from src(e) to dst(e, value) for every e, with K loads per thread issued before
// the first of their stores: a global-to-LDS copy keeps K loads in flight instead of waiting on each one.  The
// loads are unconditional (indexes past the end read element n - 1 again), so no branch separates them.
template <int TH, int K, typename Src, typename Dst>
__device__ __forceinline__ void copy_elems(int n, Src src, Dst dst) {
  for (int base = 0; base < n; base += TH * K) {
    float2 v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = src(min(base + k * TH + opaque_tid(), n - 1));
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int e = base + k * TH + opaque_tid();
      if (e < n) dst(e, v[k]);
    }
  }
}

// The twiddle table of a length-L transform, copied from global memory into LDS after the c^2 sequences.
template <int TH>
__device__ __forceinline__ float2* stage_twiddles(float2* pcsh, int nseq, int L, const float2* tw) {
  float2* t = pcsh + (size_t)nseq * seq_stride(L);
  copy_elems<TH, 4>(L, [&](int i) { return gld(tw + i); }, [&](int i, float2 v) { t[i] = v; });
  return t;
}

template <typename F>
__device__ __forceinline__ int find_pc(const PcDesc* t, int count, int bid, F first) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first(t[mid]) <= bid) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Solve (diag(d) + conj(U) U^T / c^2) x = F on one group of N = c^2 members, in place (F becomes x), with
// d_{s c + t} = dscale (eh[s] + ew[t])^2: eh, ew the symbols 2 - 2 cos of the stencil along each axis at the
// member's frequencies.  The member with the smallest d is eliminated through the rank-one equation when the
// rank-one term dominates its row (the frequency nearest 0, where d is tiny or, at K = 0, zero): there the
// Sherman-Morrison form would cancel catastrophically.  Every array index is a compile-time constant (the
// pivot is selected, never indexed).  Reciprocals are the hardware's (1 ulp); d = 0 occurs only at the pivot
// member, whose reciprocal is unused.
template <int C>
__device__ __forceinline__ void group_solve(float2 (&F)[C * C], const float2 (&U)[C * C], const float (&eh)[C],
                                            const float (&ew)[C], float dscale) {
  constexpr int N = C * C;
  const float c2 = (float)N;
  // d_j and its reciprocal are recomputed where needed rather than held (register pressure)
  auto dof = [&](int j) {
    const float sym = eh[j / C] + ew[j % C];
    return dscale * sym * sym;
  };
  int js = 0;
  float dmin = 0.0f;
  float2 Uj = U[0];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const float dj = dof(j);
    if (j == 0 || dj < dmin) {
      dmin = dj;
      js = j;
      Uj = U[j];
    }
  }
  const float u2 = Uj.x * Uj.x + Uj.y * Uj.y;
  const bool pivot = dmin * c2 < u2;
  // S = U^T x / c^2 from the normal equation, scaled by dmin in the pivot case
  float2 num = make_float2(0.0f, 0.0f);
  float den = pivot ? c2 * dmin : c2;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const float rk = __builtin_amdgcn_rcpf(dof(k));
    const float wk = pivot ? (k == js ? 1.0f : dmin * rk) : rk;
    num = cadd(num, make_float2(wk * (U[k].x * F[k].x - U[k].y * F[k].y), wk * (U[k].x * F[k].y + U[k].y * F[k].x)));
    den += wk * (U[k].x * U[k].x + U[k].y * U[k].y);
  }
  const float rden = __builtin_amdgcn_rcpf(den);
  const float2 S = make_float2(num.x * rden, num.y * rden);
  // x_j = (F_j - conj(U_j) S) / d_j; in the pivot case x_js instead from c^2 S = sum_j U_j x_j
  float2 rest = make_float2(0.0f, 0.0f);
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const bool piv = pivot && j == js;
    const float rj = piv ? 1.0f : __builtin_amdgcn_rcpf(dof(j));
    const float2 t = csub(F[j], cmul(conjf2(U[j]), S));
    F[j] = make_float2(t.x * rj, t.y * rj);
    if (!piv) rest = cadd(rest, cmul(U[j], F[j]));
  }
  if (pivot) {
    const float2 t = csub(make_float2(c2 * S.x, c2 * S.y), rest);  // U_js x_js
    const float ru2 = __builtin_amdgcn_rcpf(u2);
    const float2 xs = make_float2((t.x * Uj.x + t.y * Uj.y) * ru2, (t.y * Uj.x - t.x * Uj.y) * ru2);
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (j == js) F[j] = xs;
  }
}

// A value that is the same in every lane, moved to a scalar register.
__device__ __forceinline__ float uniform(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}

// 2D DFT of a C x C block in registers (A[al C + be]): A[s C + t] <- sum_{al, be} A[al C + be] w_c^{al s + be t}.
template <int C>
__device__ __forceinline__ void dft2(float2 (&A)[C * C]) {
#pragma unroll
  for (int al = 0; al < C; ++al) {
    float2 v[C];
#pragma unroll
    for (int be = 0; be < C; ++be) v[be] = A[al * C + be];
    Dft<C>::run(v);
#pragma unroll
    for (int t = 0; t < C; ++t) A[al * C + t] = v[t];
  }
#pragma unroll
  for (int t = 0; t < C; ++t) {
    float2 v[C];
#pragma unroll
    for (int al = 0; al < C; ++al) v[al] = A[al * C + t];
    Dft<C>::run(v);
#pragma unroll
    for (int s = 0; s < C; ++s) A[s * C + t] = v[s];
  }
}

// The per-cell work of the column pass for LR frequency (k1, k2): twiddle, C x C DFT to the group's c^2
// frequencies, the group operation (store U, apply the data term, or solve with P), inverse C x C DFT (1/C^2),
// conjugate twiddle; the result is left conjugated in LDS for the inverse column transforms.  The twiddle
// e^{-2 pi i (al k1 / H + be k2 / W)} is applied as its two factors.
template <int C>
__device__ __forceinline__ void cell_op(int op, const PcDesc& d, float2* pcsh, int h, int k1, int k2, float dscale) {
  constexpr int N = C * C;
  const int w = d.g.w, Sh = seq_stride(h);
  float2 ta[C], tb[C];  // tb (k2 is the workgroup's) is kept in scalar registers
#pragma unroll
  for (int a = 0; a < C; ++a) {
    ta[a] = gld(d.twH + a * k1);
    const float2 t = gld(d.twW + a * k2);
    tb[a] = make_float2(uniform(t.x), uniform(t.y));
  }
  float2 A[N];
#pragma unroll
  for (int al = 0; al < C; ++al)
#pragma unroll
    for (int be = 0; be < C; ++be) A[al * C + be] = cmul(cmul(pcsh[pd(al * C + be, Sh, k1)], ta[al]), tb[be]);
  dft2<C>(A);
  float2* uc = d.uhat + ((size_t)k1 * w + k2) * N;
  if (op == kPcColsKernel) {
#pragma unroll
    for (int j = 0; j < N; ++j) gst(uc + j, A[j]);
    return;
  }
  float2 U[N];
#pragma unroll
  for (int j = 0; j < N; ++j) U[j] = gld(uc + j);
  if (op == kPcColsData) {  // B^T D^T D B in the Fourier domain: conj(U_j) / c^2 * sum_k U_k F_k
    float2 S = make_float2(0.0f, 0.0f);
#pragma unroll
    for (int k = 0; k < N; ++k) S = cadd(S, cmul(U[k], A[k]));
    S = make_float2(S.x / (float)N, S.y / (float)N);
#pragma unroll
    for (int j = 0; j < N; ++j) A[j] = cmul(conjf2(U[j]), S);
  } else {
    float eh[C], ew[C];
#pragma unroll
    for (int s = 0; s < C; ++s) {
      eh[s] = 2.0f - 2.0f * gld(d.twH + k1 + s * h).x;
      ew[s] = uniform(2.0f - 2.0f * gld(d.twW + k2 + s * w).x);
    }
    group_solve<C>(A, U, eh, ew, dscale);
  }
  // inverse C x C DFT by conjugation: A = conj(sum_{s,t} X w^{-(al s + be t)}); the value wanted is
  // conj(A)/N * conj(tw), and it is stored conjugated: A tw / N
#pragma unroll
  for (int j = 0; j < N; ++j) A[j] = conjf2(A[j]);
  dft2<C>(A);
  const float inv = 1.0f / (float)N;
#pragma unroll
  for (int al = 0; al < C; ++al)
#pragma unroll
    for (int be = 0; be < C; ++be) {
      const float2 v = cmul(cmul(A[al * C + be], ta[al]), tb[be]);
      pcsh[pd(al * C + be, Sh, k1)] = make_float2(v.x * inv, v.y * inv);
    }
}

__device__ __forceinline__ bool band_runs(const ChanState* st, int band, int nbands) {
  return band < nbands && st[band].active;
}

}  // namespace

// C consecutive floats of a plane (16-byte aligned for C = 4, 8-byte for C = 2).
template <int C>
__device__ __forceinline__ void ldc(const float* p, float (&v)[C]) {
  if constexpr (C == 4) {
    const float4 t = gld((const float4*)p);
    v[0] = t.x, v[1] = t.y, v[2] = t.z, v[3] = t.w;
  } else if constexpr (C == 2) {
    const float2 t = gld((const float2*)p);
    v[0] = t.x, v[1] = t.y;
  } else {
#pragma unroll
    for (int k = 0; k < C; ++k) v[k] = gld(p + k);
  }
}
template <int C>
__device__ __forceinline__ void stc(float* p, const float (&v)[C]) {
  if constexpr (C == 4) {
    gst((float4*)p, make_float4(v[0], v[1], v[2], v[3]));
  } else if constexpr (C == 2) {
    gst((float2*)p, make_float2(v[0], v[1]));
  } else {
#pragma unroll
    for (int k = 0; k < C; ++k) gst(p + k, v[k]);
  }
}
// ------------------------------------------------------------------------------------------- row pass ---
// op kPcRowsStart: the bands' residual r[prev] as it is; kPcRowsUpdate: r[cur] = r[prev] - alpha q first (the
// residual update of iteration k; the iterate's update z += alpha p is done by the direction kernel, which reads
// p anyway); kPcRowsKernel: the blur kernel embedded in an H x W
// plane with its centre tap at (0, 0), in band a of pair 0.  Partial sums of |r|^2 per band go to slot 0 of
// the band's partials (one per LR row).  Each thread moves whole cells: the C x C pixels (c m + al, c n + be)
// of LR pixel (m, n) on the way in, the c^2 spectral values of frequency (m, k2) on the way out.

template <int C, bool MIXED, int TH>
__device__ __forceinline__ void rows_fwd(int op, const PcDesc& d, const ChanState* sst, int pair, int m, int prev,
                                         int cur, float2* pcsh, double* red) {
  constexpr int C2 = C * C;
  const Geom& g = d.g;
  const int W = g.W, w = g.w;
  const int ba = 2 * pair, bb = 2 * pair + 1;
  const bool ra = op != kPcRowsKernel && band_runs(sst, ba, g.N);
  const bool rb = op != kPcRowsKernel && band_runs(sst, bb, g.N);
  const float al_a = ra ? (float)sst[ba].alpha : 0.0f, al_b = rb ? (float)sst[bb].alpha : 0.0f;
  const size_t HW = (size_t)g.H * W;
  const int Sw = seq_stride(w);
  double acc_a = 0.0, acc_b = 0.0;
  for (int n = threadIdx.x; n < w; n += TH) {
#pragma unroll
    for (int al = 0; al < C; ++al) {
      const int i = C * m + al;
      const size_t e = (size_t)i * W + (size_t)C * n;
      float va[C], vb[C];
#pragma unroll
      for (int be = 0; be < C; ++be) va[be] = vb[be] = 0.0f;
      if (op == kPcRowsKernel) {
#pragma unroll
        for (int be = 0; be < C; ++be) {
          // plane (i, j) holds u[(i + R) mod H][(j + R) mod W] where that is inside the kernel
          int a = i + g.R, b = C * n + be + g.R;
          if (a >= g.H) a -= g.H;
          if (b >= W) b -= W;
          if (a < g.n && b < g.n) va[be] = gld(d.u + a * g.n + b);
        }
      } else {
#pragma unroll
        for (int band = 0; band < 2; ++band) {
          if (!(band == 0 ? ra : rb)) continue;
          const size_t o = (size_t)(band == 0 ? ba : bb) * HW + e;
          const float al = band == 0 ? al_a : al_b;
          float rv[C];
          ldc<C>(d.r[prev] + o, rv);
          if (op == kPcRowsUpdate) {
            float qv[C];
            ldc<C>(d.q + o, qv);
#pragma unroll
            for (int k = 0; k < C; ++k) rv[k] = fmaf(-al, qv[k], rv[k]);
            stc<C>(d.r[cur] + o, rv);
          }
          double ss = 0.0;
#pragma unroll
          for (int k = 0; k < C; ++k) ss += (double)rv[k] * rv[k];
          if (band == 0) acc_a += ss;
          else acc_b += ss;
#pragma unroll
          for (int k = 0; k < C; ++k) (band == 0 ? va : vb)[k] = rv[k];
        }
      }
#pragma unroll
      for (int be = 0; be < C; ++be) pcsh[pd(al * C + be, Sw, n)] = make_float2(va[be], vb[be]);
    }
  }
  const float2* twl = stage_twiddles<TH>(pcsh, C2, w, d.tww);
  __syncthreads();
  fft_lds<TH, MIXED, row_elems(TH), !MIXED>(pcsh, w, C2, d.rw, d.nrw, twl);
  float2* out = d.spec + ((size_t)pair * g.h + m) * (size_t)w * C2;
  // consecutive threads: consecutive values of a cell row
  copy_elems<TH, 8>(
      w * C2, [&](int e) { return pcsh[pd(e % C2, Sw, e / C2)]; }, [&](int e, float2 v) { gst(out + e, v); });
  if (op == kPcRowsKernel) return;
  double v[2] = {acc_a, acc_b};
  block_sums<2, TH / 64>(v, red);
  if (threadIdx.x == 0) {
    if (ra) gst(d.partials + (size_t)ba * d.pstride * 3 + (size_t)m * 3 + 0, v[0]);
    if (rb) gst(d.partials + (size_t)bb * d.pstride * 3 + (size_t)m * 3 + 0, v[1]);
  }
}

template <bool MIXED, int TH>
__device__ __forceinline__ void rows_fwd_c(int op, const PcDesc& d, const ChanState* sst, int pair, int m, int prev,
                                           int cur, float2* pcsh, double* red) {
  switch (d.g.c) {
    case 4: rows_fwd<4, MIXED, TH>(op, d, sst, pair, m, prev, cur, pcsh, red); break;
    case 3: rows_fwd<3, MIXED, TH>(op, d, sst, pair, m, prev, cur, pcsh, red); break;
    case 2: rows_fwd<2, MIXED, TH>(op, d, sst, pair, m, prev, cur, pcsh, red); break;
    default: rows_fwd<1, MIXED, TH>(op, d, sst, pair, m, prev, cur, pcsh, red); break;
  }
}

template <bool MIXED, int TH>
__global__ __launch_bounds__(TH) void k_pc_rows(int op, const PcDesc* __restrict__ t, int count,
                                               const ChanState* __restrict__ st, int prev, int cur) {
  extern __shared__ float2 pcsh[];
  __shared__ double red[2 * (TH / 64)];
  const int si = find_pc(t, count, (int)blockIdx.x, [](const PcDesc& d) { return d.row_block0; });
  const PcDesc& d = t[si];
  const Geom& g = d.g;
  const int local = (int)blockIdx.x - d.row_block0;
  const int npair = op == kPcRowsKernel ? 1 : d.npair;
  if (local >= npair * g.h) return;
  const int pair = local / g.h, m = local - pair * g.h;
  const ChanState* sst = st + d.band0;
  if (op != kPcRowsKernel && !band_runs(sst, 2 * pair, g.N) && !band_runs(sst, 2 * pair + 1, g.N)) return;
  // a launch for tables with mixed-radix lengths still runs the power-of-two passes on the scenes that allow them
  if (MIXED && d.mixed_w) rows_fwd_c<true, TH>(op, d, sst, pair, m, prev, cur, pcsh, red);
  else rows_fwd_c<false, TH>(op, d, sst, pair, m, prev, cur, pcsh, red);
}

// ---------------------------------------------------------------------------------------- column pass ---
// op kPcColsSolve: forward length-h transforms, the group solve of every cell, inverse transforms (unscaled;
// the inverse c x c DFT carries 1/c^2).  op kPcColsData: the same with the data term B^T D^T D B applied to
// every group instead of P^{-1}.  op kPcColsKernel: forward transforms and the c x c DFT of pair 0 (the
// embedded kernel), stored as U in the cell layout.  Each thread moves whole cells.
//
// Persistent workgroups, as many per compute unit as the LDS holds: workgroup b owns every G-th LR column of the
// table and transforms the running band pairs of a column together, as many as the launch's element budget
// allows (short columns), so that U of the column is reused from the L2 cache.  The next group's columns are
// loaded into registers while the current group is transformed.

constexpr size_t kPcCuLds = 160 * 1024;    // LDS of a compute unit
constexpr int kColPf = kPcMaxElems / TC;  // complex values per thread of one item's column

// Items of one column processed together: up to kColGroup band pairs of one LR column, as many as fit in the
// element budget of the launch (short columns would otherwise leave most of the workgroup idle in the cell
// operations and the transforms).
constexpr int kColGroup = 8;

__host__ __device__ __forceinline__ int col_group_max(const PcDesc& d, int budget) {
  if (d.mixed_h && budget > kPcSmallElems) budget = kPcSmallElems;  // the mixed-radix passes' register budget
  const int per = d.g.h * d.g.c * d.g.c;
  int k = budget / per;
  k = k < 1 ? 1 : k;
  k = k > kColGroup ? kColGroup : k;
  return k > d.npair ? d.npair : k;
}

// Issue the loads of the columns (h cells of C^2 values each) of the pairs gp[0..cnt), LR column k2, into
// registers: element E of the group is item E / (h C^2), element E % (h C^2) of that item's column.
// E / per for E < kPcMaxElems by a float product (the quotient is below 8 and its fraction at least 1/(2 per)
// away from an integer, far beyond the product's rounding).
__device__ __forceinline__ int item_of(int E, float inv_per) { return __float2int_rz(((float)E + 0.5f) * inv_per); }

// GR: groups of several pairs; otherwise one pair (gp[0]) and no item split.
template <int C, bool GR>
__device__ __forceinline__ void col_prefetch(const PcDesc& d, const int* gp, int cnt, int k2, float2 (&pf)[kColPf]) {
  constexpr int C2 = C * C;
  const int per = d.g.h * C2, n = cnt * per, w = d.g.w;
  const float inv_per = 1.0f / (float)per;
  const size_t pstride = (size_t)d.g.h * w * C2;
  const float2* sp0 = d.spec + (GR ? 0 : gp[0] * pstride) + (size_t)k2 * C2;
#pragma unroll
  for (int k = 0; k < kColPf; ++k) {
    if (k * TC < n) {  // uniform
      const int E = min(k * TC + opaque_tid(), n - 1);
      const int it = GR ? item_of(E, inv_per) : 0, e = E - it * per;
      pf[k] = gld(sp0 + (GR ? gp[it] * pstride : 0) + (size_t)(e / C2) * w * C2 + e % C2);
    }
  }
}

// The prefetched columns into the LDS sequences: item it's sequences are it C^2 .. it C^2 + C^2 - 1.
template <int C, bool GR>
__device__ __forceinline__ void col_stage(const PcDesc& d, int cnt, const float2 (&pf)[kColPf], float2* pcsh) {
  constexpr int C2 = C * C;
  const int per = d.g.h * C2, n = cnt * per, Sh = seq_stride(d.g.h);
  const float inv_per = 1.0f / (float)per;
#pragma unroll
  for (int k = 0; k < kColPf; ++k) {
    const int E = k * TC + opaque_tid();
    if (k * TC < n && E < n) {
      const int it = GR ? item_of(E, inv_per) : 0, e = E - it * per;
      pcsh[pd(it * C2 + e % C2, Sh, e / C2)] = pf[k];
    }
  }
}

// Transforms, cell operations and the store of one group whose columns are in LDS (twl: the length-h twiddles).
template <int C, bool MIXED, bool GR>
__device__ __forceinline__ void cols_body(int op, const PcDesc& d, const int* gp, int cnt, int k2, float2* pcsh,
                                          const float2* twl) {
  constexpr int C2 = C * C;
  const Geom& g = d.g;
  const int h = g.h, w = g.w;
  const int Sh = seq_stride(h);
  // forward transforms, the cell operations, inverse transforms: one copy of the transform code for both
#pragma unroll 1
  for (int pass = 0;; ++pass) {
    fft_lds<TC, MIXED, kPcMaxElems, !MIXED>(pcsh, h, cnt * C2, d.rh, d.nrh, twl);
    if (pass == 1) break;
    const float dscale = op == kPcColsSolve ? (float)((double)g.lam * d.mbar[0]) : 0.0f;
#pragma unroll 1
    for (int idx = opaque_tid(); idx < cnt * h; idx += TC) {
      const int it = GR ? idx / h : 0, k1 = idx - it * h;
      cell_op<C>(op, d, pcsh + (size_t)it * C2 * Sh, h, k1, k2, dscale);
    }
    if (op == kPcColsKernel) return;
    __syncthreads();
  }
  const int per = h * C2;
  const float inv_per = 1.0f / (float)per;
  const size_t pstride = (size_t)h * w * C2;
  float2* sp0 = d.spec + (GR ? 0 : gp[0] * pstride) + (size_t)k2 * C2;
  copy_elems<TC, 8>(
      cnt * per,
      [&](int E) {
        const int it = GR ? item_of(E, inv_per) : 0, e = E - it * per;
        return conjf2(pcsh[pd(it * C2 + e % C2, Sh, e / C2)]);
      },
      [&](int E, float2 v) {
        const int it = GR ? item_of(E, inv_per) : 0, e = E - it * per;
        gst(sp0 + (GR ? gp[it] * pstride : 0) + (size_t)(e / C2) * w * C2 + e % C2, v);
      });
}

// The items of one scene that this workgroup owns: the LR columns k2 = k0, k0 + G, k0 + 2G, ... (G workgroups)
// and, per column, its band pairs with a running band, taken kmax at a time (U of the column is reused from L2
// by every pair).  The next group's columns are in flight while the current group is transformed.
template <int C, bool MIXED, bool GR>
__device__ __forceinline__ void cols_scene(int op, const PcDesc& d, const ChanState* sst, int k0, int G,
                                           float2* pcsh, int kmax, int* gsh) {
  const int np = d.npair;
  const int hi = (d.g.w - k0 + G - 1) / G * np;  // items: l = j np + pair for the j-th owned column
  auto runs = [&](int l) {
    const int pair = l % np;
    return op == kPcColsKernel ? pair == 0
                               : band_runs(sst, 2 * pair, d.g.N) || band_runs(sst, 2 * pair + 1, d.g.N);
  };
  auto next = [&](int l) {
    for (; l < hi; ++l)
      if (runs(l)) break;
    return l;
  };
  // the group starting at running item l: running items of l's column, at most kmax, their pairs into gp (every
  // thread writes the same values); returns the item after the group
  auto group = [&](int l, int* gp, int& cnt) {
    const int j = l / np;
    cnt = 0;
    for (; l < hi && l / np == j && cnt < kmax; l = next(l + 1)) gp[cnt++] = l % np;
    return l;
  };
  auto col_of = [&](int l) { return k0 + (l / np) * G; };
  int l = next(0);
  if (l >= hi) return;
  int* gp = gsh;
  int* gpn = gsh + kColGroup;
  int cnt = 0, cntn = 0;
  __syncthreads();  // the group buffers of a previous scene are no longer read
  int nx = group(l, gp, cnt);
  float2 pf[kColPf];
  col_prefetch<C, GR>(d, gp, cnt, col_of(l), pf);
  __syncthreads();  // the LDS of a previous scene is no longer read
  const float2* twl = stage_twiddles<TC>(pcsh, kmax * C * C, d.g.h, d.twh);
  while (l < hi) {
    col_stage<C, GR>(d, cnt, pf, pcsh);
    int nnx = hi;
    if (nx < hi) {
      nnx = group(nx, gpn, cntn);
      col_prefetch<C, GR>(d, gpn, cntn, col_of(nx), pf);
    }
    __syncthreads();
    cols_body<C, MIXED, GR>(op, d, gp, cnt, col_of(l), pcsh, twl);
    __syncthreads();  // the LDS reads of this group are done
    l = nx;
    nx = nnx;
    cnt = cntn;
    int* t = gp;  // the prefetched group becomes the current one
    gp = gpn;
    gpn = t;
  }
}

template <bool MIXED>
__device__ __forceinline__ void cols_scene_c(int op, const PcDesc& d, const ChanState* sst, int k0, int G,
                                             float2* pcsh, int budget, int* gsh) {
  const int kmax = op == kPcColsKernel ? 1 : col_group_max(d, budget);
  if (kmax > 1) {
    switch (d.g.c) {
      case 4: cols_scene<4, MIXED, true>(op, d, sst, k0, G, pcsh, kmax, gsh); break;
      case 3: cols_scene<3, MIXED, true>(op, d, sst, k0, G, pcsh, kmax, gsh); break;
      case 2: cols_scene<2, MIXED, true>(op, d, sst, k0, G, pcsh, kmax, gsh); break;
      default: cols_scene<1, MIXED, true>(op, d, sst, k0, G, pcsh, kmax, gsh); break;
    }
  } else {
    switch (d.g.c) {
      case 4: cols_scene<4, MIXED, false>(op, d, sst, k0, G, pcsh, 1, gsh); break;
      case 3: cols_scene<3, MIXED, false>(op, d, sst, k0, G, pcsh, 1, gsh); break;
      case 2: cols_scene<2, MIXED, false>(op, d, sst, k0, G, pcsh, 1, gsh); break;
      default: cols_scene<1, MIXED, false>(op, d, sst, k0, G, pcsh, 1, gsh); break;
    }
  }
}

// Persistent: workgroup b owns the columns b, b + G, b + 2G, ... of the table's columns (every scene's LR
// columns one after another), so the scenes that still have running bands are spread over all workgroups.
template <bool MIXED>
__global__ __launch_bounds__(TC) void k_pc_cols(int op, const PcDesc* __restrict__ t, int count,
                                               const ChanState* __restrict__ st, int budget) {
  extern __shared__ float2 pcsh[];
  __shared__ int gsh[2 * kColGroup];  // the band pairs of the current and the prefetched group
  const int G = (int)gridDim.x, b = (int)blockIdx.x;
  for (int si = 0; si < count; ++si) {
    const PcDesc& d = t[si];
    const int k0 = ((b - d.col_block0) % G + G) % G;  // first owned column of the scene
    if (k0 >= d.g.w) continue;
    const ChanState* sst = st + d.band0;
    if (MIXED && d.mixed_h) cols_scene_c<true>(op, d, sst, k0, G, pcsh, budget, gsh);
    else cols_scene_c<false>(op, d, sst, k0, G, pcsh, budget, gsh);
  }
}

// ------------------------------------------------------------------------------------ inverse row pass ---
// s = P^{-1} r for both bands of a pair (inverse length-w transforms, scale 1/(h w)), and the partial sums of
// r[cur]^T s per band into slot 1 of the band's partials.

template <int C, bool MIXED, int TH>
__device__ __forceinline__ void rows_inv(const PcDesc& d, const ChanState* sst, int pair, int m, int cur,
                                         float2* pcsh, double* red) {
  constexpr int C2 = C * C;
  const Geom& g = d.g;
  const int W = g.W, w = g.w;
  const int ba = 2 * pair, bb = 2 * pair + 1;
  const bool ra = band_runs(sst, ba, g.N), rb = band_runs(sst, bb, g.N);
  const float2* in = d.spec + ((size_t)pair * g.h + m) * (size_t)w * C2;
  const int Sw = seq_stride(w);
  copy_elems<TH, 16>(
      w * C2, [&](int e) { return conjf2(gld(in + e)); }, [&](int e, float2 v) { pcsh[pd(e % C2, Sw, e / C2)] = v; });
  const float2* twl = stage_twiddles<TH>(pcsh, C2, w, d.tww);
  __syncthreads();
  fft_lds<TH, MIXED, row_elems(TH), !MIXED>(pcsh, w, C2, d.rw, d.nrw, twl);
  const float scale = 1.0f / ((float)g.h * (float)w);
  const size_t HW = (size_t)g.H * W;
  double acc_a = 0.0, acc_b = 0.0;
  for (int n = threadIdx.x; n < w; n += TH) {
#pragma unroll
    for (int al = 0; al < C; ++al) {
      const size_t e = (size_t)(C * m + al) * W + (size_t)C * n;
      float sa[C], sb[C];
#pragma unroll
      for (int be = 0; be < C; ++be) {
        const float2 v = pcsh[pd(al * C + be, Sw, n)];
        sa[be] = v.x * scale;
        sb[be] = -v.y * scale;
      }
      if (ra) {
        const size_t o = (size_t)ba * HW + e;
        float rv[C];
        ldc<C>(d.r[cur] + o, rv);
        stc<C>(d.s + o, sa);
#pragma unroll
        for (int k = 0; k < C; ++k) acc_a += (double)rv[k] * sa[k];
      }
      if (rb) {
        const size_t o = (size_t)bb * HW + e;
        float rv[C];
        ldc<C>(d.r[cur] + o, rv);
        stc<C>(d.s + o, sb);
#pragma unroll
        for (int k = 0; k < C; ++k) acc_b += (double)rv[k] * sb[k];
      }
    }
  }
  double v[2] = {acc_a, acc_b};
  block_sums<2, TH / 64>(v, red);
  if (threadIdx.x == 0) {
    if (ra) gst(d.partials + (size_t)ba * d.pstride * 3 + (size_t)m * 3 + 1, v[0]);
    if (rb) gst(d.partials + (size_t)bb * d.pstride * 3 + (size_t)m * 3 + 1, v[1]);
  }
}

template <bool MIXED, int TH>
__device__ __forceinline__ void rows_inv_c(const PcDesc& d, const ChanState* sst, int pair, int m, int cur,
                                           float2* pcsh, double* red) {
  switch (d.g.c) {
    case 4: rows_inv<4, MIXED, TH>(d, sst, pair, m, cur, pcsh, red); break;
    case 3: rows_inv<3, MIXED, TH>(d, sst, pair, m, cur, pcsh, red); break;
    case 2: rows_inv<2, MIXED, TH>(d, sst, pair, m, cur, pcsh, red); break;
    default: rows_inv<1, MIXED, TH>(d, sst, pair, m, cur, pcsh, red); break;
  }
}

template <bool MIXED, int TH>
__global__ __launch_bounds__(TH) void k_pc_rows_inv(const PcDesc* __restrict__ t, int count,
                                                   const ChanState* __restrict__ st, int cur) {
  extern __shared__ float2 pcsh[];
  __shared__ double red[2 * (TH / 64)];
  const int si = find_pc(t, count, (int)blockIdx.x, [](const PcDesc& d) { return d.row_block0; });
  const PcDesc& d = t[si];
  const Geom& g = d.g;
  const int local = (int)blockIdx.x - d.row_block0;
  if (local >= d.npair * g.h) return;
  const int pair = local / g.h, m = local - pair * g.h;
  const ChanState* sst = st + d.band0;
  if (!band_runs(sst, 2 * pair, g.N) && !band_runs(sst, 2 * pair + 1, g.N)) return;
  if (MIXED && d.mixed_w) rows_inv_c<true, TH>(d, sst, pair, m, cur, pcsh, red);
  else rows_inv_c<false, TH>(d, sst, pair, m, cur, pcsh, red);
}

// --------------------------------------------------------------------------------------------- mbar ---
// mbar = mean of diag(M_LY).  Summing eq. (matting_matrix)'s diagonal over all pixels window by window gives
// sum_k (|w| - 1 - var_k dinv_k), and var_k dinv_k = 1 - (eps/|w|) dinv_k where dinv_k != 0 (0 otherwise):
// mbar = |w| - 1 - mean_k(var_k dinv_k), one reduction over the dinv plane.

__global__ __launch_bounds__(kBlock) void k_pc_mbar(const PcDesc* __restrict__ t, double* __restrict__ part) {
  __shared__ double red[kWaves];
  const PcDesc& d = t[blockIdx.y];
  const Geom& g = d.g;
  const size_t HW = (size_t)g.H * g.W;
  const double epsw = (double)g.eps / (double)((2 * g.r + 1) * (2 * g.r + 1));
  const float* di = d.DI;
  double acc = 0.0;
  for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < HW; e += (size_t)gridDim.x * kBlock) {
    const double v = di[e];
    acc += v != 0.0 ? 1.0 - epsw * v : 0.0;
  }
  double v[1] = {acc};
  block_partials<1>(v, red, part + (size_t)blockIdx.y * gridDim.x + blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_pc_mbar_fin(const PcDesc* __restrict__ t, int nblk,
                                                        const double* __restrict__ part) {
  __shared__ double red[kWaves];
  const PcDesc& d = t[blockIdx.x];
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kBlock) s += part[(size_t)blockIdx.x * nblk + i];
  double v[1] = {s};
  block_sums<1>(v, red);
  if (threadIdx.x == 0) {
    const Geom& g = d.g;
    const double nw = (double)((2 * g.r + 1) * (2 * g.r + 1));
    d.mbar[0] = nw - 1.0 - v[0] / ((double)g.H * (double)g.W);
  }
}

// -------------------------------------------------------------------------------- polish (Z step) helpers ---
// out = a + sb * b over n floats.
__global__ __launch_bounds__(kBlock) void k_pc_axpy(const float* __restrict__ a, const float* __restrict__ b,
                                                    float* __restrict__ out, float sb, size_t n) {
  for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock)
    out[e] = fmaf(sb, b[e], a[e]);
}

// Sets the scalar weight of the Fourier solve of every scene (mbar in P = B^T D^T D B + lambda mbar L^T L).
__global__ void k_pc_set_mbar(const PcDesc* __restrict__ t, int count, double v) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) t[i].mbar[0] = v;
}

// ------------------------------------------------------------------------------------------------ host ---

int pc_radices(int L, int* rad) {
  // the power of two 2^a as radix-8 passes plus at most two radix-4 passes (radix 2 only for a = 1)
  int a = 0;
  while (L % 2 == 0) {
    L /= 2;
    ++a;
  }
  int n = 0;
  const int e8 = a % 3 == 1 && a >= 4 ? a / 3 - 1 : a / 3;
  for (int i = 0; i < e8; ++i) rad[n++] = 8;
  int rest = a - 3 * e8;  // 0, 1, 2 or 4
  while (rest >= 2) {
    rad[n++] = 4;
    rest -= 2;
  }
  if (rest == 1) rad[n++] = 2;
  for (int r : {7, 5, 3})
    while (L % r == 0 && n < kPcMaxRad) {
      rad[n++] = r;
      L /= r;
    }
  return L == 1 ? n : -1;
}

// The plan of the transform passes (rows: col = false, columns: col = true): for a power of two 2^a, a >= 6,
// radix-16 passes (a / 4 of them) and one pass of 4 or 8 for the rest (a = 4k + 1: 16^(k-1) 8 4), fewer LDS
// passes and barriers than radix 8; with allow32 and a >= 9 radix-32 passes (a / 5 of them) and one of 4, 8 or
// 16 for the rest (a = 5k + 1: 32^(k-1) 16 4); otherwise pc_radices.  allow32: the columns, and the rows that
// only the full-size row workgroups take (c^2 w > kPcSmallElems; their threads hold 16 values, so half of them
// idle in a radix-32 pass).  For comparison runs, LLP_COL_RADIX / LLP_ROW_RADIX = 8 keep the radix-8 plan and
// LLP_COL_RADIX / LLP_ROW_RADIX = 16 the radix-16 plan.
static int env_radix(const char* name) {
  const char* e = getenv(name);
  return e ? atoi(e) : 0;
}

int pc_wide_radices(int L, int* rad, bool col, bool allow32) {
  static const int col_radix = env_radix("LLP_COL_RADIX"), row_radix = env_radix("LLP_ROW_RADIX");
  const bool narrow = (col ? col_radix : row_radix) == 8;
  int a = 0;
  while (a < 30 && (1 << a) < L) ++a;
  if (narrow || (1 << a) != L || a < 6) return pc_radices(L, rad);
  int n = 0;
  if (allow32 && a >= 9 && (col ? col_radix : row_radix) != 16) {
    const int k = a / 5, rest = a % 5;
    for (int i = 0; i < (rest == 1 ? k - 1 : k); ++i) rad[n++] = 32;
    if (rest == 1) {
      rad[n++] = 16;
      rad[n++] = 4;
    } else if (rest > 1) {
      rad[n++] = 1 << rest;
    }
    return n;
  }
  const int k = a / 4, rest = a % 4;
  for (int i = 0; i < (rest == 1 ? k - 1 : k); ++i) rad[n++] = 16;
  if (rest == 1) {
    rad[n++] = 8;
    rad[n++] = 4;
  } else if (rest == 2) {
    rad[n++] = 4;
  } else if (rest == 3) {
    rad[n++] = 8;
  }
  return n;
}

// Whether a transform of length L needs a radix with the smaller per-thread budget.
static bool pc_small_radix(int L) {
  int rad[kPcMaxRad];
  const int n = pc_radices(L, rad);
  for (int i = 0; i < n; ++i)
    if (rad[i] != 8 && rad[i] != 4) return true;
  return false;
}

// Dynamic LDS of a pass over transforms of length L: c^2 padded sequences and the twiddle table.
static size_t pc_lds_bytes(int c, int L) { return ((size_t)c * c * seq_stride(L) + L) * sizeof(float2); }

bool pc_supported(const Geom& g) {
  int rad[kPcMaxRad];
  if (g.c < 1 || g.c > 4 || g.r < 1 || !(g.lam > 0.0f)) return false;
  if ((size_t)g.c * g.W > (size_t)kPcMaxElems || (size_t)g.c * g.H > (size_t)kPcMaxElems) return false;
  if (pc_lds_bytes(g.c, g.w) > (size_t)kPcMaxLds || pc_lds_bytes(g.c, g.h) > (size_t)kPcMaxLds) return false;
  if (pc_radices(g.w, rad) < 0 || pc_radices(g.h, rad) < 0) return false;
  if (pc_small_radix(g.w) && (size_t)g.c * g.W > (size_t)kPcSmallElems) return false;
  if (pc_small_radix(g.h) && (size_t)g.c * g.H > (size_t)kPcSmallElems) return false;
  return true;
}

int pc_row_blocks(const Geom& g) { return ((g.N + 1) / 2) * g.h; }
int pc_col_blocks(const Geom& g) { return g.w; }  // LR columns (the column pass takes every band pair of one)

size_t pc_spec_floats(const Geom& g) { return (size_t)((g.N + 1) / 2) * g.H * g.W * 2; }
size_t pc_uhat_floats(const Geom& g) { return (size_t)g.H * g.W * 2; }
size_t pc_tw_floats(const Geom& g) { return (size_t)2 * (g.h + g.w + g.H + g.W); }

// The plans of a scene's row and column transforms.
static int row_plan(const Geom& g, int* rad) {
  return pc_wide_radices(g.w, rad, false, (size_t)g.c * g.c * g.w > (size_t)kPcSmallElems);
}
static int col_plan(const Geom& g, int* rad) { return pc_wide_radices(g.h, rad, true, true); }

// The pass-major twiddles of a length-L transform (L complex values): pass p, of radix R over sub-transforms of
// length Ns, holds e^{-2 pi i t k / (Ns R)} for k < Ns, 0 < t < R at sum_{q < p} Ns_q (R_q - 1) + (t - 1) Ns +
// k; the passes use L - 1 entries and the last is unused.  FP64 evaluated, rounded once.
static float* pass_twiddles(const Geom& g, float* out, bool col) {  // L = h (columns) or w (rows)
  int rad[kPcMaxRad];
  const int n = col ? col_plan(g, rad) : row_plan(g, rad);
  const int L = col ? g.h : g.w;
  float* end = out + 2 * (size_t)L;
  int Ns = 1;
  for (int p = 0; p < n; ++p) {
    const int R = rad[p];
    for (int t = 1; t < R; ++t)
      for (int k = 0; k < Ns; ++k) {
        const double a = -2.0 * M_PI * (double)t * (double)k / ((double)Ns * (double)R);
        *out++ = (float)cos(a);
        *out++ = (float)sin(a);
      }
    Ns *= R;
  }
  while (out < end) *out++ = 0.0f;
  return end;
}

void pc_twiddles(const Geom& g, float* out) {
  out = pass_twiddles(g, out, true);
  out = pass_twiddles(g, out, false);
  const int lens[2] = {g.H, g.W};
  for (int L : lens)
    for (int m = 0; m < L; ++m) {
      const double a = -2.0 * M_PI * (double)m / (double)L;
      *out++ = (float)cos(a);
      *out++ = (float)sin(a);
    }
}

void pc_fill(PcDesc& d, const Geom& g, float* tw_dev) {
  d.g = g;
  d.npair = (g.N + 1) / 2;
  float2* tw = (float2*)tw_dev;
  d.twh = tw;
  d.tww = tw + g.h;
  d.twH = tw + g.h + g.w;
  d.twW = tw + g.h + g.w + g.H;
  d.nrw = row_plan(g, d.rw);
  d.nrh = col_plan(g, d.rh);
  d.mixed_w = pc_small_radix(g.w);
  d.mixed_h = pc_small_radix(g.h);
}

hipError_t pc_prepare() {
  const int bytes = kPcMaxLds;
  const void* kernels[10] = {(const void*)k_pc_rows<false, T>,      (const void*)k_pc_rows<true, T>,
                             (const void*)k_pc_rows<false, TS>,     (const void*)k_pc_rows<true, TS>,
                             (const void*)k_pc_cols<false>,         (const void*)k_pc_cols<true>,
                             (const void*)k_pc_rows_inv<false, T>,  (const void*)k_pc_rows_inv<true, T>,
                             (const void*)k_pc_rows_inv<false, TS>, (const void*)k_pc_rows_inv<true, TS>};
  for (const void* k : kernels) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static size_t pc_row_lds(const PcDesc* h_tab, int count) {
  size_t m = 0;
  for (int i = 0; i < count; ++i) {
    const Geom& g = h_tab[i].g;
    const size_t b = pc_lds_bytes(g.c, g.w);
    if (b > m) m = b;
  }
  return m;
}

// The column pass's LDS: the largest scene's group of kmax columns (pairs) of c^2 sequences, plus its twiddles.
static size_t pc_col_lds(const PcDesc* h_tab, int count, int budget) {
  size_t m = 0;
  for (int i = 0; i < count; ++i) {
    const Geom& g = h_tab[i].g;
    const int k = col_group_max(h_tab[i], budget);
    const size_t b = ((size_t)k * g.c * g.c * seq_stride(g.h) + g.h) * sizeof(float2);
    if (b > m) m = b;
  }
  return m;
}

void pc_plan(PcDesc* h_tab, int count, PcPlan* plan) {
  PcPlan P;
  P.count = count;
  for (int i = 0; i < count; ++i) {
    h_tab[i].row_block0 = P.row_blocks;
    h_tab[i].col_block0 = P.col_blocks;
    P.row_blocks += pc_row_blocks(h_tab[i].g);
    P.col_blocks += pc_col_blocks(h_tab[i].g);
    P.bands += h_tab[i].g.N;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&P.cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                               hipSuccess || P.cus < 1)
    P.cus = 256;
  P.row_lds = pc_row_lds(h_tab, count);
  P.col_budget = kPcColBudget;
  if (const char* e = getenv("LLP_COL_BUDGET")) {  // launch-shape override (elements per column group)
    const int v = atoi(e);
    if (v >= 1 && v <= kPcMaxElems) P.col_budget = v;
  }
  P.col_lds = pc_col_lds(h_tab, count, P.col_budget);
  P.small_rows = true;
  for (int i = 0; i < count; ++i) {
    const Geom& g = h_tab[i].g;
    P.mixed |= pc_small_radix(g.w) || pc_small_radix(g.h);
    P.small_rows &= (size_t)g.c * g.c * g.w <= (size_t)kPcSmallElems;
  }
  *plan = P;
}

hipError_t launch_pc_rows(int op, const PcDesc* t, const PcPlan& P, const ChanState* st, int prev, int cur,
                          hipStream_t s) {
  if (P.row_blocks <= 0) return hipSuccess;
  if (P.small_rows) {
    if (P.mixed)
      hipLaunchKernelGGL((k_pc_rows<true, TS>), dim3(P.row_blocks), dim3(TS), P.row_lds, s, op, t, P.count, st, prev,
                         cur);
    else
      hipLaunchKernelGGL((k_pc_rows<false, TS>), dim3(P.row_blocks), dim3(TS), P.row_lds, s, op, t, P.count, st, prev,
                         cur);
  } else if (P.mixed) {
    hipLaunchKernelGGL((k_pc_rows<true, T>), dim3(P.row_blocks), dim3(T), P.row_lds, s, op, t, P.count, st, prev, cur);
  } else {
    hipLaunchKernelGGL((k_pc_rows<false, T>), dim3(P.row_blocks), dim3(T), P.row_lds, s, op, t, P.count, st, prev,
                       cur);
  }
  return hipGetLastError();
}

hipError_t launch_pc_cols(int op, const PcDesc* t, const PcPlan& P, const ChanState* st, hipStream_t s) {
  if (P.col_blocks <= 0) return hipSuccess;
  // persistent workgroups: as many per compute unit as its LDS holds (one for 1024-point columns at c = 4)
  const int per_cu = std::max(1, std::min((int)(kPcCuLds / (P.col_lds + 1024)), 2048 / TC));
  const int grid = std::max(1, std::min(P.col_blocks, P.cus * per_cu));
  if (P.mixed)
    hipLaunchKernelGGL(k_pc_cols<true>, dim3(grid), dim3(TC), P.col_lds, s, op, t, P.count, st, P.col_budget);
  else
    hipLaunchKernelGGL(k_pc_cols<false>, dim3(grid), dim3(TC), P.col_lds, s, op, t, P.count, st, P.col_budget);
  return hipGetLastError();
}

hipError_t launch_pc_rows_inv(const PcDesc* t, const PcPlan& P, const ChanState* st, int cur, hipStream_t s) {
  if (P.row_blocks <= 0) return hipSuccess;
  if (P.small_rows) {
    if (P.mixed)
      hipLaunchKernelGGL((k_pc_rows_inv<true, TS>), dim3(P.row_blocks), dim3(TS), P.row_lds, s, t, P.count, st, cur);
    else
      hipLaunchKernelGGL((k_pc_rows_inv<false, TS>), dim3(P.row_blocks), dim3(TS), P.row_lds, s, t, P.count, st, cur);
  } else if (P.mixed) {
    hipLaunchKernelGGL((k_pc_rows_inv<true, T>), dim3(P.row_blocks), dim3(T), P.row_lds, s, t, P.count, st, cur);
  } else {
    hipLaunchKernelGGL((k_pc_rows_inv<false, T>), dim3(P.row_blocks), dim3(T), P.row_lds, s, t, P.count, st, cur);
  }
  return hipGetLastError();
}

hipError_t launch_pc_axpy(const float* a, const float* b, float* out, float sb, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_pc_axpy, dim3((unsigned)blocks), dim3(kBlock), 0, s, a, b, out, sb, n);
  return hipGetLastError();
}

hipError_t launch_pc_set_mbar(const PcDesc* t, int count, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_pc_set_mbar, dim3(1), dim3(64), 0, s, t, count, v);
  return hipGetLastError();
}

hipError_t launch_pc_mbar(const PcDesc* t, int count, double* part, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pc_mbar, dim3(kPcMbarBlocks, count), dim3(kBlock), 0, s, t, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pc_mbar_fin, dim3(count), dim3(kBlock), 0, s, t, kPcMbarBlocks, part);
  return hipGetLastError();
}

}  // namespace llp
