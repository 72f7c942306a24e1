// Device building blocks for the power-of-two 2D DFT passes on gfx950.
//
// A length-N transform (N = A*B, 8 <= N <= 1024) is split four-step style:
// B-strided columns of length A are transformed in registers, multiplied by
// the twiddles W_N^{n2*k1}, transposed through LDS, and transformed again with
// length B.  One LDS exchange per transform, natural-order input and output,
// and every global access of a thread group is a contiguous run of T elements.
//
// Data distributions over the T = B threads that own one transform:
//   D_in : thread t holds x[B*i + t],          i  in [0, A)
//   D_out: thread t holds X[t + T*q + A*k2],   q in [0, A/T), k2 in [0, B)
// The forward transform maps D_in -> D_out, the inverse maps D_out -> D_in.
// The inverse is unnormalised (sum with e^{+j...}); callers fold 1/N where
// the product needs it (Sec. III-B, eq. (23), reading R10).
#pragma once

#include <hip/hip_runtime.h>

namespace bccb {

// ---------------------------------------------------------------------------
// complex helpers (float2 = interleaved re, im)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// ---------------------------------------------------------------------------
// Compile-time unit roots e^{-j 2 pi k / 32}, k < 32, from a Taylor series on
// the first octant (enough terms for double precision) and octant symmetry.
// ---------------------------------------------------------------------------
namespace detail {
constexpr double kPi = 3.14159265358979323846;
constexpr double tsin(double x) {
  double t = x, s = x;
  for (int n = 1; n < 14; ++n) { t *= -x * x / ((2.0 * n) * (2.0 * n + 1.0)); s += t; }
  return s;
}
constexpr double tcos(double x) {
  double t = 1.0, s = 1.0;
  for (int n = 1; n < 14; ++n) { t *= -x * x / ((2.0 * n - 1.0) * (2.0 * n)); s += t; }
  return s;
}
struct Roots32 {
  float c[32];
  float s[32];
  constexpr Roots32() : c(), s() {
    for (int k = 0; k < 32; ++k) {
      const int q = k / 8, r = k % 8;
      const double a = 2.0 * kPi * r / 32.0;          // in [0, pi/2)
      const double cr = (r <= 4) ? tcos(a) : tsin(kPi / 2 - a);
      const double sr = (r <= 4) ? tsin(a) : tcos(kPi / 2 - a);
      double C = 0.0, S = 0.0;                        // cos, sin of 2 pi k / 32
      if (q == 0) { C = cr; S = sr; }
      else if (q == 1) { C = -sr; S = cr; }
      else if (q == 2) { C = -cr; S = -sr; }
      else { C = sr; S = -cr; }
      c[k] = static_cast<float>(C);
      s[k] = static_cast<float>(S);
    }
  }
};
constexpr Roots32 kRoots{};

constexpr int brev(int i, int n) {
  int r = 0;
  for (int b = 1; b < n; b <<= 1) { r = (r << 1) | (i & 1); i >>= 1; }
  return r;
}
}  // namespace detail

// v * e^{-+ j 2 pi j / len} (minus for forward, plus for inverse); len | 32, all
// arguments are compile-time constants after unrolling, so the trivial roots
// (1, -+j, and the 45-degree ones) cost no multiply by zero.
template <bool INV>
__device__ __forceinline__ float2 rot_const(float2 v, int j, int len) {
  const int k = (j * (32 / len)) & 31;
  if (k == 0) return v;
  if (k == 8) return INV ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
  if (k == 16) return make_float2(-v.x, -v.y);
  if (k == 24) return INV ? make_float2(v.y, -v.x) : make_float2(-v.y, v.x);
  const float c = detail::kRoots.c[k];
  const float s = INV ? detail::kRoots.s[k] : -detail::kRoots.s[k];
  return make_float2(v.x * c - v.y * s, v.x * s + v.y * c);
}

// In-register DFT of N <= 32 points held in v[0..N-1] (natural order in and out).
// Radix-2 decimation in time after a compile-time bit-reversal permutation.
template <int N, bool INV>
__device__ __forceinline__ void dft_reg(float2* v) {
  static_assert(N >= 1 && N <= 32 && (N & (N - 1)) == 0, "register DFT size");
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int j = detail::brev(i, N);
    if (j > i) { const float2 t = v[i]; v[i] = v[j]; v[j] = t; }
  }
#pragma unroll
  for (int len = 2; len <= N; len <<= 1) {
#pragma unroll
    for (int i = 0; i < N; i += len) {
#pragma unroll
      for (int j = 0; j < len / 2; ++j) {
        const float2 a = v[i + j];
        const float2 b = rot_const<INV>(v[i + j + len / 2], j, len);
        v[i + j] = cadd(a, b);
        v[i + j + len / 2] = csub(a, b);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Four-step shapes: N = A * B with A >= B, T = B threads per transform and
// E = A elements per thread.
// ---------------------------------------------------------------------------
template <int N> struct Shape;
template <> struct Shape<8>    { static constexpr int A = 4,  B = 2;  };
template <> struct Shape<16>   { static constexpr int A = 4,  B = 4;  };
template <> struct Shape<32>   { static constexpr int A = 8,  B = 4;  };
template <> struct Shape<64>   { static constexpr int A = 8,  B = 8;  };
template <> struct Shape<128>  { static constexpr int A = 16, B = 8;  };
template <> struct Shape<256>  { static constexpr int A = 16, B = 16; };
template <> struct Shape<512>  { static constexpr int A = 32, B = 16; };
template <> struct Shape<1024> { static constexpr int A = 32, B = 32; };

template <int N>
struct FFT {
  static constexpr int A = Shape<N>::A;
  static constexpr int B = Shape<N>::B;
  static constexpr int T = B;        // threads per transform
  static constexpr int E = A;        // elements per thread
  static constexpr int Q = A / T;    // k1 groups per thread in D_out
  static constexpr int PAD = 1;
  static constexpr int LDS = A * (B + PAD);   // float2 slots per transform

  // global element index of register slot e in each distribution
  __device__ static __forceinline__ int in_index(int t, int e) { return B * e + t; }
  __device__ static __forceinline__ int out_index(int t, int e) {
    const int q = e / B, k2 = e % B;
    return t + T * q + A * k2;
  }

  // LDS slot of (k1, n2); `stride` separates the transforms that share one LDS array
  __device__ static __forceinline__ int slot(int k1, int n2) { return k1 * (B + PAD) + n2; }

  // D_in -> D_out.  tw[j] = e^{-j 2 pi j/N} (table in LDS or global); the LDS
  // slot of (k1, n2) for this transform is sm[slot(k1, n2) * ss], so several
  // transforms can interleave in one array.  Contains one __syncthreads():
  // every thread of the block must call it.  Thread t only writes the slots
  // (., t) it later reads back itself and reads rows (t + T q, .) it wrote
  // itself in a preceding inverse, so back-to-back forward/inverse calls on
  // the same area need no extra barrier.
  __device__ static __forceinline__ void forward(float2* v, int t, const float2* tw, float2* sm, int ss) {
    dft_reg<A, false>(v);
#pragma unroll
    for (int k1 = 1; k1 < A; ++k1) v[k1] = cmul(v[k1], tw[(t * k1) & (N - 1)]);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) sm[slot(k1, t) * ss] = v[k1];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) v[q * B + n2] = sm[slot(t + T * q, n2) * ss];
#pragma unroll
    for (int q = 0; q < Q; ++q) dft_reg<B, false>(v + q * B);
  }

  // D_out -> D_in, unnormalised inverse.  Same synchronisation contract.
  __device__ static __forceinline__ void inverse(float2* v, int t, const float2* tw, float2* sm, int ss) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      dft_reg<B, true>(v + q * B);
      const int k1 = t + T * q;
#pragma unroll
      for (int n2 = 1; n2 < B; ++n2) v[q * B + n2] = cmulc(v[q * B + n2], tw[(n2 * k1) & (N - 1)]);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) sm[slot(t + T * q, n2) * ss] = v[q * B + n2];
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) v[k1] = sm[slot(k1, t) * ss];
    dft_reg<A, true>(v);
  }
};

}  // namespace bccb
