// Device building blocks for the power-of-two 2D DFT passes on gfx950.
//
// A length-N transform (8 <= N <= 1024) is a mixed-radix Stockham FFT spread
// over T = N/E threads that hold E elements each.  Stage s has radix R_s (E,
// or the remainder 2^(log2 N mod log2 E) last); a thread does E/R_s radix-R_s
// butterflies per stage in registers and the stages exchange data through LDS
// in natural (autosort) order, so input and output are in natural order and
// every global access of the T threads is a contiguous run.
//
// E is the knob between latency and throughput: E = 4 spreads a 256-point row
// over a full wave (4 stages, 3 exchanges), E = 16 packs it into 16 threads
// (2 stages, 1 exchange).
//
// Register layouts (g < E/R, r < R, j = t + T*g):
//   forward input : v[g*R0 + r]   = x[j + r*N/R0]        (R0 = first forward radix)
//   forward output: v[g*Rl + r]   = X[j + r*N/Rl]        (Rl = last forward radix)
// The inverse runs the stages in reverse order, so it takes the forward
// output layout and returns the forward input layout.  The inverse is
// unnormalised (e^{+j...}); callers fold 1/N where needed (eq. (23), R10).
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
constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
}  // namespace detail

// v * e^{-+ j 2 pi j / len} (minus for forward, plus for inverse); len | 32 and
// all arguments are compile-time constants after unrolling, so the trivial
// roots cost no multiply by zero.
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

// Ordering of LDS exchanges: the whole block (WAVE = false), or, when every
// transform lives inside one wavefront, only that wavefront: its LDS operations
// are performed in program order, so a compiler-level barrier with wavefront
// fences suffices and the block's other waves are not held up.
template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Mixed-radix Stockham FFT of N points over T = N/E threads.  WAVE: the T
// threads of every transform sit in one wavefront (T <= 64, rows aligned).
// ---------------------------------------------------------------------------
template <int N, int E, bool WAVE = false>
struct Stockham {
  static_assert((N & (N - 1)) == 0 && N >= 8 && N <= 1024, "N");
  static_assert((E & (E - 1)) == 0 && E >= 2 && E <= 32 && E <= N, "E");
  static constexpr int T = N / E;
  static constexpr int LOGN = detail::ilog2(N);
  static constexpr int LOGE = detail::ilog2(E);
  static constexpr int NFULL = LOGN / LOGE;
  static constexpr int REM = 1 << (LOGN % LOGE);          // 1 if none
  static constexpr int NST = NFULL + (REM > 1 ? 1 : 0);  // number of stages
  static constexpr int R0 = E;                            // first forward radix
  static constexpr int RL = (REM > 1) ? REM : E;          // last forward radix

  // radix of stage s in forward order; the inverse uses the reverse order
  static constexpr int fwd_radix(int s) { return s < NFULL ? E : REM; }
  static constexpr int radix(int s, bool inv) { return inv ? fwd_radix(NST - 1 - s) : fwd_radix(s); }
  static constexpr int span(int s, bool inv) {  // product of the radices before stage s
    int p = 1;
    for (int i = 0; i < s; ++i) p *= radix(i, inv);
    return p;
  }

  // LDS slot of exchange element i: one padding slot after every 8, so the
  // stage writes (stride R in i) spread over the banks instead of piling onto few
  __device__ static __forceinline__ int px(int i) { return i + (i >> 3); }

  // element index held in register slot e, for a layout whose stage radix is R
  template <int R>
  __device__ static __forceinline__ int layout_index(int t, int e) {
    return t + T * (e / R) + (e % R) * (N / R);
  }
  __device__ static __forceinline__ int in_index(int t, int e) { return layout_index<R0>(t, e); }
  __device__ static __forceinline__ int out_index(int t, int e) { return layout_index<RL>(t, e); }

  // One stage.  On entry v holds the stage input in layout<R> (stage 0: the
  // caller loaded it; later stages: read here from LDS).  Every LDS write
  // phase is preceded by a barrier so that no thread overwrites a slot another
  // thread of the previous read phase still needs; `sm[i*ss]` is slot i.
  template <bool INV, int S>
  __device__ static __forceinline__ void stage(float2* v, int t, const float2* tw, float2* sm, int ss,
                                               bool sync0 = true) {
    constexpr int R = radix(S, INV);
    constexpr int NS = span(S, INV);
    constexpr int G = E / R;
    if constexpr (S > 0) {
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int r = 0; r < R; ++r) v[g * R + r] = sm[px(t + T * g + r * (N / R)) * ss];
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int j = t + T * g;
      const int k = j & (NS - 1);
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float2 w = tw[(r * k * (N / (NS * R))) & (N - 1)];
          v[g * R + r] = INV ? cmulc(v[g * R + r], w) : cmul(v[g * R + r], w);
        }
      }
      dft_reg<R, INV>(v + g * R);
    }
    if constexpr (S + 1 < NST) {
      if (S > 0 || sync0) lds_sync<WAVE>();
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int j = t + T * g;
        const int k = j & (NS - 1);
        const int base = (j / NS) * NS * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) sm[px(base + r * NS) * ss] = v[g * R + r];
      }
      lds_sync<WAVE>();
      stage<INV, S + 1>(v, t, tw, sm, ss);
    }
  }

  // v: forward input layout -> forward output layout.  Every thread of the
  // block must call it (it contains barriers when NST > 1).  sync0 = false
  // skips the barrier before the first LDS write when nothing may still read sm.
  __device__ static __forceinline__ void forward(float2* v, int t, const float2* tw, float2* sm, int ss,
                                                 bool sync0 = true) {
    stage<false, 0>(v, t, tw, sm, ss, sync0);
  }
  // v: forward output layout -> forward input layout, unnormalised inverse.
  __device__ static __forceinline__ void inverse(float2* v, int t, const float2* tw, float2* sm, int ss,
                                                 bool sync0 = true) {
    stage<true, 0>(v, t, tw, sm, ss, sync0);
  }

  // Two-area form: exchange i goes through area A (i even) or B (i odd), so a
  // write never meets a read of the same area still in flight and each
  // exchange needs one barrier instead of two.  The first exchange writes A
  // after a barrier only when `sync0` (A may still be read by the caller).
  // After the call the area of the last exchange is B iff kLastB; a following
  // transform may start in the other area with sync0 = false.
  static constexpr bool kTwoArea = NST >= 3;
  static constexpr bool kLastB = NST >= 2 && ((NST - 2) & 1) == 1;

  template <bool INV, int S>
  __device__ static __forceinline__ void stage2(float2* v, int t, const float2* tw, float2* smA, float2* smB, int ss,
                                                bool sync0) {
    constexpr int R = radix(S, INV);
    constexpr int NS = span(S, INV);
    constexpr int G = E / R;
    if constexpr (S > 0) {
      const float2* rd = ((S - 1) & 1) ? smB : smA;
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int r = 0; r < R; ++r) v[g * R + r] = rd[px(t + T * g + r * (N / R)) * ss];
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int j = t + T * g;
      const int k = j & (NS - 1);
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float2 w = tw[(r * k * (N / (NS * R))) & (N - 1)];
          v[g * R + r] = INV ? cmulc(v[g * R + r], w) : cmul(v[g * R + r], w);
        }
      }
      dft_reg<R, INV>(v + g * R);
    }
    if constexpr (S + 1 < NST) {
      float2* wr = (S & 1) ? smB : smA;
      if constexpr (S == 0) {
        if (sync0) lds_sync<WAVE>();
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int j = t + T * g;
        const int k = j & (NS - 1);
        const int base = (j / NS) * NS * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) wr[px(base + r * NS) * ss] = v[g * R + r];
      }
      lds_sync<WAVE>();
      stage2<INV, S + 1>(v, t, tw, smA, smB, ss, sync0);
    }
  }
  __device__ static __forceinline__ void forward2(float2* v, int t, const float2* tw, float2* smA, float2* smB, int ss,
                                                  bool sync0) {
    stage2<false, 0>(v, t, tw, smA, smB, ss, sync0);
  }
  __device__ static __forceinline__ void inverse2(float2* v, int t, const float2* tw, float2* smA, float2* smB, int ss,
                                                  bool sync0) {
    stage2<true, 0>(v, t, tw, smA, smB, ss, sync0);
  }
};


}  // namespace bccb
