// FP64 (complex128) row and column passes: the eq. (23) product and the ISTA / FISTA / ADMM
// iterations of the full passes, in double precision, for accuracy studies at the level of the
// paper's FP64 comparison (Table I).  Layouts and the split into passes are those of the FP32
// passes (passes.h): grids [L2][L1], row pass = transforms along l1 plus the update, column
// pass = DFT_cols, spectral multiplier, IDFT_cols.  Each transform is an iterative radix-2 FFT
// in LDS (bit-reversed load, log2 N butterfly stages, one thread per butterfly), simple rather
// than fast: this path is about the arithmetic, the FP32 passes about speed.
#include <hip/hip_runtime.h>

#include "passes_f64.h"

namespace bccb {

namespace {

__device__ __forceinline__ double2 dadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 dsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 dmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// S_k(z) = z (1 - k/|z|) for |z| > k, else 0 (R3)
__device__ __forceinline__ double2 dshrink(double2 z, double k) {
  const double a = sqrt(z.x * z.x + z.y * z.y);
  if (!(a > k)) return make_double2(0.0, 0.0);
  const double f = 1.0 - k / a;
  return make_double2(z.x * f, z.y * f);
}

__device__ __forceinline__ int brev_n(int i, int logn) { return static_cast<int>(__brev(static_cast<unsigned>(i)) >> (32 - logn)); }

// In-place FFT of the N points x[0..N) in LDS, already in bit-reversed order, by the T = N/2
// threads t of one transform; tw[j] = e^{-j 2 pi j / N}; INV conjugates the twiddles
// (unnormalised).  The block meets between stages.
template <bool INV>
__device__ void fft_lds(double2* x, int N, int t, bool active, const double2* tw) {
  for (int len = 2; len <= N; len <<= 1) {
    const int half = len >> 1;
    if (active) {
      const int grp = t / half, k = t - grp * half;
      const int i0 = grp * len + k;
      double2 w = tw[k * (N / len)];
      if (INV) w.y = -w.y;
      const double2 a = x[i0];
      const double2 b = dmul(x[i0 + half], w);
      x[i0] = dadd(a, b);
      x[i0 + half] = dsub(a, b);
    }
    __syncthreads();
  }
}

// Row pass: R rows per block, N/2 threads each.
__global__ __launch_bounds__(512) void k_row64(RowArgs64 a, int N, int logn, int R) {
  extern __shared__ double2 sh[];
  double2* tw = sh;                       // [N]
  const int T = N / 2;
  const int r = threadIdx.x / T, t = threadIdx.x - (threadIdx.x / T) * T;
  const int row = blockIdx.x * R + r;
  const bool active = r < R && row < a.nrows;
  double2* x = sh + N + static_cast<size_t>(r) * N;
  const size_t base = static_cast<size_t>(row) * N;
  for (int j = threadIdx.x; j < N; j += blockDim.x) tw[j] = a.tw[j];
  if (a.mode != ROW64_FWD) {
    // the row spectrum, bit reversed for the inverse transform
    if (active)
      for (int j = t; j < N; j += T) x[brev_n(j, logn)] = a.xy[base + j];
    __syncthreads();
    fft_lds<true>(x, N, t, active, tw);
    if (active) {
      for (int j = t; j < N; j += T) {
        const size_t idx = base + j;
        const double2 u = x[j];   // IDFT_rows (unnormalised; the column pass folded 1/L in)
        const int l2 = row % a.rows_per_scene;
        const bool in = a.act_cols == 0 || (j < a.act_cols && l2 < a.act_rows);
        double2 out = u;
        if (a.mode == ROW64_INV) {
          a.dst[idx] = make_double2(u.x * a.scale, u.y * a.scale);
          continue;
        } else if (a.mode == ROW64_ISTA) {
          const double2 c = in ? dshrink(dadd(u, a.rhs[idx]), a.kappa) : make_double2(0.0, 0.0);
          if (a.last) a.out_c[idx] = c;
          out = c;
        } else if (a.mode == ROW64_FISTA) {
          const double2 c = in ? dshrink(dadd(u, a.rhs[idx]), a.kappa) : make_double2(0.0, 0.0);
          const double2 cp = a.state[idx];
          a.state[idx] = c;
          out = make_double2(c.x + a.beta * (c.x - cp.x), c.y + a.beta * (c.y - cp.y));
        } else {   // ROW64_ADMM: c = w + u; z = S(c + v); v += c - z; next input z - v
          const double2 c = in ? dadd(a.rhs[idx], u) : make_double2(0.0, 0.0);
          const double2 v = a.state[idx];
          const double2 z = dshrink(dadd(c, v), a.kappa);
          const double2 vn = dsub(dadd(v, c), z);
          a.state[idx] = vn;
          if (a.last) {
            a.out_z[idx] = z;
            if (a.out_c) a.out_c[idx] = c;
          }
          out = dsub(z, vn);
        }
        x[j] = out;
      }
    }
    __syncthreads();
    if (a.mode == ROW64_INV || a.last) return;   // whole block returns together
    // forward transform of the next input: re-load in bit-reversed order
    double2 keep[2];
    if (active)
      for (int q = 0, j = t; j < N; j += T, ++q) keep[q] = x[j];
    __syncthreads();
    if (active)
      for (int q = 0, j = t; j < N; j += T, ++q) x[brev_n(j, logn)] = keep[q];
    __syncthreads();
  } else {
    if (active) {
      for (int j = t; j < N; j += T) {
        double2 v = a.src ? a.src[base + j] : make_double2(0.0, 0.0);
        if (!(isfinite(v.x) && isfinite(v.y)) && a.flag) *a.flag = 1;
        x[brev_n(j, logn)] = v;
      }
    }
    __syncthreads();
  }
  fft_lds<false>(x, N, t, active, tw);
  if (active)
    for (int j = t; j < N; j += T) a.xy[base + j] = x[j];
}

// Column pass: R columns per block (adjacent k1, so loads of one l2 are contiguous), N/2
// threads per column.
__global__ __launch_bounds__(512) void k_col64(ColArgs64 a, int N, int logn, int R) {
  extern __shared__ double2 sh[];
  double2* tw = sh;
  const int T = N / 2;
  const int r = threadIdx.x / T, t = threadIdx.x - (threadIdx.x / T) * T;
  const int k1_0 = blockIdx.x * R;
  const bool active = r < R && k1_0 + r < a.L1;
  for (int j = threadIdx.x; j < N; j += blockDim.x) tw[j] = a.tw[j];
  // load: consecutive threads read consecutive columns of one l2
  for (int idx = threadIdx.x; idx < N * R; idx += blockDim.x) {
    const int c = idx % R, l2 = idx / R;
    if (k1_0 + c < a.L1) sh[N + static_cast<size_t>(c) * N + brev_n(l2, logn)] = a.xy[static_cast<size_t>(l2) * a.L1 + k1_0 + c];
  }
  __syncthreads();
  double2* x = sh + N + static_cast<size_t>(r) * N;
  if (a.mode != COL64_INV) {
    // DFT_cols, the spectral multiplier, and back to bit-reversed order for the inverse
    fft_lds<false>(x, N, t, active, tw);
    double2 keep[2];
    if (active) {
      const int k1 = k1_0 + r;
      for (int q = 0, k2 = t; k2 < N; k2 += T, ++q) {
        const double om = a.omega[static_cast<size_t>(k2) * a.L1 + k1];
        const double m = a.mode == COL64_AFFINE ? a.ca + a.cb * om : a.scale / (om + a.rho);
        keep[q] = make_double2(x[k2].x * m, x[k2].y * m);
      }
    }
    __syncthreads();
    if (active)
      for (int q = 0, k2 = t; k2 < N; k2 += T, ++q) x[brev_n(k2, logn)] = keep[q];
    __syncthreads();
  }
  // (COL64_INV: the column was loaded spectral, already bit reversed)
  fft_lds<true>(x, N, t, active, tw);
  for (int idx = threadIdx.x; idx < N * R; idx += blockDim.x) {
    const int c = idx % R, l2 = idx / R;
    if (k1_0 + c < a.L1) a.xy[static_cast<size_t>(l2) * a.L1 + k1_0 + c] = sh[N + static_cast<size_t>(c) * N + l2];
  }
}

// S[k2][k1] = scale * sum over kept (m1, m2) folding onto (k1, k2) of (-1)^(m1+m2) y_m
__global__ void k_scatter64(const double2* __restrict__ y, const int* __restrict__ sensor_of, int M1, int M2,
                            int L1, int L2, double scale, double2* __restrict__ S, int* flag) {
  const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<long>(L1) * L2) return;
  const int k1 = static_cast<int>(idx % L1), k2 = static_cast<int>(idx / L1);
  double2 acc = make_double2(0.0, 0.0);
  bool ok = true;
  for (int m2 = k2; m2 < M2; m2 += L2)
    for (int m1 = k1; m1 < M1; m1 += L1) {
      const int s = sensor_of[m2 * M1 + m1];
      if (s < 0) continue;
      const double2 v = y[s];
      ok = ok && isfinite(v.x) && isfinite(v.y);
      acc = ((m1 + m2) & 1) ? dsub(acc, v) : dadd(acc, v);
    }
  if (!ok && flag) *flag = 1;
  S[idx] = make_double2(acc.x * scale, acc.y * scale);
}

__global__ void k_spectral_div64(double2* xy, const double* omega, double rho, long n) {
  for (long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * blockDim.x) {
    const double d = 1.0 / (omega[i] + rho);
    xy[i] = make_double2(xy[i].x * d, xy[i].y * d);
  }
}

__global__ void k_fill64(double2* p, long n) {
  for (long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * blockDim.x)
    p[i] = make_double2(0.0, 0.0);
}

__global__ void k_copy64(double2* d, const double2* s, long n) {
  for (long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * blockDim.x)
    d[i] = s[i];
}

int ilog2i(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

int blocks_for(long n) {
  long b = (n + 255) / 256;
  return static_cast<int>(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

}  // namespace

int launch_row64(int N, const RowArgs64& a, hipStream_t s) {
  if (N < 2 || N > 1024 || (N & (N - 1))) return -1;
  const int T = N / 2;
  const int R = T >= 256 ? 1 : 256 / T;
  const size_t shm = sizeof(double2) * static_cast<size_t>(N) * (1 + R);
  hipLaunchKernelGGL(k_row64, dim3((a.nrows + R - 1) / R), dim3(R * T), shm, s, a, N, ilog2i(N), R);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_col64(int N, const ColArgs64& a, hipStream_t s) {
  if (N < 2 || N > 1024 || (N & (N - 1))) return -1;
  const int T = N / 2;
  int R = T >= 256 ? 1 : 256 / T;
  if (R > a.L1) R = a.L1;
  const size_t shm = sizeof(double2) * static_cast<size_t>(N) * (1 + R);
  hipLaunchKernelGGL(k_col64, dim3((a.L1 + R - 1) / R), dim3(R * T), shm, s, a, N, ilog2i(N), R);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_scatter64(const double2* y, const int* sensor_of, int M1, int M2, int L1, int L2, double scale,
                     double2* S, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter64, dim3(static_cast<unsigned>((static_cast<long>(L1) * L2 + 255) / 256)), dim3(256), 0,
                     s, y, sensor_of, M1, M2, L1, L2, scale, S, flag);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_spectral_div64(double2* xy, const double* omega, double rho, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_spectral_div64, dim3(blocks_for(n)), dim3(256), 0, s, xy, omega, rho, n);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_fill64(double2* p, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill64, dim3(blocks_for(n)), dim3(256), 0, s, p, n);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_copy64(double2* d, const double2* src, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy64, dim3(blocks_for(n)), dim3(256), 0, s, d, src, n);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace bccb
