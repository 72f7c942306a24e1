// Kernels of plans on a zero-padded embedding (general element spacing, any grid length):
// separable steering-vector products for D_s^H y and D_s c, and the copies between the
// caller's L1 x L2 grid and the padded P1 x P2 transform grid.
#include "kernels.h"
#include "spaced_kernels.h"

namespace bccb {

namespace {

__device__ __forceinline__ bool finite2s(float2 v) { return __builtin_isfinite(v.x) && __builtin_isfinite(v.y); }

// U[m2][l1] = scale * sum over kept m1 of conj(W1[m1][l1]) y[sensor(m1, m2)]
__global__ __launch_bounds__(256) void k_adj_stage1(const float2* __restrict__ y, const int* __restrict__ sensor_of,
                                                    const float2* __restrict__ W1, int M1, int M2, int A1, float scale,
                                                    float2* __restrict__ U, int* flag) {
  const int l1 = blockIdx.x * blockDim.x + threadIdx.x;
  const int m2 = blockIdx.y;
  if (l1 >= A1 || m2 >= M2) return;
  float ax = 0.f, ay = 0.f;
  bool ok = true;
  for (int m1 = 0; m1 < M1; ++m1) {
    const int s = sensor_of[m2 * M1 + m1];
    if (s < 0) continue;
    const float2 v = y[s];
    ok = ok && finite2s(v);
    const float2 w = W1[static_cast<long>(m1) * A1 + l1];
    ax += w.x * v.x + w.y * v.y;   // conj(w) v
    ay += w.x * v.y - w.y * v.x;
  }
  if (!ok && flag) *flag = 1;
  U[static_cast<long>(m2) * A1 + l1] = make_float2(ax * scale, ay * scale);
}

// out[l2 * ld + l1] = sum_{m2} conj(W2[m2][l2]) U[m2][l1] for l1 < A1, l2 < A2; zero for the
// rest of the out_cols x out_rows window
__global__ __launch_bounds__(256) void k_adj_stage2(const float2* __restrict__ U, const float2* __restrict__ W2, int M2,
                                                    int A1, int A2, int out_cols, int out_rows, int ld,
                                                    float2* __restrict__ out) {
  const int l1 = blockIdx.x * blockDim.x + threadIdx.x;
  const int l2 = blockIdx.y;
  if (l1 >= out_cols || l2 >= out_rows) return;
  float ax = 0.f, ay = 0.f;
  if (l1 < A1 && l2 < A2) {
    for (int m2 = 0; m2 < M2; ++m2) {
      const float2 w = W2[static_cast<long>(m2) * A2 + l2];
      const float2 u = U[static_cast<long>(m2) * A1 + l1];
      ax += w.x * u.x + w.y * u.y;
      ay += w.x * u.y - w.y * u.x;
    }
  }
  out[static_cast<long>(l2) * ld + l1] = make_float2(ax, ay);
}

// T[l2][m1] = sum_{l1 < A1} W1[m1][l1] c[l2][l1]  (c: [A2][A1], row stride ldc)
__global__ __launch_bounds__(256) void k_fwd_stage1(const float2* __restrict__ c, int ldc, const float2* __restrict__ W1,
                                                    int M1, int A1, int A2, float2* __restrict__ T, int* flag) {
  const int m1 = blockIdx.x * blockDim.x + threadIdx.x;
  const int l2 = blockIdx.y;
  if (m1 >= M1 || l2 >= A2) return;
  float ax = 0.f, ay = 0.f;
  bool ok = true;
  const float2* row = c + static_cast<long>(l2) * ldc;
  const float2* w = W1 + static_cast<long>(m1) * A1;
  for (int l1 = 0; l1 < A1; ++l1) {
    const float2 v = row[l1];
    ok = ok && finite2s(v);
    const float2 ww = w[l1];
    ax += ww.x * v.x - ww.y * v.y;
    ay += ww.x * v.y + ww.y * v.x;
  }
  if (!ok && flag) *flag = 1;
  T[static_cast<long>(l2) * M1 + m1] = make_float2(ax, ay);
}

// Per block: sum over its sensors m of 1/2 |y_m - (D_s c)_m|^2, (D_s c)_m = sum_{l2} W2[m2][l2] T[l2][m1]
__global__ __launch_bounds__(256) void k_fwd_resid(const float2* __restrict__ T, const float2* __restrict__ W2,
                                                   const int2* __restrict__ sensors, const float2* __restrict__ y,
                                                   int M, int M1, int A2, double* __restrict__ partial) {
  __shared__ double red[256];
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  double r2 = 0.0;
  if (m < M) {
    const int2 s = sensors[m];
    float ax = 0.f, ay = 0.f;
    for (int l2 = 0; l2 < A2; ++l2) {
      const float2 w = W2[static_cast<long>(s.y) * A2 + l2];
      const float2 t = T[static_cast<long>(l2) * M1 + s.x];
      ax += w.x * t.x - w.y * t.y;
      ay += w.x * t.y + w.y * t.x;
    }
    const double dx = static_cast<double>(y[m].x) - ax, dy = static_cast<double>(y[m].y) - ay;
    r2 = 0.5 * (dx * dx + dy * dy);
  }
  red[threadIdx.x] = r2;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// dst [P2][P1] <- src [A2][A1] (src == nullptr: zeros), zero outside the window
__global__ void k_pad(const float2* __restrict__ src, int A1, int A2, int P1, int P2, float2* __restrict__ dst) {
  const long n = static_cast<long>(P1) * P2;
  for (long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<long>(gridDim.x) * blockDim.x) {
    const int l1 = static_cast<int>(i % P1), l2 = static_cast<int>(i / P1);
    dst[i] = (src && l1 < A1 && l2 < A2) ? src[static_cast<long>(l2) * A1 + l1] : make_float2(0.f, 0.f);
  }
}

// dst [A2][A1] <- the window of src [P2][P1]
__global__ void k_crop(const float2* __restrict__ src, int A1, int A2, int P1, float2* __restrict__ dst) {
  const long n = static_cast<long>(A1) * A2;
  for (long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<long>(gridDim.x) * blockDim.x) {
    const int l1 = static_cast<int>(i % A1), l2 = static_cast<int>(i / A1);
    dst[i] = src[static_cast<long>(l2) * P1 + l1];
  }
}

int grid_blocks(long n) {
  long b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  return static_cast<int>(b < 1 ? 1 : b);
}

}  // namespace

int launch_sep_adjoint(const float2* y, const int* sensor_of, const float2* W1, const float2* W2, int M1, int M2,
                       int A1, int A2, float scale, float2* U, int out_cols, int out_rows, int ld, float2* out,
                       int* flag, hipStream_t s) {
  if (A1 < 1 || A2 < 1 || out_cols < A1 || out_rows < A2 || ld < out_cols) return -1;
  hipLaunchKernelGGL(k_adj_stage1, dim3((A1 + 255) / 256, M2), dim3(256), 0, s, y, sensor_of, W1, M1, M2, A1, scale,
                     U, flag);
  hipLaunchKernelGGL(k_adj_stage2, dim3((out_cols + 255) / 256, out_rows), dim3(256), 0, s, U, W2, M2, A1, A2,
                     out_cols, out_rows, ld, out);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_sep_resid(const float2* c, int ldc, const float2* W1, const float2* W2, const int2* sensors,
                     const float2* y, int M, int M1, int A1, int A2, float2* T, double* partial, int* nblocks,
                     int* flag, hipStream_t s) {
  const int nb = (M + 255) / 256;
  if (nb > kReduceBlocks || M < 1) return -1;
  hipLaunchKernelGGL(k_fwd_stage1, dim3((M1 + 255) / 256, A2), dim3(256), 0, s, c, ldc, W1, M1, A1, A2, T, flag);
  hipLaunchKernelGGL(k_fwd_resid, dim3(nb), dim3(256), 0, s, T, W2, sensors, y, M, M1, A2, partial);
  *nblocks = nb;
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_pad(const float2* src, int A1, int A2, int P1, int P2, float2* dst, hipStream_t s) {
  if (A1 > P1 || A2 > P2) return -1;
  hipLaunchKernelGGL(k_pad, dim3(grid_blocks(static_cast<long>(P1) * P2)), dim3(256), 0, s, src, A1, A2, P1, P2, dst);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_crop(const float2* src, int A1, int A2, int P1, float2* dst, hipStream_t s) {
  if (A1 > P1) return -1;
  hipLaunchKernelGGL(k_crop, dim3(grid_blocks(static_cast<long>(A1) * A2)), dim3(256), 0, s, src, A1, A2, P1, dst);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace bccb
