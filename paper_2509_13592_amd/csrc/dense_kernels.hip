// The "regular" dense implementation the paper compares against (Sec. II-B,
// Sec. III-C): the explicit L x L iteration matrix -- I - mu G for ISTA/FISTA,
// (G + rho I)^-1 for ADMM -- multiplied by the iterate every iteration, with the
// proximal/momentum/dual updates fused into the matrix-vector product's
// epilogue.  O(L^2) bytes per iteration, streamed from HBM once.
#include "fft_device.h"
#include "kernels.h"

namespace bccb {

namespace {

constexpr int kRows = 8;        // matrix rows per block (each iterate load feeds 8 rows)
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kThreads = 256;

__device__ __forceinline__ float2 shrink_d(float2 z, float k) {
  const float a2 = z.x * z.x + z.y * z.y;
  if (!(a2 > k * k)) return make_float2(0.f, 0.f);
  const float f = 1.f - k * __builtin_amdgcn_rsqf(a2);
  return make_float2(z.x * f, z.y * f);
}

// R[l][l'] = col[((l1 - l1') mod L1) + ((l2 - l2') mod L2) L1]: the BCCB matrix with first column col.
__global__ __launch_bounds__(256) void k_dense_build(const float2* __restrict__ col, int L1, int L2,
                                                     float2* __restrict__ R) {
  const long L = static_cast<long>(L1) * L2;
  const long row = blockIdx.x;
  const int r1 = static_cast<int>(row % L1), r2 = static_cast<int>(row / L1);
  for (long j = static_cast<long>(blockIdx.y) * 256 + threadIdx.x; j < L; j += static_cast<long>(gridDim.y) * 256) {
    const int c1 = static_cast<int>(j % L1), c2 = static_cast<int>(j / L1);
    const int d1 = (r1 - c1 + L1) % L1, d2 = (r2 - c2 + L2) % L2;
    R[row * L + j] = col[static_cast<long>(d2) * L1 + d1];
  }
}

// y = R x for kRows rows per block; mode 0: plain product into out,
// 1: ISTA/FISTA epilogue, 2: ADMM epilogue.
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_dense_gemv(DenseArgs a) {
  __shared__ float red[kRows][2][kThreads];
  const long L = a.L;
  const long row0 = static_cast<long>(blockIdx.x) * kRows;
  const float4* x4 = reinterpret_cast<const float4*>(a.x);
  const long L2v = L / 2;  // float4 = two complex values
  float accr[kRows], acci[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) accr[r] = acci[r] = 0.f;
  for (long j = threadIdx.x; j < L2v; j += kThreads) {
    const float4 xv = x4[j];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const v4f* rp = reinterpret_cast<const v4f*>(a.R + (row0 + r) * L) + j;
      const v4f m = __builtin_nontemporal_load(rp);   // streamed once: do not keep in cache
      accr[r] += m.x * xv.x - m.y * xv.y + m.z * xv.z - m.w * xv.w;
      acci[r] += m.x * xv.y + m.y * xv.x + m.z * xv.w + m.w * xv.z;
    }
  }
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    red[r][0][threadIdx.x] = accr[r];
    red[r][1][threadIdx.x] = acci[r];
  }
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
#pragma unroll
      for (int r = 0; r < kRows; ++r) {
        red[r][0][threadIdx.x] += red[r][0][threadIdx.x + s];
        red[r][1][threadIdx.x] += red[r][1][threadIdx.x + s];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < kRows) {
    const long row = row0 + threadIdx.x;
    const float2 u = make_float2(red[threadIdx.x][0][0], red[threadIdx.x][1][0]);
    if constexpr (MODE == 0) {
      a.out[row] = u;
    } else if constexpr (MODE == 1) {
      // c = S_kappa(R z + mu b); z_next = c + beta (c - c_prev)
      const float2 c = shrink_d(make_float2(u.x + a.rhs[row].x, u.y + a.rhs[row].y), a.kappa);
      const float2 cp = a.state[row];
      a.state[row] = c;
      a.out[row] = make_float2(c.x + a.beta * (c.x - cp.x), c.y + a.beta * (c.y - cp.y));
    } else {
      // c = w + rho (G + rho I)^-1 (z - v); z = S(c + v); v += c - z; next input z - v
      const float2 c = make_float2(a.rhs[row].x + a.rho * u.x, a.rhs[row].y + a.rho * u.y);
      const float2 v = a.state[row];
      const float2 z = shrink_d(make_float2(c.x + v.x, c.y + v.y), a.kappa);
      const float2 vn = make_float2(v.x + c.x - z.x, v.y + c.y - z.y);
      a.state[row] = vn;
      if (a.out_z) a.out_z[row] = z;
      a.out[row] = make_float2(z.x - vn.x, z.y - vn.y);
    }
  }
}

}  // namespace

int launch_dense_build(const float2* col, int L1, int L2, float2* R, hipStream_t s) {
  const long L = static_cast<long>(L1) * L2;
  long by = (L + 255) / 256;
  if (by > 64) by = 64;
  const dim3 grid(static_cast<unsigned>(L), static_cast<unsigned>(by));
  hipLaunchKernelGGL(k_dense_build, grid, dim3(256), 0, s, col, L1, L2, R);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_dense_gemv(int mode, const DenseArgs& a, hipStream_t s) {
  if (a.L % kRows != 0 || a.L % 2 != 0) return -1;
  const dim3 grid(static_cast<unsigned>(a.L / kRows));
  switch (mode) {
    case 0: hipLaunchKernelGGL(k_dense_gemv<0>, grid, dim3(kThreads), 0, s, a); break;
    case 1: hipLaunchKernelGGL(k_dense_gemv<1>, grid, dim3(kThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_dense_gemv<2>, grid, dim3(kThreads), 0, s, a); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace bccb
