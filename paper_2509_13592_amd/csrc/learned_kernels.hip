// Element-wise and reduction kernels of the learned unrolled FISTA: layer
// spectra from the parameters, parameter gradients, Adam, per-scene sums.
#include "fft_device.h"
#include "kernels.h"
#include "lista.h"

namespace bccb {

namespace {

constexpr int kTaps = 5;
constexpr int kHalf = 2;

template <int NV>
__device__ void block_sum(double (&val)[NV], double* out, bool is_max0 = false) {
  __shared__ double red[NV][256];
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < NV; ++k) red[k][tid] = val[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
#pragma unroll
      for (int k = 0; k < NV; ++k)
        red[k][tid] = (is_max0 && k == 0) ? fmax(red[k][tid], red[k][tid + s]) : red[k][tid] + red[k][tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k] = red[k][0];
  }
}

// Omega'_k = Omega + Delta_k (*) Omega (circular, centred 5x5), mulc_k = (1 - mu_k Omega'_k)/L,
// dscal_k = {theta_k mu_k, mu_k}.
__global__ __launch_bounds__(256) void k_lista_prepare(const float* __restrict__ params, const float* __restrict__ omega,
                                                       float mu0, int L1, int L2, float2* __restrict__ mulc,
                                                       float2* __restrict__ omp, float* __restrict__ dscal) {
  const int k = blockIdx.y;
  const long L = static_cast<long>(L1) * L2;
  const long f = static_cast<long>(blockIdx.x) * 256 + threadIdx.x;
  const float* p = params + k * kListaPerLayer;
  const float mu = p[0] * mu0;
  if (f == 0) {
    dscal[2 * k] = p[1] * mu;
    dscal[2 * k + 1] = mu;
  }
  if (f >= L) return;
  const int k1 = static_cast<int>(f % L1), k2 = static_cast<int>(f / L1);
  float re = omega[f], im = 0.f;
#pragma unroll
  for (int a = -kHalf; a <= kHalf; ++a) {
    const int r2 = ((k2 - a) % L2 + L2) % L2;
#pragma unroll
    for (int b = -kHalf; b <= kHalf; ++b) {
      const int r1 = ((k1 - b) % L1 + L1) % L1;
      const int ti = (a + kHalf) * kTaps + (b + kHalf);
      const float o = omega[static_cast<long>(r2) * L1 + r1];
      re += p[2 + ti] * o;
      im += p[2 + kTaps * kTaps + ti] * o;
    }
  }
  omp[k * L + f] = make_float2(re, im);
  const float invL = 1.f / static_cast<float>(L);
  mulc[k * L + f] = make_float2((1.f - mu * re) * invL, (-mu * im) * invL);
}

__global__ __launch_bounds__(256) void k_sum_groups(const float2* __restrict__ part, int groups, long L,
                                                    float2* __restrict__ out) {
  for (long f = static_cast<long>(blockIdx.x) * 256 + threadIdx.x; f < L; f += static_cast<long>(gridDim.x) * 256) {
    double re = 0.0, im = 0.0;
    for (int g = 0; g < groups; ++g) {
      re += part[g * L + f].x;
      im += part[g * L + f].y;
    }
    out[f] = make_float2(static_cast<float>(re), static_cast<float>(im));
  }
}

// Block 0: -Re sum conj(gm) Omega'_j.  Blocks 1..25: Delta gradient of tap (a, b):
// sum_f (-mu_j gm_f) Omega[f - (a, b)].  Block 26: per-scene threshold and data-term
// sums from the row partials.  out: [27][2] doubles.
__global__ __launch_bounds__(256) void k_lista_layer_grad(const float2* __restrict__ gm, const float2* __restrict__ omp,
                                                          const float* __restrict__ omega, int L1, int L2,
                                                          const float* __restrict__ dscal, const float* __restrict__ params,
                                                          const double* __restrict__ row_part, int nscenes,
                                                          const float* __restrict__ tau, double* __restrict__ out) {
  const long L = static_cast<long>(L1) * L2;
  const int blk = blockIdx.x;
  const double mu = dscal[1];
  double acc[2] = {0.0, 0.0};
  if (blk == 0) {
    for (long f = threadIdx.x; f < L; f += 256) acc[0] -= static_cast<double>(gm[f].x) * omp[f].x + static_cast<double>(gm[f].y) * omp[f].y;
  } else if (blk <= kTaps * kTaps) {
    const int ti = blk - 1;
    const int a = ti / kTaps - kHalf, b = ti % kTaps - kHalf;
    for (long f = threadIdx.x; f < L; f += 256) {
      const int k1 = static_cast<int>(f % L1), k2 = static_cast<int>(f / L1);
      const int r2 = ((k2 - a) % L2 + L2) % L2, r1 = ((k1 - b) % L1 + L1) % L1;
      const double o = omega[static_cast<long>(r2) * L1 + r1];
      acc[0] -= mu * gm[f].x * o;
      acc[1] -= mu * gm[f].y * o;
    }
  } else {
    const double theta = params[1];
    for (int s = threadIdx.x; s < nscenes; s += 256) {
      double dk = 0.0, db = 0.0;
      for (int r = 0; r < L2; ++r) {
        dk += row_part[2 * (static_cast<long>(s) * L2 + r)];
        db += row_part[2 * (static_cast<long>(s) * L2 + r) + 1];
      }
      acc[0] += dk * mu * tau[s];            // d loss / d theta_j
      acc[1] += dk * theta * tau[s] + db;    // d loss / d mu_j (threshold and mu_j b terms)
    }
  }
  block_sum<2>(acc, out + 2 * blk);
}

__global__ void k_lista_grad_write(const double* __restrict__ lg, float mu0, float* __restrict__ grad) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double dmu = lg[0] + lg[2 * (kTaps * kTaps + 1) + 1];
  grad[0] = static_cast<float>(dmu * mu0);
  grad[1] = static_cast<float>(lg[2 * (kTaps * kTaps + 1)]);
  for (int t = 0; t < kTaps * kTaps; ++t) {
    grad[2 + t] = static_cast<float>(lg[2 * (1 + t)]);
    grad[2 + kTaps * kTaps + t] = static_cast<float>(lg[2 * (1 + t) + 1]);
  }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int n, float lr, float b1, float b2, float eps, float bc1, float bc2,
                       const float* __restrict__ lr_scale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float rate = lr_scale ? lr * lr_scale[i] : lr;
  p[i] -= rate * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// per (scene, block): {sum |x|^2, sum |x - y|^2}
__global__ __launch_bounds__(256) void k_scene_sums(const float2* __restrict__ x, const float2* __restrict__ y, long L,
                                                    double* __restrict__ part) {
  const int s = blockIdx.y;
  double acc[2] = {0.0, 0.0};
  const float2* xs = x + s * L;
  const float2* ys = y ? y + s * L : nullptr;
  for (long i = static_cast<long>(blockIdx.x) * 256 + threadIdx.x; i < L; i += static_cast<long>(gridDim.x) * 256) {
    const double xr = xs[i].x, xi = xs[i].y;
    acc[0] += xr * xr + xi * xi;
    if (ys) {
      const double dr = xr - ys[i].x, di = xi - ys[i].y;
      acc[1] += dr * dr + di * di;
    }
  }
  block_sum<2>(acc, part + 2 * (static_cast<long>(s) * gridDim.x + blockIdx.x));
}

__global__ void k_scene_sums_final(const double* __restrict__ part, int nb, int n, double* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  double a = 0.0, b = 0.0;
  for (int k = 0; k < nb; ++k) {
    a += part[2 * (static_cast<long>(s) * nb + k)];
    b += part[2 * (static_cast<long>(s) * nb + k) + 1];
  }
  out[2 * s] = a;
  out[2 * s + 1] = b;
}

// out[phys scene] = sum of the scene's row partials, for the n logical scenes of the map
__global__ void k_rows_to_scene(const double* __restrict__ part, int rows_per_scene, int n, const int* __restrict__ map,
                                double* __restrict__ out) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n) return;
  const int s = map ? map[l] : l;
  double a = 0.0;
  for (int r = 0; r < rows_per_scene; ++r) a += part[static_cast<long>(s) * rows_per_scene + r];
  out[s] = a;
}

}  // namespace

constexpr int kSumBlocks = 16;

int lista_prepare(const float* params, const float* omega, float mu0, int L1, int L2, int K, float2* mulc, float2* omp,
                  float* dscal, hipStream_t s) {
  const long L = static_cast<long>(L1) * L2;
  hipLaunchKernelGGL(k_lista_prepare, dim3(static_cast<unsigned>((L + 255) / 256), K), dim3(256), 0, s, params, omega,
                     mu0, L1, L2, mulc, omp, dscal);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int lista_layer_grad(const float2* gm_part, int groups, float2* gm, const float2* omp, const float* omega, int L1,
                     int L2, const float* dscal, const float* params, const double* row_part, int nscenes,
                     const float* tau, double* lg, float mu0, float* grad, hipStream_t s) {
  const long L = static_cast<long>(L1) * L2;
  long bx = (L + 255) / 256;
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(k_sum_groups, dim3(static_cast<unsigned>(bx)), dim3(256), 0, s, gm_part, groups, L, gm);
  hipLaunchKernelGGL(k_lista_layer_grad, dim3(kTaps * kTaps + 2), dim3(256), 0, s, gm, omp, omega, L1, L2, dscal, params,
                     row_part, nscenes, tau, lg);
  hipLaunchKernelGGL(k_lista_grad_write, dim3(1), dim3(1), 0, s, lg, mu0, grad);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps, float bc1,
                float bc2, const float* lr_scale, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, bc1, bc2, lr_scale);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int scene_sums(const float2* x, const float2* y, long L, int n, double* part, double* out, hipStream_t s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(k_scene_sums, dim3(kSumBlocks, n), dim3(256), 0, s, x, y, L, part);
  hipLaunchKernelGGL(k_scene_sums_final, dim3((n + 255) / 256), dim3(256), 0, s, part, kSumBlocks, n, out);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int rows_to_scene(const double* part, int rows_per_scene, int n, const int* map, double* out, hipStream_t s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(k_rows_to_scene, dim3((n + 255) / 256), dim3(256), 0, s, part, rows_per_scene, n, map, out);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace bccb
