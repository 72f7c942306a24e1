// Internal launch interface of the learned unrolled FISTA kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace bccb {

constexpr int kListaPerLayer = 52;   // s, theta, Re Delta[5][5], Im Delta[5][5]
constexpr int kSumBlocksPerScene = 16;

int lista_prepare(const float* params, const float* omega, float mu0, int L1, int L2, int K, float2* mulc, float2* omp,
                  float* dscal, hipStream_t s);
int lista_layer_grad(const float2* gm_part, int groups, float2* gm, const float2* omp, const float* omega, int L1,
                     int L2, const float* dscal, const float* params, const double* row_part, int nscenes,
                     const float* tau, double* lg, float mu0, float* grad, hipStream_t s);
int launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps, float bc1,
                float bc2, const float* lr_scale, hipStream_t s);
// per scene {sum |x|^2, sum |x - y|^2} (y nullable); part: n * 16 * 2 doubles; out: n * 2 doubles
int scene_sums(const float2* x, const float2* y, long L, int n, double* part, double* out, hipStream_t s);
int rows_to_scene(const double* part, int rows_per_scene, int n, const int* map, double* out, hipStream_t s);

}  // namespace bccb
