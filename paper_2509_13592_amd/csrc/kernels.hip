// BCCB Gram-matvec passes and fused LASSO epilogues for gfx950.
//
// The product R c = IDFT2(Omega . DFT2(C)) of eq. (23) is split into a row pass
// (transforms along l1, contiguous) and a column pass (transforms along l2,
// stride L1).  Grids are [L2][L1] row-major, c(l1 + l2*L1) = C(l1, l2)
// (Sec. II-A, reading R9).  One solver iteration is
//   column pass: DFT_cols -> multiply by the BCCB spectrum -> IDFT_cols
//   row pass   : IDFT_rows -> proximal/momentum/ADMM update -> DFT_rows
// so the state crosses HBM once per pass and the spectral multiply, the soft
// threshold (eq. (9)), the FISTA momentum (eqs. (10)-(12)) and the ADMM updates
// (eqs. (13)-(15)) never take a pass of their own.
#include "fft_device.h"
#include "kernels.h"

namespace bccb {

namespace {

constexpr int kRowThreads = 256;

__device__ __forceinline__ bool finite2(float2 v) {
  return __builtin_isfinite(v.x) && __builtin_isfinite(v.y);
}

// Complex soft threshold S_k(z) = z max(1 - k/|z|, 0), zero for |z| <= k (R3).
__device__ __forceinline__ float2 shrink(float2 z, float k) {
  const float a2 = z.x * z.x + z.y * z.y;
  if (!(a2 > k * k)) return make_float2(0.f, 0.f);
  const float f = 1.f - k / sqrtf(a2);
  return make_float2(z.x * f, z.y * f);
}

// ---------------------------------------------------------------------------
// Row pass
// ---------------------------------------------------------------------------
template <int N, int MODE>
__global__ __launch_bounds__(kRowThreads) void k_row(RowArgs a) {
  using F = FFT<N>;
  constexpr int T = F::T, E = F::E;
  constexpr int R = kRowThreads / T;                 // rows per block
  __shared__ float2 sm[R * F::LDS];
  __shared__ float2 stw[N];

  const int tid = threadIdx.x;
  for (int j = tid; j < N; j += kRowThreads) stw[j] = a.tw[j];
  const int r = tid / T, t = tid % T;
  const int row = blockIdx.x * R + r;
  const bool active = row < a.nrows;
  float2* smr = sm + r * F::LDS;
  const size_t base = static_cast<size_t>(active ? row : 0) * N;
  float2 v[E];
  __syncthreads();

  if constexpr (MODE == ROW_FWD) {
    bool ok = true;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      float2 x = make_float2(0.f, 0.f);
      if (active && a.src) x = a.src[base + F::in_index(t, e)];
      ok = ok && finite2(x);
      v[e] = x;
    }
    if (!ok && a.flag) *a.flag = 1;
    F::forward(v, t, stw, smr, 1);
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) a.xy[base + F::out_index(t, e)] = v[e];
    }
  } else if constexpr (MODE == ROW_INV) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = active ? a.xy[base + F::out_index(t, e)] : make_float2(0.f, 0.f);
    F::inverse(v, t, stw, smr, 1);
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) a.dst[base + F::in_index(t, e)] = cscale(v[e], a.scale);
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = active ? a.xy[base + F::out_index(t, e)] : make_float2(0.f, 0.f);
    F::inverse(v, t, stw, smr, 1);
    const int scene = active ? row / a.rows_per_scene : 0;
    const float kappa = a.kscale ? a.kappa * a.kscale[scene] : a.kappa;
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const size_t idx = base + F::in_index(t, e);
        if constexpr (MODE == ROW_ISTA) {
          const float2 c = shrink(cadd(v[e], a.rhs[idx]), kappa);
          if (a.last) a.out_c[idx] = c;
          v[e] = c;
        } else if constexpr (MODE == ROW_FISTA) {
          const float2 c = shrink(cadd(v[e], a.rhs[idx]), kappa);
          const float2 cp = a.state[idx];
          a.state[idx] = c;
          v[e] = make_float2(c.x + a.beta * (c.x - cp.x), c.y + a.beta * (c.y - cp.y));
        } else {  // ROW_ADMM
          const float2 c = cadd(a.rhs[idx], v[e]);
          const float2 vv = a.state[idx];
          const float2 z = shrink(cadd(c, vv), kappa);
          const float2 vn = csub(cadd(vv, c), z);
          a.state[idx] = vn;
          if (a.last) {
            a.out_z[idx] = z;
            if (a.out_c) a.out_c[idx] = c;
          }
          v[e] = csub(z, vn);
        }
      }
    }
    if (!a.last) {
      F::forward(v, t, stw, smr, 1);
      if (active) {
#pragma unroll
        for (int e = 0; e < E; ++e) a.xy[base + F::out_index(t, e)] = v[e];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Column pass: a block owns W adjacent columns of one scene; lane = c + W*t.
// ---------------------------------------------------------------------------
template <int N>
struct ColCfg {
  static constexpr int T = FFT<N>::T;
  static constexpr int WMAX = 256 / T;
};

template <int N, int MODE>
__global__ __launch_bounds__(256) void k_col(ColArgs a, int W) {
  using F = FFT<N>;
  constexpr int T = F::T, E = F::E;
  constexpr int WMAX = ColCfg<N>::WMAX;
  __shared__ float2 sm[WMAX * F::LDS];
  __shared__ float2 stw[N];

  const int tid = threadIdx.x;
  const int nthreads = W * T;
  for (int j = tid; j < N; j += nthreads) stw[j] = a.tw[j];
  const int c = tid % W, t = tid / W;
  const int strips = a.L1 / W;
  const int scene = blockIdx.x / strips;
  const int col = (blockIdx.x % strips) * W + c;
  const size_t plane = static_cast<size_t>(N) * a.L1;
  float2* g = a.xy + scene * plane + col;
  float2* sms = sm + c;
  float2 v[E];
  __syncthreads();

  constexpr bool kFwd = (MODE == COL_FWD || MODE == COL_FILTER_AFFINE || MODE == COL_FILTER_ADMM ||
                         MODE == COL_FILTER_CPLX);
  constexpr bool kInv = (MODE != COL_FWD);
  constexpr bool kMul = (MODE != COL_FWD && MODE != COL_INV);

  if constexpr (kFwd) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = g[static_cast<size_t>(F::in_index(t, e)) * a.L1];
    F::forward(v, t, stw, sms, W);
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = g[static_cast<size_t>(F::out_index(t, e)) * a.L1];
  }

  if constexpr (kMul) {
    if constexpr (MODE == COL_FILTER_CPLX) {
      const float2* m = a.mulc + scene * a.mulc_stride + col;
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = cmul(v[e], m[static_cast<size_t>(F::out_index(t, e)) * a.L1]);
    } else {
      const float* om = a.omega + scene * a.omega_stride + col;
      if constexpr (MODE == COL_FILTER_AFFINE || MODE == COL_MULINV_AFFINE) {
        const float2 ab = a.coef[scene];
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const float m = ab.x + ab.y * om[static_cast<size_t>(F::out_index(t, e)) * a.L1];
          v[e] = cscale(v[e], m);
        }
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const float m = a.scale / (om[static_cast<size_t>(F::out_index(t, e)) * a.L1] + a.rho);
          v[e] = cscale(v[e], m);
        }
      }
    }
  }

  if constexpr (kInv) {
    F::inverse(v, t, stw, sms, W);
    const float s = (MODE == COL_INV) ? a.scale : 1.f;
#pragma unroll
    for (int e = 0; e < E; ++e) g[static_cast<size_t>(F::in_index(t, e)) * a.L1] = cscale(v[e], s);
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) g[static_cast<size_t>(F::out_index(t, e)) * a.L1] = v[e];
  }
}

// ---------------------------------------------------------------------------
// Scatter of the snapshot onto the spectral grid (A^H y, reading R11)
// ---------------------------------------------------------------------------
__global__ void k_scatter(const float2* __restrict__ y, const int* __restrict__ sensor_of, int M1,
                          int M2, int L1, int L2, float scale, float2* __restrict__ S, int* flag) {
  const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<long>(L1) * L2) return;
  const int k1 = static_cast<int>(idx % L1), k2 = static_cast<int>(idx / L1);
  float2 acc = make_float2(0.f, 0.f);
  bool ok = true;
  for (int m2 = k2; m2 < M2; m2 += L2) {
    for (int m1 = k1; m1 < M1; m1 += L1) {
      const int s = sensor_of[m2 * M1 + m1];
      if (s >= 0) {
        const float2 yv = y[s];
        ok = ok && finite2(yv);
        if ((m1 + m2) & 1) acc = csub(acc, yv);
        else acc = cadd(acc, yv);
      }
    }
  }
  if (!ok && flag) *flag = 1;
  S[idx] = cscale(acc, scale);
}

// ---------------------------------------------------------------------------
// Reductions (FP32 inputs, FP64 accumulation, one partial per block)
// ---------------------------------------------------------------------------
template <int NV>
__device__ void block_reduce(double (&val)[NV], const bool (&is_max)[NV], double* out) {
  __shared__ double red[NV][256];
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < NV; ++k) red[k][tid] = val[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
#pragma unroll
      for (int k = 0; k < NV; ++k)
        red[k][tid] = is_max[k] ? fmax(red[k][tid], red[k][tid + s]) : red[k][tid] + red[k][tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) out[blockIdx.x * NV + k] = red[k][0];
  }
}

__global__ __launch_bounds__(256) void k_resid(const float2* spec, const float2* y, const int2* sensors,
                                               int M, int L1, int L2, double* partial) {
  double acc[1] = {0.0};
  const bool mx[1] = {false};
  for (int m = blockIdx.x * 256 + threadIdx.x; m < M; m += gridDim.x * 256) {
    const int2 s = sensors[m];
    const float2 X = spec[(s.y % L2) * L1 + (s.x % L1)];
    const double sg = ((s.x + s.y) & 1) ? -1.0 : 1.0;
    const double dr = static_cast<double>(y[m].x) - sg * X.x;
    const double di = static_cast<double>(y[m].y) - sg * X.y;
    acc[0] += dr * dr + di * di;
  }
  block_reduce<1>(acc, mx, partial);
}

__global__ __launch_bounds__(256) void k_kkt(const float2* c, const float2* b, const float2* gc, float tau,
                                             long L, double* partial) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const bool mx[4] = {false, true, false, false};
  for (long l = static_cast<long>(blockIdx.x) * 256 + threadIdx.x; l < L; l += static_cast<long>(gridDim.x) * 256) {
    const double cr = c[l].x, ci = c[l].y;
    const double br = b[l].x, bi = b[l].y;
    const double gr = br - gc[l].x, gi = bi - gc[l].y;
    const double ac = sqrt(cr * cr + ci * ci);
    double e;
    if (ac > 0.0) {
      const double er = gr - tau * cr / ac, ei = gi - tau * ci / ac;
      e = sqrt(er * er + ei * ei);
    } else {
      e = fmax(sqrt(gr * gr + gi * gi) - tau, 0.0);
    }
    acc[0] += e * e;
    acc[1] = fmax(acc[1], e);
    acc[2] += ac;
    acc[3] += br * br + bi * bi;
  }
  block_reduce<4>(acc, mx, partial);
}

__global__ __launch_bounds__(256) void k_absmax(const float2* b, long L, double* partial) {
  double acc[1] = {0.0};
  const bool mx[1] = {true};
  for (long l = static_cast<long>(blockIdx.x) * 256 + threadIdx.x; l < L; l += static_cast<long>(gridDim.x) * 256) {
    const double br = b[l].x, bi = b[l].y;
    acc[0] = fmax(acc[0], sqrt(br * br + bi * bi));
  }
  block_reduce<1>(acc, mx, partial);
}

__global__ void k_fill(float2* p, long n) {
  for (long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * blockDim.x)
    p[i] = make_float2(0.f, 0.f);
}

__global__ void k_copy(float2* dst, const float2* src, long n) {
  for (long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Dispatch
// ---------------------------------------------------------------------------
template <int N>
int row_dispatch(int mode, const RowArgs& a, hipStream_t s) {
  constexpr int R = kRowThreads / FFT<N>::T;
  const int blocks = (a.nrows + R - 1) / R;
  if (blocks <= 0) return 0;
  switch (mode) {
    case ROW_FWD: hipLaunchKernelGGL((k_row<N, ROW_FWD>), dim3(blocks), dim3(kRowThreads), 0, s, a); break;
    case ROW_INV: hipLaunchKernelGGL((k_row<N, ROW_INV>), dim3(blocks), dim3(kRowThreads), 0, s, a); break;
    case ROW_ISTA: hipLaunchKernelGGL((k_row<N, ROW_ISTA>), dim3(blocks), dim3(kRowThreads), 0, s, a); break;
    case ROW_FISTA: hipLaunchKernelGGL((k_row<N, ROW_FISTA>), dim3(blocks), dim3(kRowThreads), 0, s, a); break;
    case ROW_ADMM: hipLaunchKernelGGL((k_row<N, ROW_ADMM>), dim3(blocks), dim3(kRowThreads), 0, s, a); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

template <int N>
int col_dispatch(int mode, const ColArgs& a, hipStream_t s) {
  constexpr int T = FFT<N>::T;
  const int W = a.L1 < ColCfg<N>::WMAX ? a.L1 : ColCfg<N>::WMAX;
  const int blocks = (a.L1 / W) * a.nscenes;
  if (blocks <= 0) return 0;
  const dim3 grid(blocks), block(W * T);
  switch (mode) {
    case COL_FWD: hipLaunchKernelGGL((k_col<N, COL_FWD>), grid, block, 0, s, a, W); break;
    case COL_INV: hipLaunchKernelGGL((k_col<N, COL_INV>), grid, block, 0, s, a, W); break;
    case COL_FILTER_AFFINE: hipLaunchKernelGGL((k_col<N, COL_FILTER_AFFINE>), grid, block, 0, s, a, W); break;
    case COL_FILTER_ADMM: hipLaunchKernelGGL((k_col<N, COL_FILTER_ADMM>), grid, block, 0, s, a, W); break;
    case COL_FILTER_CPLX: hipLaunchKernelGGL((k_col<N, COL_FILTER_CPLX>), grid, block, 0, s, a, W); break;
    case COL_MULINV_AFFINE: hipLaunchKernelGGL((k_col<N, COL_MULINV_AFFINE>), grid, block, 0, s, a, W); break;
    case COL_MULINV_ADMM: hipLaunchKernelGGL((k_col<N, COL_MULINV_ADMM>), grid, block, 0, s, a, W); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace

int launch_row(int N, int mode, const RowArgs& a, hipStream_t s) {
  switch (N) {
    case 8: return row_dispatch<8>(mode, a, s);
    case 16: return row_dispatch<16>(mode, a, s);
    case 32: return row_dispatch<32>(mode, a, s);
    case 64: return row_dispatch<64>(mode, a, s);
    case 128: return row_dispatch<128>(mode, a, s);
    case 256: return row_dispatch<256>(mode, a, s);
    case 512: return row_dispatch<512>(mode, a, s);
    case 1024: return row_dispatch<1024>(mode, a, s);
    default: return -2;
  }
}

int launch_col(int N, int mode, const ColArgs& a, hipStream_t s) {
  switch (N) {
    case 8: return col_dispatch<8>(mode, a, s);
    case 16: return col_dispatch<16>(mode, a, s);
    case 32: return col_dispatch<32>(mode, a, s);
    case 64: return col_dispatch<64>(mode, a, s);
    case 128: return col_dispatch<128>(mode, a, s);
    case 256: return col_dispatch<256>(mode, a, s);
    case 512: return col_dispatch<512>(mode, a, s);
    case 1024: return col_dispatch<1024>(mode, a, s);
    default: return -2;
  }
}

int launch_scatter(const float2* y, const int* sensor_of, int M1, int M2, int L1, int L2, float scale,
                   float2* S, int* flag, hipStream_t s) {
  const long L = static_cast<long>(L1) * L2;
  const int blocks = static_cast<int>((L + 255) / 256);
  hipLaunchKernelGGL(k_scatter, dim3(blocks), dim3(256), 0, s, y, sensor_of, M1, M2, L1, L2, scale, S, flag);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_resid(const float2* spec, const float2* y, const int2* sensors, int M, int L1, int L2,
                 double* partial, int* nblocks, hipStream_t s) {
  int blocks = (M + 255) / 256;
  if (blocks > kReduceBlocks) blocks = kReduceBlocks;
  if (blocks < 1) blocks = 1;
  *nblocks = blocks;
  hipLaunchKernelGGL(k_resid, dim3(blocks), dim3(256), 0, s, spec, y, sensors, M, L1, L2, partial);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_kkt(const float2* c, const float2* b, const float2* gc, float tau, long L, double* partial,
               int* nblocks, hipStream_t s) {
  long blocks = (L + 255) / 256;
  if (blocks > kReduceBlocks) blocks = kReduceBlocks;
  *nblocks = static_cast<int>(blocks);
  hipLaunchKernelGGL(k_kkt, dim3(blocks), dim3(256), 0, s, c, b, gc, tau, L, partial);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_absmax(const float2* b, long L, double* partial, int* nblocks, hipStream_t s) {
  long blocks = (L + 255) / 256;
  if (blocks > kReduceBlocks) blocks = kReduceBlocks;
  *nblocks = static_cast<int>(blocks);
  hipLaunchKernelGGL(k_absmax, dim3(blocks), dim3(256), 0, s, b, L, partial);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_fill(float2* p, long n, hipStream_t s) {
  long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) return 0;
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, p, n);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_copy(float2* dst, const float2* src, long n, hipStream_t s) {
  long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) return 0;
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, dst, src, n);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace bccb
