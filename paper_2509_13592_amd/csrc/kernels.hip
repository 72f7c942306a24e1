// Scatter, reduction and fill kernels, and the per-length pass dispatch.
#include "fft_device.h"
#include "kernels.h"

namespace bccb {

namespace {

__device__ __forceinline__ bool finite2(float2 v) {
  return __builtin_isfinite(v.x) && __builtin_isfinite(v.y);
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

__global__ void k_scatter_batch(const SceneDesc* __restrict__ desc, int L1, int L2, float2* __restrict__ S,
                                int* flag) {
  const long L = static_cast<long>(L1) * L2;
  const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int scene = blockIdx.y;
  if (idx >= L) return;
  const SceneDesc d = desc[scene];
  const int k1 = static_cast<int>(idx % L1), k2 = static_cast<int>(idx / L1);
  float2 acc = make_float2(0.f, 0.f);
  bool ok = true;
  for (int m2 = k2; m2 < d.M2; m2 += L2) {
    for (int m1 = k1; m1 < d.M1; m1 += L1) {
      const int s = d.sensor_of[m2 * d.M1 + m1];
      if (s >= 0) {
        const float2 yv = d.y[s];
        ok = ok && finite2(yv);
        if ((m1 + m2) & 1) acc = make_float2(acc.x - yv.x, acc.y - yv.y);
        else acc = make_float2(acc.x + yv.x, acc.y + yv.y);
      }
    }
  }
  if (!ok && flag) *flag = 1;
  S[scene * L + idx] = make_float2(acc.x * d.scale, acc.y * d.scale);
}

__global__ void k_gather_batch(const SceneDesc* __restrict__ desc, long L, const float2* __restrict__ src) {
  const int scene = blockIdx.y;
  float2* out = desc[scene].out;
  for (long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x; i < L; i += static_cast<long>(gridDim.x) * blockDim.x)
    out[i] = src[scene * L + i];
}

__global__ void k_sup_rhs(const SupRhsDesc* __restrict__ desc, const int* __restrict__ src_ptr,
                          const int* __restrict__ src, float2* __restrict__ rhs, int* flag) {
  const SupRhsDesc d = desc[blockIdx.y];
  const int jl = blockIdx.x * blockDim.x + threadIdx.x;
  if (jl >= d.nentries) return;
  const int j = d.entry_off + jl;
  float2 acc = make_float2(0.f, 0.f);
  bool ok = true;
  for (int q = src_ptr[j]; q < src_ptr[j + 1]; ++q) {
    const int code = src[q];
    const float2 yv = d.y[code >> 1];
    ok = ok && finite2(yv);
    if (code & 1) acc = make_float2(acc.x - yv.x, acc.y - yv.y);
    else acc = make_float2(acc.x + yv.x, acc.y + yv.y);
  }
  if (!ok && flag) *flag = 1;
  rhs[d.rhs_off + jl] = make_float2(acc.x * d.scale, acc.y * d.scale);
}

__global__ void k_fill(float2* p, long n) {
  for (long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * blockDim.x)
    p[i] = make_float2(0.f, 0.f);
}

__global__ void k_fill_int(int* p, long n, int value) {
  for (long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * blockDim.x)
    p[i] = value;
}

__global__ void k_momentum(float2* __restrict__ out, const float2* __restrict__ a, const float2* __restrict__ b,
                           float beta, long L, const int* __restrict__ map) {
  const int s = map ? map[blockIdx.y] : static_cast<int>(blockIdx.y);
  const size_t off = static_cast<size_t>(s) * L;
  for (long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x; i < L; i += static_cast<long>(gridDim.x) * blockDim.x) {
    const float2 x = a[off + i], y = b[off + i];
    out[off + i] = make_float2(x.x + beta * (x.x - y.x), x.y + beta * (x.y - y.y));
  }
}

__global__ void k_copy(float2* dst, const float2* src, long n) {
  for (long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += static_cast<long>(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

// Streaming copy in 16-byte vectors (the achievable-bandwidth ceiling of the device):
// each thread keeps U loads in flight before storing, consecutive threads take
// consecutive vectors, the grid strides over the rest.  NT: non-temporal hints.
typedef float v4f_t __attribute__((ext_vector_type(4)));
template <int U, bool NT>
__global__ __launch_bounds__(256) void k_stream_copy(const v4f_t* __restrict__ src, v4f_t* __restrict__ dst, long n) {
  const long stride = static_cast<long>(gridDim.x) * blockDim.x;
  long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < n; i += U * stride) {
    v4f_t r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) r[u] = NT ? __builtin_nontemporal_load(src + i + u * stride) : src[i + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (NT) __builtin_nontemporal_store(r[u], dst + i + u * stride);
      else dst[i + u * stride] = r[u];
    }
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Dispatch
// ---------------------------------------------------------------------------
}  // namespace

int launch_row(int N, const PassCfg& c, int mode, const RowArgs& a0, hipStream_t s) {
  RowArgs a = a0;
  a.spread = c.spread;
  switch (N) {
    case 8: return row_launch_8(c.E, mode, a, c.rpb, s);
    case 16: return row_launch_16(c.E, mode, a, c.rpb, s);
    case 32: return row_launch_32(c.E, mode, a, c.rpb, s);
    case 64: return row_launch_64(c.E, mode, a, c.rpb, s);
    case 128: return row_launch_128(c.E, mode, a, c.rpb, s);
    case 256: return row_launch_256(c.E, mode, a, c.rpb, s);
    case 512: return row_launch_512(c.E, mode, a, c.rpb, s);
    case 1024: return row_launch_1024(c.E, mode, a, c.rpb, s);
    default: return -2;
  }
}

int launch_col(int N, const PassCfg& c, int mode, const ColArgs& a0, hipStream_t s) {
  ColArgs a = a0;
  a.spread = c.spread;
  switch (N) {
    case 8: return col_launch_8(c.E, mode, a, c.W, s);
    case 16: return col_launch_16(c.E, mode, a, c.W, s);
    case 32: return col_launch_32(c.E, mode, a, c.W, s);
    case 64: return col_launch_64(c.E, mode, a, c.W, s);
    case 128: return col_launch_128(c.E, mode, a, c.W, s);
    case 256: return col_launch_256(c.E, mode, a, c.W, s);
    case 512: return col_launch_512(c.E, mode, a, c.W, s);
    case 1024: return col_launch_1024(c.E, mode, a, c.W, s);
    default: return -2;
  }
}

int lista_launch(int N, int which, const void* args, int E, int rpb_or_w, int groups, hipStream_t s) {
  switch (N) {
    case 8: return lista_launch_8(which, args, E, rpb_or_w, groups, s);
    case 16: return lista_launch_16(which, args, E, rpb_or_w, groups, s);
    case 32: return lista_launch_32(which, args, E, rpb_or_w, groups, s);
    case 64: return lista_launch_64(which, args, E, rpb_or_w, groups, s);
    case 128: return lista_launch_128(which, args, E, rpb_or_w, groups, s);
    case 256: return lista_launch_256(which, args, E, rpb_or_w, groups, s);
    case 512: return lista_launch_512(which, args, E, rpb_or_w, groups, s);
    case 1024: return lista_launch_1024(which, args, E, rpb_or_w, groups, s);
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

int launch_scatter_batch(const SceneDesc* desc, int n, int L1, int L2, float2* S, int* flag, hipStream_t s) {
  if (n <= 0) return 0;
  const long L = static_cast<long>(L1) * L2;
  const dim3 grid(static_cast<unsigned>((L + 255) / 256), static_cast<unsigned>(n));
  hipLaunchKernelGGL(k_scatter_batch, grid, dim3(256), 0, s, desc, L1, L2, S, flag);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_gather_batch(const SceneDesc* desc, int n, long L, const float2* src, hipStream_t s) {
  if (n <= 0) return 0;
  long bx = (L + 255) / 256;
  if (bx > 64) bx = 64;
  const dim3 grid(static_cast<unsigned>(bx), static_cast<unsigned>(n));
  hipLaunchKernelGGL(k_gather_batch, grid, dim3(256), 0, s, desc, L, src);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_sup_rhs(const SupRhsDesc* desc, int nscenes, int max_entries, const int* src_ptr, const int* src,
                   float2* rhs, int* flag, hipStream_t s) {
  if (nscenes <= 0 || max_entries <= 0) return 0;
  const dim3 grid(static_cast<unsigned>((max_entries + 255) / 256), static_cast<unsigned>(nscenes));
  hipLaunchKernelGGL(k_sup_rhs, grid, dim3(256), 0, s, desc, src_ptr, src, rhs, flag);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_fill(float2* p, long n, hipStream_t s) {
  long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) return 0;
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, p, n);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_fill_int(int* p, long n, int value, hipStream_t s) {
  long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) return 0;
  hipLaunchKernelGGL(k_fill_int, dim3(blocks), dim3(256), 0, s, p, n, value);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_momentum(float2* out, const float2* a, const float2* b, float beta, long L, int n, const int* map,
                    hipStream_t s) {
  if (n <= 0) return 0;
  long bx = (L + 255) / 256;
  if (bx > 64) bx = 64;
  hipLaunchKernelGGL(k_momentum, dim3(static_cast<unsigned>(bx), static_cast<unsigned>(n)), dim3(256), 0, s, out, a, b,
                     beta, L, map);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_copy(float2* dst, const float2* src, long n, hipStream_t s) {
  long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) return 0;
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, dst, src, n);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_stream_copy(const void* src, void* dst, long n16, int variant, hipStream_t s) {
  if (n16 <= 0) return 0;
  // variant: bits 0-1 select 1, 2, 4 or 8 loads in flight per thread, bit 2 the non-temporal
  // hints, bits 3-5 the workgroups per CU (1 << k)
  const int U = 1 << (variant & 3);
  const bool nt = (variant >> 2) & 1;
  long blocks = static_cast<long>(256) << ((variant >> 3) & 7);
  const long need = (n16 + 255) / 256;
  if (blocks > need) blocks = need;
  const dim3 g(static_cast<unsigned>(blocks)), b(256);
  const v4f_t* sp = static_cast<const v4f_t*>(src);
  v4f_t* dp = static_cast<v4f_t*>(dst);
  switch (U * 2 + (nt ? 1 : 0)) {
    case 2: hipLaunchKernelGGL((k_stream_copy<1, false>), g, b, 0, s, sp, dp, n16); break;
    case 3: hipLaunchKernelGGL((k_stream_copy<1, true>), g, b, 0, s, sp, dp, n16); break;
    case 4: hipLaunchKernelGGL((k_stream_copy<2, false>), g, b, 0, s, sp, dp, n16); break;
    case 5: hipLaunchKernelGGL((k_stream_copy<2, true>), g, b, 0, s, sp, dp, n16); break;
    case 8: hipLaunchKernelGGL((k_stream_copy<4, false>), g, b, 0, s, sp, dp, n16); break;
    case 9: hipLaunchKernelGGL((k_stream_copy<4, true>), g, b, 0, s, sp, dp, n16); break;
    case 16: hipLaunchKernelGGL((k_stream_copy<8, false>), g, b, 0, s, sp, dp, n16); break;
    default: hipLaunchKernelGGL((k_stream_copy<8, true>), g, b, 0, s, sp, dp, n16); break;
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace bccb
