// Harmonic and direction extraction from recovered coefficient grids: bccb_extract_peaks.
//
// Sec. II-A: the support of the sparse estimate c marks the harmonic tuples present, and each
// tuple gives a direction through eq. (2), f1 = gamma1 cos(phi) sin(theta),
// f2 = gamma2 sin(phi) sin(theta).  Two kernels per call:
//   k_peak_candidates: eight grid points per thread; a point whose |c|^2 (re*re + im*im, each
//     product and the sum rounded to FP32, no fused multiply-add) exceeds the threshold and
//     beats its 8 neighbours (equal values: the smaller linear index ranks higher; the grid
//     wraps at half spacing) appends the key (~bits(|c|^2) << 32 | index) to its scene's list;
//   k_peak_select: one workgroup per scene sorts the keys in LDS (bitonic, ascending = the
//     strongest first, ties by index) and, for the first max_peaks, refines the harmonic to
//     the |c|-weighted mean offset of its 3 x 3 neighbourhood, sums the neighbourhood's
//     coefficients as the amplitude and inverts eq. (2).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "plan_internal.h"

namespace bccb {

namespace {

constexpr int kCandCap = 4096;   // local maxima kept per scene (sorted in 32 KB of LDS)

// |c|^2 with each product and the sum rounded on its own: contraction into a fused
// multiply-add (which hipcc does by default, through these intrinsics too) is switched off,
// so the value is the one any IEEE FP32 evaluation of re*re + im*im gives
__device__ __forceinline__ float mag2_rn(float2 v) {
#pragma clang fp contract(off)
  const float a = v.x * v.x;
  const float b = v.y * v.y;
  return a + b;
}

struct GridInfo {
  int L1, L2;
  int wrap;
  float min_mag2;
};


// Is point i of a scene (|c|^2 = v > threshold) a local maximum?  Appends its key if so.
__device__ __forceinline__ void consider_point(const float2* __restrict__ cs, long i, float v, const GridInfo& g,
                                               unsigned long long* __restrict__ cand, int* __restrict__ count,
                                               int scene) {
  const int l1 = static_cast<int>(i % g.L1), l2 = static_cast<int>(i / g.L1);
  bool best = true;
  for (int d2 = -1; d2 <= 1; ++d2) {
    for (int d1 = -1; d1 <= 1; ++d1) {
      if (d1 == 0 && d2 == 0) continue;
      int n1 = l1 + d1, n2 = l2 + d2;
      if (g.wrap) {
        n1 = n1 < 0 ? n1 + g.L1 : (n1 >= g.L1 ? n1 - g.L1 : n1);
        n2 = n2 < 0 ? n2 + g.L2 : (n2 >= g.L2 ? n2 - g.L2 : n2);
      } else if (n1 < 0 || n1 >= g.L1 || n2 < 0 || n2 >= g.L2) {
        continue;
      }
      const long ni = static_cast<long>(n2) * g.L1 + n1;
      const float w = mag2_rn(cs[ni]);
      if (w > v || (w == v && ni < i)) best = false;
    }
  }
  if (!best) return;
  const int slot = atomicAdd(&count[scene], 1);
  if (slot < kCandCap) {
    const unsigned long long key =
        (static_cast<unsigned long long>(~__float_as_uint(v)) << 32) | static_cast<unsigned long long>(i);
    cand[static_cast<long>(scene) * kCandCap + slot] = key;
  }
}

// A block covers 256 x 8 consecutive points of one scene: each thread loads 8 points as four
// 16-byte vectors of two points (VEC, scenes of an even number of points, 16-byte aligned) or
// as 8 single points strided by 256, all loads in flight before any point is tested.
template <bool VEC>
__global__ __launch_bounds__(256) void k_peak_candidates(const float2* __restrict__ c, GridInfo g,
                                                         unsigned long long* __restrict__ cand,
                                                         int* __restrict__ count) {
  constexpr int kPts = 8;
  const int scene = blockIdx.y;
  const long L = static_cast<long>(g.L1) * g.L2;
  const float2* cs = c + static_cast<long>(scene) * L;
  const long block0 = static_cast<long>(blockIdx.x) * (256 * kPts);
  float v[kPts];
  long idx[kPts];
  if constexpr (VEC) {
    const float4* c4 = reinterpret_cast<const float4*>(cs);
#pragma unroll
    for (int k = 0; k < kPts / 2; ++k) {
      const long j = block0 / 2 + 256L * k + threadIdx.x;   // vector j holds points 2j, 2j + 1
      float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
      if (2 * j < L) q = c4[j];
      v[2 * k] = mag2_rn(make_float2(q.x, q.y));
      v[2 * k + 1] = mag2_rn(make_float2(q.z, q.w));
      idx[2 * k] = 2 * j;
      idx[2 * k + 1] = 2 * j + 1;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kPts; ++k) {
      const long i = block0 + 256L * k + threadIdx.x;
      v[k] = i < L ? mag2_rn(cs[i]) : 0.f;
      idx[k] = i;
    }
  }
#pragma unroll
  for (int k = 0; k < kPts; ++k)
    if (idx[k] < L && v[k] > g.min_mag2) consider_point(cs, idx[k], v[k], g, cand, count, scene);
}

struct SelectArgs {
  const float2* c;
  const unsigned long long* cand;
  const int* count;
  bccb_peak* peaks;
  int* counts_out;
  int L1, L2, wrap, max_peaks;
  double gamma1, gamma2;
};

__global__ __launch_bounds__(256) void k_peak_select(SelectArgs a) {
  __shared__ unsigned long long keys[kCandCap];
  const int scene = blockIdx.x;
  const int tid = threadIdx.x;
  const int total = a.count[scene];
  if (total > kCandCap) {   // too many maxima above the threshold: reported, nothing written
    if (tid == 0) a.counts_out[scene] = -1;
    return;
  }
  int P = 1;
  while (P < total) P <<= 1;
  for (int j = tid; j < P; j += blockDim.x)
    keys[j] = j < total ? a.cand[static_cast<long>(scene) * kCandCap + j] : ~0ull;
  __syncthreads();
  // bitonic sort, ascending
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = tid; t < P; t += blockDim.x) {
        const int u = t ^ j;
        if (u > t) {
          const unsigned long long x = keys[t], y = keys[u];
          const bool up = (t & k) == 0;
          if ((x > y) == up) {
            keys[t] = y;
            keys[u] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  const int n = total < a.max_peaks ? total : a.max_peaks;
  if (tid == 0) a.counts_out[scene] = n;
  for (int q = tid; q < n; q += blockDim.x) {
    const unsigned long long key = keys[q];
    const long idx = static_cast<long>(key & 0xffffffffull);
    const float m2 = __uint_as_float(~static_cast<unsigned>(key >> 32));
    const long L = static_cast<long>(a.L1) * a.L2;
    const float2* cs = a.c + static_cast<long>(scene) * L;
    const int l1 = static_cast<int>(idx % a.L1), l2 = static_cast<int>(idx / a.L1);
    float sw = 0.f, s1 = 0.f, s2 = 0.f, ar = 0.f, ai = 0.f;
    for (int d2 = -1; d2 <= 1; ++d2) {
      for (int d1 = -1; d1 <= 1; ++d1) {
        int n1 = l1 + d1, n2 = l2 + d2;
        if (a.wrap) {
          n1 = n1 < 0 ? n1 + a.L1 : (n1 >= a.L1 ? n1 - a.L1 : n1);
          n2 = n2 < 0 ? n2 + a.L2 : (n2 >= a.L2 ? n2 - a.L2 : n2);
        } else if (n1 < 0 || n1 >= a.L1 || n2 < 0 || n2 >= a.L2) {
          continue;
        }
        const float2 v = cs[static_cast<long>(n2) * a.L1 + n1];
        const float w = sqrtf(mag2_rn(v));
        sw += w;
        s1 += w * static_cast<float>(d1);
        s2 += w * static_cast<float>(d2);
        ar += v.x;
        ai += v.y;
      }
    }
    const float o1 = sw > 0.f ? s1 / sw : 0.f, o2 = sw > 0.f ? s2 / sw : 0.f;
    // f_l = -gamma + l 2 gamma / L (eq. (16)) plus the refined offset, in double
    double f1 = -a.gamma1 + (l1 + static_cast<double>(o1)) * (2.0 * a.gamma1 / a.L1);
    double f2 = -a.gamma2 + (l2 + static_cast<double>(o2)) * (2.0 * a.gamma2 / a.L2);
    if (a.wrap) {   // the half-spacing grid is periodic in f with period 1
      f1 = f1 - floor(f1 + 0.5);
      f2 = f2 - floor(f2 + 0.5);
    }
    const double u = f1 / a.gamma1, w = f2 / a.gamma2;
    const double s = u * u + w * w;
    double phi = atan2(w, u);
    if (phi >= 3.14159265358979323846) phi -= 2.0 * 3.14159265358979323846;
    bccb_peak pk;
    pk.index = static_cast<int>(idx);
    pk.mag2 = m2;
    pk.f1 = static_cast<float>(f1);
    pk.f2 = static_cast<float>(f2);
    pk.phi = static_cast<float>(phi);
    pk.theta = s <= 1.0 ? static_cast<float>(asin(sqrt(s))) : __builtin_nanf("");
    pk.amp.re = ar;
    pk.amp.im = ai;
    a.peaks[static_cast<long>(scene) * a.max_peaks + q] = pk;
  }
}

}  // namespace

}  // namespace bccb

using namespace bccb;

extern "C" int bccb_extract_peaks(bccb_plan_t p, const bccb_c32* c, int batch, int max_peaks, float min_mag2,
                                  bccb_peak* peaks, int* counts) {
  if (!p || !c || !peaks || !counts || batch < 1 || batch > 65535 || max_peaks < 1 || max_peaks > 1024)
    return BCCB_E_INVALID;
  if (!(min_mag2 >= 0.f) || !std::isfinite(min_mag2)) return BCCB_E_INVALID;
  const int L1 = p->emb ? p->A1 : p->L1, L2 = p->emb ? p->A2 : p->L2;
  const long L = static_cast<long>(L1) * L2;
  if (L >= (1L << 31)) return BCCB_E_UNSUPPORTED;
  if (p->cand_batch < batch) {
    BCCB_HIP(hipStreamSynchronize(p->stream));   // nothing in flight reads the old lists
    if (p->d_cand) (void)hipFree(p->d_cand);
    if (p->d_ccount) (void)hipFree(p->d_ccount);
    p->d_cand = nullptr;
    p->d_ccount = nullptr;
    p->cand_batch = 0;
    if (hipMalloc(reinterpret_cast<void**>(&p->d_cand), static_cast<size_t>(batch) * kCandCap * 8) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&p->d_ccount), static_cast<size_t>(batch) * sizeof(int)) != hipSuccess)
      return BCCB_E_NOMEM;
    p->cand_batch = batch;
  }
  const hipStream_t s = p->stream;
  BCCB_TRY(kern(launch_fill_int(p->d_ccount, batch, 0, s)));
  GridInfo g;
  g.L1 = L1;
  g.L2 = L2;
  g.wrap = (p->gamma1 == 0.5 && p->gamma2 == 0.5) ? 1 : 0;
  g.min_mag2 = min_mag2;
  const long per_block = 256L * 8;
  const dim3 cgrid(static_cast<unsigned>((L + per_block - 1) / per_block), batch);
  const bool vec = (L % 2 == 0) && (reinterpret_cast<uintptr_t>(c) % 16 == 0);
  if (vec)
    hipLaunchKernelGGL(k_peak_candidates<true>, cgrid, dim3(256), 0, s, reinterpret_cast<const float2*>(c), g,
                       p->d_cand, p->d_ccount);
  else
    hipLaunchKernelGGL(k_peak_candidates<false>, cgrid, dim3(256), 0, s, reinterpret_cast<const float2*>(c), g,
                       p->d_cand, p->d_ccount);
  SelectArgs a;
  a.c = reinterpret_cast<const float2*>(c);
  a.cand = p->d_cand;
  a.count = p->d_ccount;
  a.peaks = peaks;
  a.counts_out = counts;
  a.L1 = L1;
  a.L2 = L2;
  a.wrap = g.wrap;
  a.max_peaks = max_peaks;
  a.gamma1 = p->gamma1;
  a.gamma2 = p->gamma2;
  hipLaunchKernelGGL(k_peak_select, dim3(batch), dim3(256), 0, s, a);
  BCCB_HIP(hipGetLastError());
  BCCB_HIP(hipStreamSynchronize(s));
  return BCCB_OK;
}
