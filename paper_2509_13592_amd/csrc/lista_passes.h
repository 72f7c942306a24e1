// Stockham-based passes of the learned unrolled FISTA backward and of the
// per-scene KKT check (templates, instantiated per length in passes_n.hip).
//
// Backward of layer j (reading R24 of the learned extension; each layer is
// u_j = IDFT2(m_j . DFT2(z_j)) + mu_j b, c_j = S_{kappa_j}(u_j),
// z_{j+1} = c_j + beta_j (c_j - c_{j-1})):
//   row pass : zbar_{j+1} = IDFT_rows(column-pass output)       (unless j = K-1)
//              cbar_j = (1 + beta_j) zbar_{j+1} - beta_{j+1} zbar_{j+2} (+ loss gradient at j = K-1)
//              ubar_j = S'_{kappa_j}(u_j)^T cbar_j, per-row partials of dkappa and <ubar, b>
//              A = DFT_rows(ubar_j),  Z = DFT_rows(z_j)
//   col pass : DFT_cols of A and Z; gm += A conj(Z) / L (summed over the scene group);
//              A = IDFT_cols(conj(m_j)/L . A)  -> row-spectral zbar_j
#pragma once

#include "passes.h"

namespace bccb {

// Deterministic sum of NV doubles over the T threads of each row of the block.
// red: rpb*T*NV doubles of LDS.  Returns the sums in thread t == 0 of the row.
template <int NV, int T>
__device__ __forceinline__ void row_sum(double* red, int r, int t, double (&val)[NV]) {
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) red[(r * T + t) * NV + k] = val[k];
  __syncthreads();
  if (t == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int i = 0; i < T; ++i) s += red[(r * T + i) * NV + k];
      val[k] = s;
    }
  }
}

template <int N, int E>
__global__ __launch_bounds__(256) void k_lista_bwd_row(ListaBwdRowArgs a, int rpb) {
  using F = Stockham<N, E>;
  constexpr int T = F::T;
  extern __shared__ float2 lds[];
  float2* stw = lds + rpb * fft_area(N);
  double* red = reinterpret_cast<double*>(stw + N);
  const int tid = threadIdx.x;
  const int nthreads = rpb * T;
  const int r = tid / T, t = tid - (tid / T) * T;
  const int row = blockIdx.x * rpb + r;
  const bool active = row < a.nrows;
  const int prow = active ? row : 0;
  const int scene = prow / a.rows_per_scene;
  float2* sm = lds + r * fft_area(N);
  const size_t base = static_cast<size_t>(prow) * N;
  const float2 zero = make_float2(0.f, 0.f);

  // unconditional loads from valid rows, zeroed afterwards (no flat address selects)
  float2 v[E], zb2[E], u[E], bb[E], c1[E], c2[E], lo[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const size_t ii = base + F::in_index(t, e);
    u[e] = a.U[ii];
    bb[e] = a.b[ii];
    v[e] = zero;
    zb2[e] = zero;
    c1[e] = zero;
    c2[e] = zero;
    lo[e] = zero;
  }
  if (a.A_in) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = a.A_in[base + F::out_index(t, e)];
  }
  if (a.zbar2) {
#pragma unroll
    for (int e = 0; e < E; ++e) zb2[e] = a.zbar2[base + F::in_index(t, e)];
  }
  if (a.Cm1) {
#pragma unroll
    for (int e = 0; e < E; ++e) c1[e] = a.Cm1[base + F::in_index(t, e)];
  }
  if (a.Cm2) {
#pragma unroll
    for (int e = 0; e < E; ++e) c2[e] = a.Cm2[base + F::in_index(t, e)];
  }
  if (a.cout) {
#pragma unroll
    for (int e = 0; e < E; ++e) lo[e] = csub(a.cout[base + F::in_index(t, e)], a.label[base + F::in_index(t, e)]);
  }
  if (!active) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = zb2[e] = u[e] = bb[e] = c1[e] = c2[e] = lo[e] = zero;
  }
  for (int j = tid; j < N; j += nthreads) stw[j] = a.tw[j];
  __syncthreads();

  if (a.A_in) {
    F::inverse(v, t, stw, sm, 1);   // v = zbar_{j+1} (spatial)
    if (active && a.zbar_store) {
#pragma unroll
      for (int e = 0; e < E; ++e) a.zbar_store[base + F::in_index(t, e)] = v[e];
    }
  }
  const float kappa = a.dscal[0] * a.tau[scene];
  const float lscale = a.cout ? static_cast<float>(a.loss_scale / a.norm_label[scene]) : 0.f;
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    float2 g = make_float2((1.f + a.beta_j) * v[e].x - a.beta_j1 * zb2[e].x,
                           (1.f + a.beta_j) * v[e].y - a.beta_j1 * zb2[e].y);
    g.x += lscale * lo[e].x;
    g.y += lscale * lo[e].y;
    const float ax2 = u[e].x * u[e].x + u[e].y * u[e].y;
    float2 gu = zero;
    if (ax2 > kappa * kappa) {
      const float ra = __builtin_amdgcn_rsqf(ax2);      // 1/|u|
      const float proj = u[e].x * g.x + u[e].y * g.y;   // Re(conj(u) g)
      const float f = 1.f - kappa * ra;
      const float w = kappa * proj * ra * ra * ra;
      gu = make_float2(f * g.x + w * u[e].x, f * g.y + w * u[e].y);
      acc[0] -= static_cast<double>(proj) * ra;
    }
    acc[1] += static_cast<double>(gu.x) * bb[e].x + static_cast<double>(gu.y) * bb[e].y;
    v[e] = gu;
  }
  F::forward(v, t, stw, sm, 1);
  if (active) {
#pragma unroll
    for (int e = 0; e < E; ++e) a.Aout[base + F::out_index(t, e)] = v[e];
  }
#pragma unroll
  for (int e = 0; e < E; ++e)
    v[e] = make_float2((1.f + a.beta_jm1) * c1[e].x - a.beta_jm1 * c2[e].x,
                       (1.f + a.beta_jm1) * c1[e].y - a.beta_jm1 * c2[e].y);
  F::forward(v, t, stw, sm, 1);
  if (active) {
#pragma unroll
    for (int e = 0; e < E; ++e) a.Zout[base + F::out_index(t, e)] = v[e];
  }
  row_sum<2, T>(red, r, t, acc);
  if (active && t == 0) {
    a.part[2 * static_cast<size_t>(prow)] = acc[0];
    a.part[2 * static_cast<size_t>(prow) + 1] = acc[1];
  }
}

template <int N, int E>
__global__ __launch_bounds__(256) void k_lista_bwd_col(ListaBwdColArgs a, int W) {
  using F = Stockham<N, E>;
  constexpr int T = F::T;
  extern __shared__ float2 lds[];
  float2* stw = lds + W * fft_area(N);
  const int tid = threadIdx.x;
  const int nthreads = W * T;
  const int c = tid % W, t = tid / W;
  const int strips = a.L1 / W;
  const int col = blockIdx.x * W + c;
  (void)strips;
  const int group = blockIdx.y;
  const size_t plane = static_cast<size_t>(N) * a.L1;
  float2* sms = lds + c;
  float2 mc[E], acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    mc[e] = a.mulc[static_cast<size_t>(F::out_index(t, e)) * a.L1 + col];
    acc[e] = make_float2(0.f, 0.f);
  }
  for (int j = tid; j < N; j += nthreads) stw[j] = a.tw[j];
  __syncthreads();
  const float invL = 1.f / static_cast<float>(plane);
  for (int s = group; s < a.nscenes; s += a.groups) {
    float2* g = a.A + s * plane + col;
    const float2* z = a.Z + s * plane + col;
    float2 v[E], w[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      v[e] = g[static_cast<size_t>(F::in_index(t, e)) * a.L1];
      w[e] = z[static_cast<size_t>(F::in_index(t, e)) * a.L1];
    }
    F::forward(v, t, stw, sms, W);
    F::forward(w, t, stw, sms, W);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const float2 p = cmulc(v[e], w[e]);   // A conj(Z)
      acc[e].x += p.x * invL;
      acc[e].y += p.y * invL;
      v[e] = cmulc(v[e], mc[e]);            // conj(m_j)/L . A
    }
    F::inverse(v, t, stw, sms, W);
#pragma unroll
    for (int e = 0; e < E; ++e) g[static_cast<size_t>(F::in_index(t, e)) * a.L1] = v[e];
  }
  float2* gp = a.gm_part + group * plane + col;
#pragma unroll
  for (int e = 0; e < E; ++e) gp[static_cast<size_t>(F::out_index(t, e)) * a.L1] = acc[e];
}

template <int N, int E>
__global__ __launch_bounds__(256) void k_kkt_row(KktRowArgs a, int rpb) {
  using F = Stockham<N, E>;
  constexpr int T = F::T;
  extern __shared__ float2 lds[];
  float2* stw = lds + rpb * fft_area(N);
  double* red = reinterpret_cast<double*>(stw + N);
  const int tid = threadIdx.x;
  const int nthreads = rpb * T;
  const int r = tid / T, t = tid - (tid / T) * T;
  const int row = blockIdx.x * rpb + r;
  const bool active = row < a.nrows;
  int scene = 0, prow = 0;
  if (active) {
    scene = row / a.rows_per_scene;
    const int within = row - scene * a.rows_per_scene;
    if (a.scene_map) scene = a.scene_map[scene];
    prow = scene * a.rows_per_scene + within;
  }
  float2* sm = lds + r * fft_area(N);
  const size_t base = static_cast<size_t>(prow) * N;
  const float2 zero = make_float2(0.f, 0.f);
  float2 v[E], cc[E], bb[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    v[e] = a.gc[base + F::out_index(t, e)];
    cc[e] = a.c[base + F::in_index(t, e)];
    bb[e] = a.b[base + F::in_index(t, e)];
  }
  if (!active) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cc[e] = bb[e] = zero;
  }
  for (int j = tid; j < N; j += nthreads) stw[j] = a.tw[j];
  __syncthreads();
  F::inverse(v, t, stw, sm, 1);
  const double tau = active ? a.tau[scene] : 0.0;
  double acc[1] = {0.0};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const double gr = static_cast<double>(bb[e].x) - v[e].x, gi = static_cast<double>(bb[e].y) - v[e].y;
    const double cr = cc[e].x, ci = cc[e].y;
    const double ac = sqrt(cr * cr + ci * ci);
    double e2;
    if (ac > 0.0) {
      const double er = gr - tau * cr / ac, ei = gi - tau * ci / ac;
      e2 = er * er + ei * ei;
    } else {
      const double d = fmax(sqrt(gr * gr + gi * gi) - tau, 0.0);
      e2 = d * d;
    }
    acc[0] += active ? e2 : 0.0;
  }
  row_sum<1, T>(red, r, t, acc);
  if (active && t == 0) a.part[prow] = acc[0];
}

// The KKT check on the kept spectral columns (sparse support): the column pass
// leaves the kept row spectra of (b - G c) / scale; this pass expands them,
// takes the row IDFT and forms the per-row sums of e^2 as k_kkt_row does.
// Dynamic LDS: rpb exchange areas + N twiddles + rpb * ncs kept values + sums.
template <int N, int E>
__global__ __launch_bounds__(256) void k_kkt_rowp(KktRowArgs a, int rpb) {
  using F = Stockham<N, E>;
  constexpr int T = F::T;
  extern __shared__ float2 lds[];
  float2* stw = lds + rpb * fft_area(N);
  const int ncs = a.ncs;
  float2* lstb = stw + N;
  double* red = reinterpret_cast<double*>(lstb + rpb * ncs);
  const int tid = threadIdx.x;
  const int nthreads = rpb * T;
  const int r = tid / T, t = tid - (tid / T) * T;
  const int row = blockIdx.x * rpb + r;
  const bool active = row < a.nrows;
  int scene = 0, prow = 0;
  if (active) {
    scene = row / a.rows_per_scene;
    const int within = row - scene * a.rows_per_scene;
    if (a.scene_map) scene = a.scene_map[scene];
    prow = scene * a.rows_per_scene + within;
  }
  float2* sm = lds + r * fft_area(N);
  float2* lst = lstb + r * ncs;
  const size_t base = static_cast<size_t>(prow) * N;
  const size_t xrow = static_cast<size_t>(prow) * ncs;
  int ks[E];
  float2 cc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    ks[e] = a.colslot[F::out_index(t, e)];
    cc[e] = keep_if(active, a.c[base + F::in_index(t, e)]);
  }
  for (int j = t; j < ncs; j += T) {
    const float2 x = a.gc[xrow + j];   // row 0 when inactive: a valid address
    lst[j] = keep_if(active, x);
  }
  for (int j = tid; j < N; j += nthreads) stw[j] = a.tw[j];
  __syncthreads();
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = keep_if(ks[e] >= 0, lst[ks[e] >= 0 ? ks[e] : 0]);
  F::inverse(v, t, stw, sm, 1);
  const double tau = active ? a.tau[scene] : 0.0;
  const double sc = a.scale;
  double acc[1] = {0.0};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const double gr = sc * v[e].x, gi = sc * v[e].y;   // b - G c
    const double cr = cc[e].x, ci = cc[e].y;
    const double ac = sqrt(cr * cr + ci * ci);
    double e2;
    if (ac > 0.0) {
      const double er = gr - tau * cr / ac, ei = gi - tau * ci / ac;
      e2 = er * er + ei * ei;
    } else {
      const double d = fmax(sqrt(gr * gr + gi * gi) - tau, 0.0);
      e2 = d * d;
    }
    acc[0] += active ? e2 : 0.0;
  }
  row_sum<1, T>(red, r, t, acc);
  if (active && t == 0) a.part[prow] = acc[0];
}

template <int N, int E>
int lista_launch_e(int which, const void* args, int rpb_or_w, int groups, hipStream_t s) {
  constexpr int T = Stockham<N, E>::T;
  if (which == 3) {  // KKT check on the kept columns
    const KktRowArgs& a = *static_cast<const KktRowArgs*>(args);
    const int rpb = rpb_or_w;
    if (rpb < 1 || rpb * T > 256 || !a.colslot || a.ncs < 1 || a.ncs > N / 2) return -1;
    const int blocks = (a.nrows + rpb - 1) / rpb;
    if (blocks <= 0) return 0;
    const size_t shm = (static_cast<size_t>(rpb) * fft_area(N) + N + static_cast<size_t>(rpb) * a.ncs) * sizeof(float2) +
                       static_cast<size_t>(rpb) * T * sizeof(double);
    if (shm > 65536) return -1;
    hipLaunchKernelGGL((k_kkt_rowp<N, E>), dim3(blocks), dim3(rpb * T), shm, s, a, rpb);
    return hipGetLastError() == hipSuccess ? 0 : -4;
  }
  if (which == 0 || which == 2) {  // row kernels
    const int rpb = rpb_or_w;
    const int nrows = which == 0 ? static_cast<const ListaBwdRowArgs*>(args)->nrows
                                 : static_cast<const KktRowArgs*>(args)->nrows;
    if (rpb < 1 || rpb * T > 256) return -1;
    const int blocks = (nrows + rpb - 1) / rpb;
    if (blocks <= 0) return 0;
    const size_t shm = (static_cast<size_t>(rpb) * fft_area(N) + N) * sizeof(float2) +
                       static_cast<size_t>(rpb) * T * 2 * sizeof(double);
    if (shm > 65536) return -1;
    if (which == 0)
      hipLaunchKernelGGL((k_lista_bwd_row<N, E>), dim3(blocks), dim3(rpb * T), shm, s,
                         *static_cast<const ListaBwdRowArgs*>(args), rpb);
    else
      hipLaunchKernelGGL((k_kkt_row<N, E>), dim3(blocks), dim3(rpb * T), shm, s, *static_cast<const KktRowArgs*>(args),
                         rpb);
  } else {
    const ListaBwdColArgs& a = *static_cast<const ListaBwdColArgs*>(args);
    const int W = rpb_or_w;
    if (W < 1 || W * T > 256 || a.L1 % W != 0 || groups < 1) return -1;
    const size_t shm = (static_cast<size_t>(W) * fft_area(N) + N) * sizeof(float2);
    if (shm > 65536) return -1;
    hipLaunchKernelGGL((k_lista_bwd_col<N, E>), dim3(a.L1 / W, groups), dim3(W * T), shm, s, a, W);
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace bccb
