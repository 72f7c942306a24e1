// Row and column pass kernels (templates), instantiated per transform length
// in passes_n.hip.
//
// The product R c = IDFT2(Omega . DFT2(C)) of eq. (23) is split into a row pass
// (transforms along l1, contiguous) and a column pass (transforms along l2,
// stride L1).  Grids are [L2][L1] row-major, c(l1 + l2*L1) = C(l1, l2)
// (Sec. II-A).  One solver iteration is
//   column pass: DFT_cols -> multiply by the BCCB spectrum -> IDFT_cols
//   row pass   : IDFT_rows -> proximal/momentum/ADMM update -> DFT_rows
// so the state crosses memory once per pass, and the spectral multiply, the
// soft threshold (eq. (9)), the FISTA momentum (eqs. (10)-(12)) and the ADMM
// updates (eqs. (13)-(15)) never take a pass of their own.
#pragma once

#include "fft_device.h"
#include "kernels.h"

namespace bccb {

__device__ __forceinline__ bool finite2(float2 v) {
  return __builtin_isfinite(v.x) && __builtin_isfinite(v.y);
}

// Complex soft threshold S_k(z) = z max(1 - k/|z|, 0), zero for |z| <= k (R3).
__device__ __forceinline__ float2 shrink(float2 z, float k) {
  const float a2 = z.x * z.x + z.y * z.y;
  if (!(a2 > k * k)) return make_float2(0.f, 0.f);
  const float f = 1.f - k * __builtin_amdgcn_rsqf(a2);
  return make_float2(z.x * f, z.y * f);
}

// ---------------------------------------------------------------------------
// Row pass: a block owns `rpb` consecutive rows, T threads each.
// Dynamic LDS: rpb * N float2 exchange slots + N twiddles.
// ---------------------------------------------------------------------------
// With spread > 1 the grid holds spread x the blocks and only every spread-th
// does work: on a GPU that deals consecutive blocks round-robin to its XCDs
// this keeps a small (single-scene) working set inside one XCD's L2.
__device__ __forceinline__ bool spread_block(int spread, int& bid) {
  bid = static_cast<int>(blockIdx.x);
  if (spread <= 1) return true;
  if (bid % spread != 0) return false;
  bid /= spread;
  return true;
}

template <int N>
struct SparseRow {
  static constexpr int CAP = N / 8;   // slots per row
};

template <int N, int E, int MODE>
__global__ __launch_bounds__(256) void k_row(RowArgs a, int rpb) {
  using F = Stockham<N, E>;
  constexpr int T = F::T;
  constexpr bool kSp = (MODE == ROW_FISTA_SP);
  constexpr bool kIter = (MODE == ROW_ISTA || MODE == ROW_FISTA || MODE == ROW_ADMM || kSp);
  constexpr bool kState = (MODE == ROW_FISTA || MODE == ROW_ADMM);
  constexpr int CAP = SparseRow<N>::CAP;
  constexpr int SPT = (CAP + T - 1) / T;   // slots read per thread
  extern __shared__ float2 lds[];
  float2* stw = lds + rpb * N;
  int* rowcnt = reinterpret_cast<int*>(stw + N);   // kSp: rpb * T ints
  int bid;
  if (!spread_block(a.spread, bid)) return;  // whole block exits together

  const int tid = threadIdx.x;
  const int nthreads = rpb * T;
  const int r = tid / T, t = tid - (tid / T) * T;
  const int row = bid * rpb + r;
  const bool active = row < a.nrows;
  float2* sm = lds + r * N;
  // logical row -> physical row of the arenas (scene compaction through scene_map)
  int scene = 0, prow = 0;
  if (active) {
    scene = row / a.rows_per_scene;
    const int within = row - scene * a.rows_per_scene;
    if (a.scene_map) scene = a.scene_map[scene];
    prow = scene * a.rows_per_scene + within;
  }
  const size_t base = static_cast<size_t>(prow) * N;
  const float2 zero = make_float2(0.f, 0.f);

  // Every global load of the pass is issued before the first barrier so the
  // latencies of the iterate, the right-hand side, the state and the twiddle
  // table overlap instead of adding up.
  // Loads read a valid row (row 0 for inactive threads) and are zeroed afterwards:
  // selecting between a global address and a local zero would turn them into
  // flat loads through a stack slot.
  float2 v[E];
  float2 rhs[kIter ? E : 1];
  float2 st[kState ? E : 1];
  if constexpr (MODE == ROW_FWD) {
    if (a.src) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = a.src[base + F::in_index(t, e)];
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = zero;
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = a.xy[base + F::out_index(t, e)];
  }
  if constexpr (kIter) {
    if (a.rhs) {
#pragma unroll
      for (int e = 0; e < E; ++e) rhs[e] = a.rhs[base + F::in_index(t, e)];
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) rhs[e] = zero;
    }
  }
  if constexpr (kState) {
#pragma unroll
    for (int e = 0; e < E; ++e) st[e] = a.state[base + F::in_index(t, e)];
  }
  // sparse storage of c_{t-1}: the row's count and all of its slots are read up
  // front (one round trip); a dense row is read after the count is known
  int rcount = 0;
  unsigned short sl_i[kSp ? SPT : 1];
  float2 sl_v[kSp ? SPT : 1];
  if constexpr (kSp) {
    rcount = a.cnt[prow];
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int j = t + T * q;
      const int jj = j < CAP ? j : 0;
      sl_i[q] = a.sidx[static_cast<size_t>(prow) * CAP + jj];
      sl_v[q] = a.sval[static_cast<size_t>(prow) * CAP + jj];
    }
  }
  if (!active) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      v[e] = zero;
      if constexpr (kIter) rhs[e] = zero;
      if constexpr (kState) st[e] = zero;
    }
    rcount = 0;
  }
  for (int j = tid; j < N; j += nthreads) stw[j] = a.tw[j];
  float2 sp[kSp ? E : 1];   // c_{t-1} at the thread's elements (sparse storage)
  if constexpr (kSp) {
    // expand the slots into the row's LDS area, then read the thread's elements
#pragma unroll
    for (int e = 0; e < E; ++e) sm[F::in_index(t, e)] = zero;
    __syncthreads();
    if (rcount <= CAP) {
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        const int j = t + T * q;
        if (j < rcount) sm[sl_i[q] < N ? sl_i[q] : N - 1] = sl_v[q];
      }
    }
    __syncthreads();
    if (rcount <= CAP) {
#pragma unroll
      for (int e = 0; e < E; ++e) sp[e] = sm[F::in_index(t, e)];
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) sp[e] = a.state[base + F::in_index(t, e)];
    }
  }
  __syncthreads();

  if constexpr (MODE == ROW_FWD) {
    bool ok = true;
#pragma unroll
    for (int e = 0; e < E; ++e) ok = ok && finite2(v[e]);
    if (!ok && a.flag) *a.flag = 1;
    F::forward(v, t, stw, sm, 1);
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) a.xy[base + F::out_index(t, e)] = v[e];
    }
  } else if constexpr (MODE == ROW_INV) {
    F::inverse(v, t, stw, sm, 1);
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) a.dst[base + F::in_index(t, e)] = cscale(v[e], a.scale);
    }
  } else {
    F::inverse(v, t, stw, sm, 1);
    float kbase = a.kappa, rs = a.rhs_scale;
    if (a.dscal) {
      kbase = a.dscal[0];
      rs = a.dscal[1];
    }
    const float kappa = a.kscale ? kbase * a.kscale[scene] : kbase;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const size_t idx = base + F::in_index(t, e);
      if constexpr (MODE == ROW_ISTA) {
        const float2 c = shrink(make_float2(v[e].x + rs * rhs[e].x, v[e].y + rs * rhs[e].y), kappa);
        if (a.last && active) a.out_c[idx] = c;
        v[e] = c;
      } else if constexpr (kSp) {
        // c_t stays in v[e] until the row's storage form is decided below
        const float2 u = make_float2(v[e].x + rs * rhs[e].x, v[e].y + rs * rhs[e].y);
        v[e] = shrink(u, kappa);
      } else if constexpr (MODE == ROW_FISTA) {
        const float2 u = make_float2(v[e].x + rs * rhs[e].x, v[e].y + rs * rhs[e].y);
        const float2 c = shrink(u, kappa);
        const float2 cp = st[e];
        if (active) {
          a.state[idx] = c;
          if (a.save_u) a.save_u[idx] = u;
          if (a.save_c) a.save_c[idx] = c;
          if (a.out_prev) a.out_prev[idx] = cp;
        }
        v[e] = make_float2(c.x + a.beta * (c.x - cp.x), c.y + a.beta * (c.y - cp.y));
      } else {  // ROW_ADMM
        const float2 c = cadd(rhs[e], v[e]);
        const float2 vv = st[e];
        const float2 z = shrink(cadd(c, vv), kappa);
        const float2 vn = csub(cadd(vv, c), z);
        if (active) {
          a.state[idx] = vn;
          if (a.last) {
            a.out_z[idx] = z;
            if (a.out_c) a.out_c[idx] = c;
          }
        }
        v[e] = csub(z, vn);
      }
    }
    if constexpr (kSp) {
      // store c_t: slots if the row has at most CAP nonzeros (not at the last
      // iteration, whose output is read densely), the dense row otherwise
      int mine = 0;
#pragma unroll
      for (int e = 0; e < E; ++e) mine += (v[e].x != 0.f || v[e].y != 0.f) ? 1 : 0;
      rowcnt[r * T + t] = mine;
      __syncthreads();
      int total = 0, before = 0;
      for (int i = 0; i < T; ++i) {
        const int ci = rowcnt[r * T + i];
        total += ci;
        before += (i < t) ? ci : 0;
      }
      const bool dense = a.last || total > CAP;
      if (active) {
        if (dense) {
#pragma unroll
          for (int e = 0; e < E; ++e) a.state[base + F::in_index(t, e)] = v[e];
        } else {
          int o = before;
#pragma unroll
          for (int e = 0; e < E; ++e) {
            if (v[e].x != 0.f || v[e].y != 0.f) {
              a.sidx[static_cast<size_t>(prow) * CAP + o] = static_cast<unsigned short>(F::in_index(t, e));
              a.sval[static_cast<size_t>(prow) * CAP + o] = v[e];
              ++o;
            }
          }
        }
        if (t == 0) a.cnt[prow] = dense ? CAP + 1 + total : total;
      }
      // momentum z = c_t + beta (c_t - c_{t-1})
#pragma unroll
      for (int e = 0; e < E; ++e)
        v[e] = make_float2(v[e].x + a.beta * (v[e].x - sp[e].x), v[e].y + a.beta * (v[e].y - sp[e].y));
    }
    if (!a.last) {
      F::forward(v, t, stw, sm, 1);
      if (active) {
#pragma unroll
        for (int e = 0; e < E; ++e) a.xy[base + F::out_index(t, e)] = v[e];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Column pass: a block owns W adjacent columns of one scene; lane = c + W*t.
// Dynamic LDS: W * N float2 exchange slots (column c at stride W) + N twiddles.
// ---------------------------------------------------------------------------
template <int N, int E, int MODE>
__global__ __launch_bounds__(256) void k_col(ColArgs a, int W) {
  using F = Stockham<N, E>;
  constexpr int T = F::T;
  extern __shared__ float2 lds[];
  float2* stw = lds + W * N;
  int bid;
  if (!spread_block(a.spread, bid)) return;  // whole block exits together

  const int tid = threadIdx.x;
  const int nthreads = W * T;
  const int c = tid % W, t = tid / W;
  const int strips = a.L1 / W;
  const int lscene = bid / strips;
  const int col = (bid - lscene * strips) * W + c;
  const int scene = a.scene_map ? a.scene_map[lscene] : lscene;
  const size_t plane = static_cast<size_t>(N) * a.L1;
  float2* g = a.xy + scene * plane + col;
  float2* sms = lds + c;

  constexpr bool kSparse = (MODE == COL_SPARSE_AFFINE || MODE == COL_SPARSE_ADMM);
  constexpr bool kFwd = (MODE == COL_FWD || MODE == COL_FILTER_AFFINE || MODE == COL_FILTER_ADMM ||
                         MODE == COL_FILTER_CPLX || kSparse);
  constexpr bool kInv = (MODE != COL_FWD);
  constexpr bool kMul = (MODE != COL_FWD && MODE != COL_INV && !kSparse);
  constexpr bool kCplx = (MODE == COL_FILTER_CPLX);

  // all global loads first (iterate, spectral multiplier, twiddles)
  float2 v[E];
  if constexpr (kFwd) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = g[static_cast<size_t>(F::in_index(t, e)) * a.L1];
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = g[static_cast<size_t>(F::out_index(t, e)) * a.L1];
  }
  float om[(kMul && !kCplx) ? E : 1];
  float2 mc[kCplx ? E : 1];
  if constexpr (kCplx) {
    const float2* m = a.mulc + scene * a.mulc_stride + col;
#pragma unroll
    for (int e = 0; e < E; ++e) mc[e] = m[static_cast<size_t>(F::out_index(t, e)) * a.L1];
  } else if constexpr (kMul) {
    const float* o = a.omega + scene * a.omega_stride + col;
#pragma unroll
    for (int e = 0; e < E; ++e) om[e] = o[static_cast<size_t>(F::out_index(t, e)) * a.L1];
  }
  for (int j = tid; j < N; j += nthreads) stw[j] = a.tw[j];
  __syncthreads();

  if constexpr (kFwd) F::forward(v, t, stw, sms, W);

  if constexpr (kCplx) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cmul(v[e], mc[e]);
  } else if constexpr (MODE == COL_FILTER_AFFINE || MODE == COL_MULINV_AFFINE) {
    const float2 ab = a.coef[scene];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cscale(v[e], ab.x + ab.y * om[e]);
  } else if constexpr (kMul) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cscale(v[e], a.scale / (om[e] + a.rho));
  } else if constexpr (kSparse) {
    // multiplier off the support; the few support bins of this column are then
    // overwritten by the thread that holds them
    float mdef;
    float2 ab = make_float2(0.f, 0.f);
    if constexpr (MODE == COL_SPARSE_AFFINE) {
      ab = a.coef[scene];
      mdef = ab.x;
    } else {
      mdef = a.scale / a.rho;
    }
    float2 src[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      src[e] = v[e];
      v[e] = cscale(v[e], mdef);
    }
    const int* ptr = a.sup_ptr + scene * a.sup_ptr_stride + col;
    const int j0 = ptr[0], j1 = ptr[1];
    const float2* rhs = a.sup_rhs + scene * a.sup_rhs_stride;
    for (int j = j0; j < j1; ++j) {
      const SupEntry en = a.sup[j];
      const float2 r = rhs[j];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (F::out_index(t, e) == en.k2) {
          if constexpr (MODE == COL_SPARSE_AFFINE) {
            const float m = ab.x + ab.y * en.omega;
            v[e] = make_float2(src[e].x * m + r.x, src[e].y * m + r.y);
          } else {
            const float d = 1.f / (en.omega + a.rho);
            const float m = a.scale * d;
            v[e] = make_float2(src[e].x * m + r.x * d, src[e].y * m + r.y * d);
          }
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
// Launchers for one N (instantiated in passes_n.hip)
// ---------------------------------------------------------------------------
template <int N, int E>
int row_launch_e(int mode, const RowArgs& a, int rpb, hipStream_t s) {
  constexpr int T = Stockham<N, E>::T;
  if (rpb < 1 || rpb * T > 256) return -1;
  const int blocks = (a.nrows + rpb - 1) / rpb;
  if (blocks <= 0) return 0;
  const size_t shm = static_cast<size_t>(rpb + 1) * N * sizeof(float2) +
                     (mode == ROW_FISTA_SP ? static_cast<size_t>(rpb) * T * sizeof(int) : 0);
  if (shm > 65536) return -1;
  if (mode == ROW_FISTA_SP && (!a.cnt || !a.sidx || !a.sval || !a.state)) return -1;
  const int spread = a.spread > 1 ? a.spread : 1;
  const dim3 grid(blocks * spread), block(rpb * T);
  switch (mode) {
    case ROW_FISTA_SP: hipLaunchKernelGGL((k_row<N, E, ROW_FISTA_SP>), grid, block, shm, s, a, rpb); break;
    case ROW_FWD: hipLaunchKernelGGL((k_row<N, E, ROW_FWD>), grid, block, shm, s, a, rpb); break;
    case ROW_INV: hipLaunchKernelGGL((k_row<N, E, ROW_INV>), grid, block, shm, s, a, rpb); break;
    case ROW_ISTA: hipLaunchKernelGGL((k_row<N, E, ROW_ISTA>), grid, block, shm, s, a, rpb); break;
    case ROW_FISTA: hipLaunchKernelGGL((k_row<N, E, ROW_FISTA>), grid, block, shm, s, a, rpb); break;
    case ROW_ADMM: hipLaunchKernelGGL((k_row<N, E, ROW_ADMM>), grid, block, shm, s, a, rpb); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

template <int N, int E>
int col_launch_e(int mode, const ColArgs& a, int W, hipStream_t s) {
  constexpr int T = Stockham<N, E>::T;
  if (W < 1 || W * T > 256 || a.L1 % W != 0) return -1;
  const int blocks = (a.L1 / W) * a.nscenes;
  if (blocks <= 0) return 0;
  const size_t shm = static_cast<size_t>(W + 1) * N * sizeof(float2);
  if (shm > 65536) return -1;
  const int spread = a.spread > 1 ? a.spread : 1;
  const dim3 grid(blocks * spread), block(W * T);
  switch (mode) {
    case COL_FWD: hipLaunchKernelGGL((k_col<N, E, COL_FWD>), grid, block, shm, s, a, W); break;
    case COL_INV: hipLaunchKernelGGL((k_col<N, E, COL_INV>), grid, block, shm, s, a, W); break;
    case COL_FILTER_AFFINE: hipLaunchKernelGGL((k_col<N, E, COL_FILTER_AFFINE>), grid, block, shm, s, a, W); break;
    case COL_FILTER_ADMM: hipLaunchKernelGGL((k_col<N, E, COL_FILTER_ADMM>), grid, block, shm, s, a, W); break;
    case COL_FILTER_CPLX: hipLaunchKernelGGL((k_col<N, E, COL_FILTER_CPLX>), grid, block, shm, s, a, W); break;
    case COL_MULINV_AFFINE: hipLaunchKernelGGL((k_col<N, E, COL_MULINV_AFFINE>), grid, block, shm, s, a, W); break;
    case COL_MULINV_ADMM: hipLaunchKernelGGL((k_col<N, E, COL_MULINV_ADMM>), grid, block, shm, s, a, W); break;
    case COL_SPARSE_AFFINE: hipLaunchKernelGGL((k_col<N, E, COL_SPARSE_AFFINE>), grid, block, shm, s, a, W); break;
    case COL_SPARSE_ADMM: hipLaunchKernelGGL((k_col<N, E, COL_SPARSE_ADMM>), grid, block, shm, s, a, W); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace bccb
