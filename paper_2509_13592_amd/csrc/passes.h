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

// c ? a : 0, selected per component: a select of whole float2 values (an
// aggregate) is lowered through memory, as a flat load from a chosen address.
__device__ __forceinline__ float2 keep_if(bool c, float2 a) {
  return make_float2(c ? a.x : 0.f, c ? a.y : 0.f);
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
// Dynamic LDS: rpb * (one or two padded exchange areas) + N twiddles (+ counts).
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


// Transform helpers over a row's (or column's) exchange areas A and B.  Two-area
// transforms take one barrier per exchange; single-area ones use A only and a
// barrier before every write.  fft_fwd / fft_inv start by writing A, after a
// barrier when `sync0` (A may still be read); fft_fwd_after_inv follows an
// fft_inv and starts in the area that transform did not use last, without a barrier.
template <class F>
__device__ __forceinline__ void fft_fwd(float2* v, int t, const float2* tw, float2* A, float2* B, bool sync0,
                                        int ss = 1) {
  if constexpr (F::kTwoArea) F::forward2(v, t, tw, A, B, ss, sync0);
  else F::forward(v, t, tw, A, ss, sync0);
}
template <class F>
__device__ __forceinline__ void fft_inv(float2* v, int t, const float2* tw, float2* A, float2* B, bool sync0 = false,
                                        int ss = 1) {
  if constexpr (F::kTwoArea) F::inverse2(v, t, tw, A, B, ss, sync0);
  else F::inverse(v, t, tw, A, ss, sync0);
}
template <class F>
__device__ __forceinline__ void fft_fwd_after_inv(float2* v, int t, const float2* tw, float2* A, float2* B, int ss = 1) {
  if constexpr (F::kTwoArea) {
    if constexpr (F::kLastB) F::forward2(v, t, tw, A, B, ss, false);
    else F::forward2(v, t, tw, B, A, ss, false);
  } else {
    F::forward(v, t, tw, A, ss);
  }
}
template <class F>
__device__ __forceinline__ void fft_inv_after_fwd(float2* v, int t, const float2* tw, float2* A, float2* B, int ss = 1) {
  if constexpr (F::kTwoArea) {
    if constexpr (F::kLastB) F::inverse2(v, t, tw, A, B, ss, false);
    else F::inverse2(v, t, tw, B, A, ss, false);
  } else {
    F::inverse(v, t, tw, A, ss);
  }
}

// Number of nonzeros of a row (T threads, `mine` each) and the count before
// thread t.  Rows of at most 64 threads sit inside one wavefront (T divides 64):
// a segmented shuffle scan; longer rows go through LDS (`cnt`: T ints per row,
// two barriers, reached by the whole block).
template <int T>
__device__ __forceinline__ void row_prefix(int mine, int t, int* cnt, int& total, int& before) {
  if constexpr (T <= 64) {
    int incl = mine;
#pragma unroll
    for (int d = 1; d < T; d <<= 1) {
      const int y = __shfl_up(incl, d, T);
      if (t >= d) incl += y;
    }
    before = incl - mine;
    total = __shfl(incl, T - 1, T);
  } else {
    __syncthreads();   // a previous call's readers are done with cnt
    cnt[t] = mine;
    __syncthreads();
    total = 0;
    before = 0;
    for (int i = 0; i < T; ++i) {
      const int ci = cnt[i];
      total += ci;
      before += (i < t) ? ci : 0;
    }
  }
}

template <int N>
struct SparseRow {
  static constexpr int CAP = N / 8;   // slots per row
};

template <int N, int E, int MODE>
__global__ __launch_bounds__(256) void k_row(RowArgs a, int rpb) {
  constexpr bool kWave = (N / E) <= 64;   // a row inside one wavefront: row-local exchanges sync the wave
  using F = Stockham<N, E, kWave>;
  constexpr int T = F::T;
  constexpr bool kSp = (MODE == ROW_FISTA_SP);
  constexpr bool kIter = (MODE == ROW_ISTA || MODE == ROW_FISTA || MODE == ROW_ADMM || kSp);
  constexpr bool kState = (MODE == ROW_FISTA || MODE == ROW_ADMM);
  constexpr int CAP = SparseRow<N>::CAP;
  constexpr int SPT = (CAP + T - 1) / T;   // slots read per thread
  constexpr int AR = fft_areas(N, E);
  constexpr int FA = fft_area(N);
  extern __shared__ float2 lds[];
  float2* stw = lds + AR * rpb * FA;
  int* rowcnt = reinterpret_cast<int*>(stw + N);   // kSp: rpb * T ints
  int bid;
  if (!spread_block(a.spread, bid)) return;  // whole block exits together

  const int tid = threadIdx.x;
  const int nthreads = rpb * T;
  const int r = tid / T, t = tid - (tid / T) * T;
  const int row = bid * rpb + r;
  const bool active = row < a.nrows;
  float2* sm = lds + AR * r * FA;      // exchange area (and slot expansion)
  float2* sm2 = sm + (AR - 1) * FA;    // second exchange area (two-area transforms)
  // logical row -> physical row of the arenas (scene compaction through scene_map)
  int scene = 0, prow = 0, within = 0;
  if (active) {
    scene = row / a.rows_per_scene;
    within = row - scene * a.rows_per_scene;
    if (a.scene_map) scene = a.scene_map[scene];
    prow = scene * a.rows_per_scene + within;
  }
  const size_t base = static_cast<size_t>(prow) * N;
  const float2 zero = make_float2(0.f, 0.f);
  // zero-padded embedding: rows at or past act_rows hold no coefficient
  const bool masked = a.act_cols > 0;
  const bool row_in = !masked || within < a.act_rows;

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
    lds_sync<kWave>();
    if (rcount <= CAP) {
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        const int j = t + T * q;
        if (j < rcount) sm[sl_i[q] < N ? sl_i[q] : N - 1] = sl_v[q];
      }
    }
    lds_sync<kWave>();
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
    fft_fwd<F>(v, t, stw, sm, sm2, false);
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) a.xy[base + F::out_index(t, e)] = v[e];
    }
  } else if constexpr (MODE == ROW_INV) {
    fft_inv<F>(v, t, stw, sm, sm2);
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) a.dst[base + F::in_index(t, e)] = cscale(v[e], a.scale);
    }
  } else {
    fft_inv<F>(v, t, stw, sm, sm2);
    float kbase = a.kappa, rs = a.rhs_scale;
    if (a.dscal) {
      kbase = a.dscal[0];
      rs = a.dscal[1];
    }
    const float kappa = a.kscale ? kbase * a.kscale[scene] : kbase;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const size_t idx = base + F::in_index(t, e);
      // inside the coefficient window of a padded embedding (always, without one)
      const bool in = !masked || (row_in && F::in_index(t, e) < a.act_cols);
      if constexpr (MODE == ROW_ISTA) {
        const float2 c = keep_if(in, shrink(make_float2(v[e].x + rs * rhs[e].x, v[e].y + rs * rhs[e].y), kappa));
        if (a.last && active) a.out_c[idx] = c;
        v[e] = c;
      } else if constexpr (kSp) {
        // c_t stays in v[e] until the row's storage form is decided below
        const float2 u = make_float2(v[e].x + rs * rhs[e].x, v[e].y + rs * rhs[e].y);
        v[e] = shrink(u, kappa);
      } else if constexpr (MODE == ROW_FISTA) {
        const float2 u = make_float2(v[e].x + rs * rhs[e].x, v[e].y + rs * rhs[e].y);
        const float2 c = keep_if(in, shrink(u, kappa));
        const float2 cp = st[e];
        if (active) {
          a.state[idx] = c;
          if (a.save_u) a.save_u[idx] = u;
          if (a.save_c) a.save_c[idx] = c;
          if (a.out_prev) a.out_prev[idx] = cp;
        }
        v[e] = make_float2(c.x + a.beta * (c.x - cp.x), c.y + a.beta * (c.y - cp.y));
      } else {  // ROW_ADMM
        const float2 c = keep_if(in, cadd(rhs[e], v[e]));
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
      int total, before;
      row_prefix<T>(mine, t, rowcnt + r * T, total, before);
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
      fft_fwd_after_inv<F>(v, t, stw, sm, sm2);
      if (active) {
#pragma unroll
        for (int e = 0; e < E; ++e) a.xy[base + F::out_index(t, e)] = v[e];
      }
    }
  }
}


// ---------------------------------------------------------------------------
// Pruned row pass (sparse spectral support).  G = IDFT2 . Omega . DFT2 and
// Omega vanishes off the support bins, so (I - mu G) z_t + mu b = z_t +
// IDFT2(-mu Omega DFT2(z_t) + mu DFT2(b)) has its spectral correction on the
// support columns only: the column pass transforms just those, and this pass
// reads / writes just those columns of the row spectra (compact [row][ncs]).
// z_t is rebuilt in the spatial domain from c_{t-1} and c_{t-2}, which are kept
// per row in SlotBufs (sparse rows as slots), so a late iteration moves a few
// bytes per row instead of the whole grid.
// Dynamic LDS: 3 rpb N float2 (expansions of c_{t-1}, c_{t-2} and the kept
// spectral columns; the first is then the transforms' exchange area) + N
// twiddles + rpb T counts.
// ---------------------------------------------------------------------------
template <int N, int E>
__device__ __forceinline__ void load_slots(const SlotBuf& b, int prow, int t, int& n, unsigned short (&si)[(N / 8 + N / E - 1) / (N / E)],
                                           float2 (&sv)[(N / 8 + N / E - 1) / (N / E)]) {
  constexpr int T = N / E;
  constexpr int CAP = N / 8;
  constexpr int SPT = (CAP + T - 1) / T;
  n = b.cnt ? b.cnt[prow] : 0;
  if (!b.cnt) return;
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    const int j = t + T * q;
    const int jj = j < CAP ? j : 0;
    si[q] = b.sidx[static_cast<size_t>(prow) * CAP + jj];
    sv[q] = b.sval[static_cast<size_t>(prow) * CAP + jj];
  }
}

template <int N, int E, int MODE>
__global__ __launch_bounds__(256) void k_rowp(RowArgs a, int rpb) {
  constexpr bool kWave = (N / E) <= 64;   // a row inside one wavefront: row-local exchanges sync the wave
  using F = Stockham<N, E, kWave>;
  constexpr int T = F::T;
  constexpr int CAP = SparseRow<N>::CAP;
  constexpr int SPT = (CAP + T - 1) / T;
  constexpr int MW = (N + 31) / 32;
  constexpr bool kTwo = F::kTwoArea;
  extern __shared__ float2 lds[];
  int bid;
  if (!spread_block(a.spread, bid)) return;  // whole block exits together

  const int tid = threadIdx.x;
  const int nthreads = rpb * T;
  const int r = tid / T, t = tid - (tid / T) * T;
  const int row = bid * rpb + r;
  const bool active = row < a.nrows;
  const int ncs = a.ncs;
  constexpr int FA = fft_area(N);
  float2* sa = lds + (2 * r) * FA;      // exchange area A; c_{t-2} expansion
  float2* sb = sa + FA;                 // exchange area B (two-area transforms); c_{t-1} expansion
  float2* stw = lds + 2 * rpb * FA;
  float2* lst = stw + N + r * ncs;      // the row's kept spectral columns, compact
  unsigned* msk = reinterpret_cast<unsigned*>(stw + N + rpb * ncs) + r * 2 * MW;   // [2][MW]
  int* rowcnt = reinterpret_cast<int*>(reinterpret_cast<unsigned*>(stw + N + rpb * ncs) + rpb * 2 * MW) + r * T;
  int scene = 0, prow = 0;
  if (active) {
    scene = row / a.rows_per_scene;
    const int within = row - scene * a.rows_per_scene;
    if (a.scene_map) scene = a.scene_map[scene];
    prow = scene * a.rows_per_scene + within;
  }
  const size_t base = static_cast<size_t>(prow) * N;
  const size_t xrow = static_cast<size_t>(prow) * ncs;
  const int* cs = a.colslot + scene * a.colslot_stride;
  const float2 zero = make_float2(0.f, 0.f);

  // kept-column slot of each of this thread's spectral bins (natural order out_index)
  int ks[E];
#pragma unroll
  for (int e = 0; e < E; ++e) ks[e] = cs[F::out_index(t, e)];

  if constexpr (MODE == ROW_PRUNED_FWD) {
    float2 v[E];
    if (a.src) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = a.src[base + F::in_index(t, e)];
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = zero;
    }
    if (!active) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = zero;
    }
    for (int j = tid; j < N; j += nthreads) stw[j] = a.tw[j];
    bool ok = true;
#pragma unroll
    for (int e = 0; e < E; ++e) ok = ok && finite2(v[e]);
    if (!ok && a.flag) *a.flag = 1;
    __syncthreads();
    fft_fwd<F>(v, t, stw, sa, sb, false);
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (ks[e] >= 0) a.xy[xrow + ks[e]] = v[e];
    }
  } else {
    // global loads, all independent: slots of c_{t-1} and c_{t-2}, the compact
    // kept columns (into LDS), the twiddles; the occupancy masks start empty
    int n1, n2;
    unsigned short i1[SPT], i2[SPT];
    float2 w1[SPT], w2[SPT];
    load_slots<N, E>(a.b1, prow, t, n1, i1, w1);
    load_slots<N, E>(a.b2, prow, t, n2, i2, w2);
    if (!active) n1 = n2 = 0;
    for (int j = t; j < ncs; j += T) {
      const float2 x = a.xy[xrow + j];   // row 0 when inactive: a valid address
      lst[j] = keep_if(active, x);
    }
    for (int j = tid; j < N; j += nthreads) stw[j] = a.tw[j];
    for (int j = t; j < 2 * MW; j += T) msk[j] = 0u;
    // dense rows go to their area straight from memory (each thread its own elements)
    const bool full1 = n1 > CAP, full2 = n2 > CAP;
    if (full1) {
#pragma unroll
      for (int e = 0; e < E; ++e) sb[F::in_index(t, e)] = a.b1.dense[base + F::in_index(t, e)];
    }
    if (full2) {
#pragma unroll
      for (int e = 0; e < E; ++e) sa[F::in_index(t, e)] = a.b2.dense[base + F::in_index(t, e)];
    }
    __syncthreads();
    // scatter the slot rows: c_{t-1} into B (it outlives a single-area transform), c_{t-2} into A
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int j = t + T * q;
      if (!full1 && j < n1) {
        const int idx = i1[q] < N ? i1[q] : N - 1;
        sb[idx] = w1[q];
        atomicOr(&msk[idx >> 5], 1u << (idx & 31));
      }
      if (!full2 && j < n2) {
        const int idx = i2[q] < N ? i2[q] : N - 1;
        sa[idx] = w2[q];
        atomicOr(&msk[MW + (idx >> 5)], 1u << (idx & 31));
      }
    }
    lds_sync<kWave>();   // the scatter is row-local
    // z_t = c_{t-1} + beta_{t-1} (c_{t-1} - c_{t-2}) at this thread's elements
    float2 z[E];
    float2 c1[kTwo ? E : 1];   // two-area transforms overwrite B: c_{t-1} stays in registers
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int idx = F::in_index(t, e);
      const float2 l1 = sb[idx], l2 = sa[idx];
      const float2 p1 = keep_if(full1 || ((msk[idx >> 5] >> (idx & 31)) & 1u), l1);
      const float2 p2 = keep_if(full2 || ((msk[MW + (idx >> 5)] >> (idx & 31)) & 1u), l2);
      z[e] = make_float2(p1.x + a.beta_prev * (p1.x - p2.x), p1.y + a.beta_prev * (p1.y - p2.y));
      if constexpr (kTwo) c1[e] = p1;
    }
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = keep_if(ks[e] >= 0, lst[ks[e] >= 0 ? ks[e] : 0]);

    fft_inv<F>(v, t, stw, sa, sb, true);   // the expansions were read from A / B
    const float kbase = a.dscal ? a.dscal[0] : a.kappa;
    const float kappa = a.kscale ? kbase * a.kscale[scene] : kbase;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = shrink(make_float2(z[e].x + v[e].x, z[e].y + v[e].y), kappa);

    if (a.last) {
      if (active) {
#pragma unroll
        for (int e = 0; e < E; ++e) a.out_c[base + F::in_index(t, e)] = v[e];
        if (a.out_prev) {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            float2 p1;
            if constexpr (kTwo) {
              p1 = c1[e];
            } else {
              const int idx = F::in_index(t, e);
              const float2 l1 = sb[idx];   // B is untouched by a single-area transform
              p1 = keep_if(full1 || ((msk[idx >> 5] >> (idx & 31)) & 1u), l1);
            }
            a.out_prev[base + F::in_index(t, e)] = p1;
          }
        }
      }
      return;   // uniform over the grid
    }
    if (a.keep_c && active) {
#pragma unroll
      for (int e = 0; e < E; ++e) a.keep_c[base + F::in_index(t, e)] = v[e];
    }
    // store c_t: slots if the row has at most CAP nonzeros, the dense row otherwise
    int mine = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) mine += (v[e].x != 0.f || v[e].y != 0.f) ? 1 : 0;
    int total, before;
    row_prefix<T>(mine, t, rowcnt, total, before);
    if (active) {
      if (total > CAP) {
#pragma unroll
        for (int e = 0; e < E; ++e) a.b0.dense[base + F::in_index(t, e)] = v[e];
      } else {
        int o = before;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if (v[e].x != 0.f || v[e].y != 0.f) {
            a.b0.sidx[static_cast<size_t>(prow) * CAP + o] = static_cast<unsigned short>(F::in_index(t, e));
            a.b0.sval[static_cast<size_t>(prow) * CAP + o] = v[e];
            ++o;
          }
        }
      }
      if (t == 0) a.b0.cnt[prow] = total > CAP ? CAP + 1 + total : total;
    }
    // z_{t+1} = c_t + beta_t (c_t - c_{t-1}); its row DFT on the kept columns
    int zmine = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      float2 p1;
      if constexpr (kTwo) {
        p1 = c1[e];
      } else {
        const int idx = F::in_index(t, e);
        const float2 l1 = sb[idx];   // B is untouched by a single-area transform
        p1 = keep_if(full1 || ((msk[idx >> 5] >> (idx & 31)) & 1u), l1);
      }
      v[e] = make_float2(v[e].x + a.beta * (v[e].x - p1.x), v[e].y + a.beta * (v[e].y - p1.y));
      zmine += (v[e].x != 0.f || v[e].y != 0.f) ? 1 : 0;
    }
    int ztot, zbefore;
    row_prefix<T>(zmine, t, rowcnt, ztot, zbefore);
    // A sparse z_{t+1} (at most CAP nonzeros in every row of the group) takes the
    // kept bins as direct sums over its nonzeros; otherwise the row FFT.  The
    // group deciding together is the wavefront when rows sync per wave, else the
    // block (the FFT's barriers are then block-wide).
    bool use_fft;
    if constexpr (kWave) use_fft = __any(ztot > CAP);
    else use_fft = __syncthreads_or(ztot > CAP);
    if (use_fft) {
      fft_fwd_after_inv<F>(v, t, stw, sa, sb);
      if (active) {
#pragma unroll
        for (int e = 0; e < E; ++e)
          if (ks[e] >= 0) a.xy[xrow + ks[e]] = v[e];
      }
    } else {
      // the row's nonzeros, compact: values in A, positions in B (both free now:
      // the inverse transform and the reads of B finished before the decision)
      if constexpr (kWave) lds_sync<true>();
      int* zpos = reinterpret_cast<int*>(sb);
      int o = zbefore;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (v[e].x != 0.f || v[e].y != 0.f) {
          sa[o] = v[e];
          zpos[o] = F::in_index(t, e);
          ++o;
        }
      }
      lds_sync<kWave>();
      if (active) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if (ks[e] >= 0) {
            const int k = F::out_index(t, e);
            float2 acc = make_float2(0.f, 0.f);
            for (int q = 0; q < ztot; ++q) {
              const float2 w = stw[(k * zpos[q]) & (N - 1)];   // e^{-j 2 pi k l / N}
              acc = cadd(acc, cmul(sa[q], w));
            }
            a.xy[xrow + ks[e]] = acc;
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Column pass: a block owns W adjacent columns of one scene; lane = c + W*t.
// Dynamic LDS: W * (one or two padded exchange areas), column c at stride W, + N twiddles.
// ---------------------------------------------------------------------------
template <int N, int E, int MODE>
__global__ __launch_bounds__(256) void k_col(ColArgs a, int W) {
  using F = Stockham<N, E>;
  constexpr int T = F::T;
  constexpr int AR = fft_areas(N, E);
  constexpr int FA = fft_area(N);
  extern __shared__ float2 lds[];
  float2* stw = lds + AR * W * FA;
  int bid;
  if (!spread_block(a.spread, bid)) return;  // whole block exits together

  // XCD-aware strip order: a GPU that deals consecutive blocks to its 8 dies in
  // turn gives die x the blocks x, x+8, ...; they take adjacent column strips,
  // so strips sharing a cache line are read through one L2
  {
    const int nb = static_cast<int>(gridDim.x);
    if (a.spread <= 1 && (nb & 7) == 0) bid = (bid & 7) * (nb >> 3) + (bid >> 3);
  }
  const int tid = threadIdx.x;
  const int nthreads = W * T;
  const int c = tid % W, t = tid / W;
  const int ncols = a.ncols ? a.ncols : a.L1;
  const int ldx = a.ldx ? a.ldx : a.L1;
  const int strips = ncols / W;
  const int lscene = bid / strips;
  const int col = (bid - lscene * strips) * W + c;
  const int scene = a.scene_map ? a.scene_map[lscene] : lscene;
  const size_t plane = static_cast<size_t>(N) * ldx;
  float2* g = a.xy + scene * plane + col;
  float2* sms = lds + c;                    // column c's exchange slots, stride W
  float2* sms2 = sms + (AR - 1) * W * FA;   // second area (two-area transforms)
  const int k1 = a.scol ? a.scol[scene * a.scol_stride + col] : col;   // spectral column

  constexpr bool kSparse = (MODE == COL_SPARSE_AFFINE || MODE == COL_SPARSE_ADMM || MODE == COL_PRUNED_AFFINE);
  constexpr bool kDil = (MODE == COL_PRUNED_CPLX);
  constexpr bool kPsi = (MODE == COL_PRUNED_ADMM || MODE == COL_PRUNED_EXPAND);
  constexpr bool kFwd = (MODE == COL_FWD || MODE == COL_FILTER_AFFINE || MODE == COL_FILTER_ADMM ||
                         MODE == COL_FILTER_CPLX || kSparse || kDil || MODE == COL_PRUNED_ADMM);
  constexpr bool kInv = (MODE != COL_FWD);
  constexpr bool kMul = (MODE != COL_FWD && MODE != COL_INV && !kSparse && !kDil && !kPsi);
  constexpr bool kCplx = (MODE == COL_FILTER_CPLX);

  // all global loads first (iterate, spectral multiplier, twiddles)
  float2 v[E];
  if constexpr (kFwd) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = g[static_cast<size_t>(F::in_index(t, e)) * ldx];
  } else if constexpr (MODE == COL_PRUNED_EXPAND) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = make_float2(0.f, 0.f);
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = g[static_cast<size_t>(F::out_index(t, e)) * ldx];
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

  if constexpr (kFwd) fft_fwd<F>(v, t, stw, sms, sms2, false, W);

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
    } else if constexpr (MODE == COL_PRUNED_AFFINE) {
      ab = make_float2(0.f, a.coef[scene].y);   // correction only: the identity stays spatial
      mdef = 0.f;
    } else {
      mdef = a.scale / a.rho;
    }
    float2 src[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      src[e] = v[e];
      v[e] = cscale(v[e], mdef);
    }
    const int* ptr = a.sup_ptr + scene * a.sup_ptr_stride + (k1 >= 0 ? k1 : 0);
    const int j0 = ptr[0], j1 = k1 >= 0 ? ptr[1] : j0;   // padding columns: no entries
    const float2* rhs = a.sup_rhs + scene * a.sup_rhs_stride;
    for (int j = j0; j < j1; ++j) {
      const SupEntry en = a.sup[j];
      const float2 r = rhs[j];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (F::out_index(t, e) == en.k2) {
          if constexpr (MODE == COL_SPARSE_AFFINE || MODE == COL_PRUNED_AFFINE) {
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

  if constexpr (kPsi) {
    // the column carries Psi_{t+1} (ADMM) or vlast (EXPAND) on its support bins,
    // zero elsewhere; each bin is held by one thread, which alone touches its entry
    float2 src[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      src[e] = v[e];
      v[e] = make_float2(0.f, 0.f);
    }
    const int* ptr = a.sup_ptr + scene * a.sup_ptr_stride + (k1 >= 0 ? k1 : 0);
    const int j0 = ptr[0], j1 = k1 >= 0 ? ptr[1] : j0;   // padding columns: no entries
    const size_t sb = static_cast<size_t>(scene) * a.sup_rhs_stride;
    for (int j = j0; j < j1; ++j) {
      const SupEntry en = a.sup[j];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (F::out_index(t, e) == en.k2) {
          if constexpr (MODE == COL_PRUNED_EXPAND) {
            v[e] = a.vlast[sb + j];
          } else {
            const float d = 1.f / (en.omega + a.rho);
            const float om = en.omega * a.scale;
            const float2 r = a.sup_rhs[sb + j], p0 = a.psi[sb + j];
            const float2 vp = make_float2((r.x - a.rho * p0.x - om * src[e].x) * d, (r.y - a.rho * p0.y - om * src[e].y) * d);
            const float2 pn = make_float2(p0.x + vp.x, p0.y + vp.y);
            a.psi[sb + j] = pn;
            a.vlast[sb + j] = vp;
            v[e] = pn;
          }
        }
      }
    }
  }

  if constexpr (kDil) {
    // correction only (the identity stays spatial): m = mulc - 1/L on the dilated
    // support bins of this column, zero elsewhere; r = (mu_k / mu) (mu S) on the plan's bins
    float2 src[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      src[e] = v[e];
      v[e] = make_float2(0.f, 0.f);
    }
    const int* ptr = a.sup_ptr + (k1 >= 0 ? k1 : 0);
    const int j0 = ptr[0], j1 = k1 >= 0 ? ptr[1] : j0;   // padding columns: no entries
    const float rs = a.dscal[1] * a.inv_mu;
    const float invL = a.scale;
    const float2* rhs = a.sup_rhs + scene * a.sup_rhs_stride;
    for (int j = j0; j < j1; ++j) {
      const DilEntry en = a.dil[j];
      float2 m = a.mulc[static_cast<size_t>(en.k2) * a.L1 + k1];
      m.x -= invL;
      float2 r = make_float2(0.f, 0.f);
      if (en.orig >= 0) {
        const float2 q = rhs[en.orig];
        r = make_float2(rs * q.x, rs * q.y);
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (F::out_index(t, e) == en.k2) {
          const float2 p = cmul(src[e], m);
          v[e] = make_float2(p.x + r.x, p.y + r.y);
        }
      }
    }
  }

  if constexpr (kInv) {
    if constexpr (kFwd) fft_inv_after_fwd<F>(v, t, stw, sms, sms2, W);
    else fft_inv<F>(v, t, stw, sms, sms2, false, W);
    const float s = (MODE == COL_INV) ? a.scale : 1.f;
#pragma unroll
    for (int e = 0; e < E; ++e) g[static_cast<size_t>(F::in_index(t, e)) * ldx] = cscale(v[e], s);
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) g[static_cast<size_t>(F::out_index(t, e)) * ldx] = v[e];
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
  const bool pruned = (mode == ROW_PRUNED || mode == ROW_PRUNED_FWD);
  const size_t shm = pruned ? static_cast<size_t>(rowp_lds_floats(N, E, rpb, a.ncs)) * sizeof(float2)
                            : (static_cast<size_t>(fft_areas(N, E)) * rpb * fft_area(N) + N) * sizeof(float2) +
                                  (mode == ROW_FISTA_SP ? static_cast<size_t>(rpb) * T * sizeof(int) : 0);
  if (shm > 65536) return -1;
  if (mode == ROW_FISTA_SP && (!a.cnt || !a.sidx || !a.sval || !a.state)) return -1;
  if (pruned && (!a.colslot || a.ncs < 1 || a.ncs > N / 2)) return -1;
  if (mode == ROW_PRUNED && (!a.b1.cnt || !a.b1.sidx || !a.b1.sval || !a.b1.dense || !a.b0.cnt || !a.b0.sidx ||
                             !a.b0.sval || !a.b0.dense || !a.out_c ||
                             (a.b2.cnt && (!a.b2.sidx || !a.b2.sval || !a.b2.dense))))
    return -1;
  const int spread = a.spread > 1 ? a.spread : 1;
  const dim3 grid(blocks * spread), block(rpb * T);
  switch (mode) {
    case ROW_FISTA_SP: hipLaunchKernelGGL((k_row<N, E, ROW_FISTA_SP>), grid, block, shm, s, a, rpb); break;
    case ROW_PRUNED_FWD: hipLaunchKernelGGL((k_rowp<N, E, ROW_PRUNED_FWD>), grid, block, shm, s, a, rpb); break;
    case ROW_PRUNED: hipLaunchKernelGGL((k_rowp<N, E, ROW_PRUNED>), grid, block, shm, s, a, rpb); break;
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
  const int ncols = a.ncols ? a.ncols : a.L1;
  if (W < 1 || W * T > 256 || ncols % W != 0) return -1;
  const bool pruned = mode == COL_PRUNED_AFFINE || mode == COL_PRUNED_CPLX || mode == COL_PRUNED_ADMM ||
                      mode == COL_PRUNED_EXPAND;
  if (pruned != (a.scol != nullptr)) return -1;
  if (mode == COL_PRUNED_CPLX && (!a.dil || !a.dscal || !a.mulc || !a.sup_rhs)) return -1;
  if ((mode == COL_PRUNED_ADMM || mode == COL_PRUNED_EXPAND) && (!a.sup_ptr || !a.sup || !a.vlast)) return -1;
  if (mode == COL_PRUNED_ADMM && (!a.psi || !a.sup_rhs || !(a.rho > 0.f))) return -1;
  const int blocks = (ncols / W) * a.nscenes;
  if (blocks <= 0) return 0;
  const size_t shm = (static_cast<size_t>(fft_areas(N, E)) * W * fft_area(N) + N) * sizeof(float2);
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
    case COL_PRUNED_AFFINE: hipLaunchKernelGGL((k_col<N, E, COL_PRUNED_AFFINE>), grid, block, shm, s, a, W); break;
    case COL_PRUNED_CPLX: hipLaunchKernelGGL((k_col<N, E, COL_PRUNED_CPLX>), grid, block, shm, s, a, W); break;
    case COL_PRUNED_ADMM: hipLaunchKernelGGL((k_col<N, E, COL_PRUNED_ADMM>), grid, block, shm, s, a, W); break;
    case COL_PRUNED_EXPAND: hipLaunchKernelGGL((k_col<N, E, COL_PRUNED_EXPAND>), grid, block, shm, s, a, W); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace bccb
