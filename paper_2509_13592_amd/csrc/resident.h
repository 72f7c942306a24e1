// Single-scene solver in one cooperative launch.
//
// The two-pass iteration (column pass, then row pass, see passes.h) moves the
// row-spectral grid through memory twice per iteration and pays two kernel
// boundaries.  For one scene of a few hundred thousand points the boundaries
// dominate.  Here G workgroups stay resident for the whole solve: workgroup g
// owns L2/G rows and L1/G columns of the grid, the per-row state (c^(t-1) of
// FISTA, v of ADMM) and the per-column spectral multiplier (Omega and the
// right-hand side on the support bins, eq. (21)) live in its registers, and
// the phases are separated by grid barriers instead of launches.  Per
// iteration: column phase (DFT_cols, multiply, IDFT_cols on the owned
// columns), barrier, row phase (IDFT_rows, the proximal / momentum / ADMM
// update of eqs. (9)-(15), DFT_rows on the owned rows), barrier.  The
// arithmetic is that of the two-pass path at E = 4 element for element.
// A pruned form of all three solvers (k_resident_pruned, further down)
// exchanges only per-group parts of the spectrum at the support bins and needs
// one barrier per iteration.
//
// The launch is cooperative (all G workgroups co-resident, or the launch
// fails), and every barrier wait is bounded in wall-clock time: a workgroup
// that waits too long raises the abort word and the flag, and every
// workgroup then leaves at its next barrier.
#pragma once

#include "passes.h"
#include "resident_api.h"

namespace bccb {

constexpr int kResidentElems = 4;

// NT threads per workgroup: 256 (1024-point chunks, 1..4 per workgroup and
// phase) or 128 (one 512-point chunk, for twice the workgroups).
template <int N1, int N2, int NT_>
struct ResidentShape {
  static constexpr int E = kResidentElems;
  static constexpr int NT = NT_;
  static constexpr int T1 = N1 / E, T2 = N2 / E;
  static constexpr int RPC = NT / T1;   // rows per chunk of the row phase
  static constexpr int CPC = NT / T2;   // columns per chunk of the column phase
  static constexpr int AR1 = fft_areas(N1, E), AR2 = fft_areas(N2, E);
  static constexpr int FA1 = fft_area(N1), FA2 = fft_area(N2);
  static constexpr int WORK = (RPC * AR1 * FA1 > CPC * AR2 * FA2) ? RPC * AR1 * FA1 : CPC * AR2 * FA2;
  static constexpr size_t LDS_BYTES = static_cast<size_t>(N1 + N2 + WORK) * sizeof(float2);
};

// Grid barrier number k (k = 1, 2, ...) of the solve tagged a.tag.  Every wave
// waits for its own stores to complete and the block meets; thread 0 publishes
// the block's stores at agent scope (one L2 write-back per block rather than one
// per wave) and writes tag | k to the block's arrival word (its own 128-byte
// line: arrivals do not contend on one address); the first wave then polls all
// G arrival words at once, one per lane, until every one holds tag | k or more
// (bounded in wall-clock time; a timeout writes the tag into the abort word and
// raises the flag, and an abort word holding the tag ends the wait), acquires
// for the block (its waves share one CU and its L1) and the block meets again.
// Words are never reset: whatever an earlier solve left is below this solve's
// tag.  Returns false when the solve is being abandoned.  kFences = false leaves
// out the agent-scope release and acquire (the L2 write-back and invalidate): for
// a caller whose exchanged data are written with store_through (complete once
// the wait above returns) and read back only with agent-scope loads issued after
// the barrier, which see the coherent copy as the arrival words do.
template <bool kFences = true>
__device__ __forceinline__ bool resident_sync(const ResidentArgs& a, int g, unsigned k, int* s_ok) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const int tid = threadIdx.x;
  if (tid < 64) {
    unsigned long long* arrive = a.sync + kResidentArriveOffset;
    const unsigned long long want = a.tag | k;
    if (tid == 0) {
      if constexpr (kFences) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(arrive + static_cast<size_t>(g) * kResidentArriveStride, want, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    int ok = 1;
    const long long t0 = wall_clock64();
    unsigned spins = 0;
    // a bounded wait step: false (and ok = 0) when the solve is abandoned; the abort
    // word is read every 64th step only, since waiting for it would also wait for
    // any poll load still in flight
    auto keep_waiting = [&]() -> bool {
      if ((++spins & 63) == 0 && __hip_atomic_load(a.sync, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == a.tag) {
        ok = 0;
        return false;
      }
      if (wall_clock64() - t0 > a.timeout_ticks) {
        if (tid == 0) {
          __hip_atomic_store(a.sync, a.tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_fetch_or(a.flag, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        ok = 0;
        return false;
      }
      __builtin_amdgcn_s_sleep(1);
      return true;
    };
    if (a.groups <= 64) {
      // one word per lane, polled by two rounds of loads in flight at once (two
      // registers taken in turn, no copy between them), so an arrival is seen
      // within about half a round trip of landing instead of a whole one
      const bool has = tid < a.groups;
      const unsigned long long* mw = arrive + static_cast<size_t>(has ? tid : 0) * kResidentArriveStride;
      unsigned long long pa = __hip_atomic_load(mw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_s_sleep(2);
      unsigned long long pb = __hip_atomic_load(mw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      while (true) {
        if (__all(!has || pa >= want)) break;
        pa = __hip_atomic_load(mw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!keep_waiting()) break;
        if (__all(!has || pb >= want)) break;
        pb = __hip_atomic_load(mw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!keep_waiting()) break;
      }
    } else {
      while (true) {
        bool mine = true;
        for (int i = tid; i < a.groups; i += 64)
          mine = mine && __hip_atomic_load(arrive + static_cast<size_t>(i) * kResidentArriveStride, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT) >= want;
        if (__all(mine)) break;
        if (!keep_waiting()) break;
      }
    }
    if constexpr (kFences) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (tid == 0) *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

// Agent-scope load of exchanged data: reads the coherent copy, never a stale
// line of this die's L2.
__device__ __forceinline__ float2 load_coherent(float2* p) {
  return __builtin_bit_cast(float2, __hip_atomic_load(reinterpret_cast<unsigned long long*>(p), __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT));
}

// Store of exchanged data, written through to the agent-coherent level at once
// (an agent-scope relaxed atomic store), so the block's release before a
// barrier finds no dirty lines of it to write back.
__device__ __forceinline__ void store_through(float2* p, float2 v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), __builtin_bit_cast(unsigned long long, v),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int N1, int N2, int MODE, int NT_>
__global__ __launch_bounds__(256) void k_resident(ResidentArgs a) {
  using S = ResidentShape<N1, N2, NT_>;
  constexpr int E = S::E, NT = S::NT, T1 = S::T1, RPC = S::RPC, CPC = S::CPC;
  constexpr int MAXCH = kResidentMaxChunks;
  using FR = Stockham<N1, E, (T1 <= 64)>;   // a row inside one wavefront: row-local exchanges sync the wave
  using FC = Stockham<N2, E>;
  constexpr bool kFista = (MODE == RES_FISTA);
  constexpr bool kAdmm = (MODE == RES_ADMM);
  constexpr bool kState = kFista || kAdmm;
  extern __shared__ float2 lds[];
  __shared__ int s_ok;
  float2* tw1 = lds;
  float2* tw2 = lds + N1;
  float2* work = tw2 + N2;

  int g;
  if (!spread_block(a.spread, g)) return;   // whole block exits together
  const int G = a.groups;
  const int nch = (N1 * N2) / (E * NT * G);   // chunks per phase, 1..MAXCH (checked by the launcher)
  const int tid = threadIdx.x;
  const int rr = tid / T1, rt = tid - (tid / T1) * T1;   // row phase: row in chunk, thread in row
  float2* rA = work + S::AR1 * rr * S::FA1;
  float2* rB = rA + (S::AR1 - 1) * S::FA1;
  const int cc = tid % CPC, ct = tid / CPC;               // column phase: column in chunk, thread in column
  float2* cA = work + cc;
  float2* cB = cA + (S::AR2 - 1) * CPC * S::FA2;
  const int row0 = g * (N2 / G), col0 = g * (N1 / G);
  const float2 zero = make_float2(0.f, 0.f);

  for (int j = tid; j < N1; j += NT) tw1[j] = a.tw1[j];
  for (int j = tid; j < N2; j += NT) tw2[j] = a.tw2[j];

  // Spectral multiplier of the owned columns: m off the support, its value and
  // the right-hand side r on the support bins (as the sparse column modes).
  float cm[MAXCH][E];
  float2 cr[MAXCH][E];
  {
    float mdef;
    float2 ab = zero;
    if constexpr (kAdmm) {
      mdef = a.scale / a.rho;
    } else {
      ab = a.coef[0];
      mdef = ab.x;
    }
#pragma unroll
    for (int ch = 0; ch < MAXCH; ++ch) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        cm[ch][e] = mdef;
        cr[ch][e] = zero;
      }
      if (ch < nch) {
        const int k1 = col0 + ch * CPC + cc;
        const int j0 = a.sup_ptr[k1], j1 = a.sup_ptr[k1 + 1];
        for (int j = j0; j < j1; ++j) {
          const SupEntry en = a.sup[j];
          const float2 r = a.sup_rhs[j];
#pragma unroll
          for (int e = 0; e < E; ++e) {
            if (FC::out_index(ct, e) == en.k2) {
              if constexpr (kAdmm) {
                const float d = 1.f / (en.omega + a.rho);
                cm[ch][e] = a.scale * d;
                cr[ch][e] = make_float2(r.x * d, r.y * d);
              } else {
                cm[ch][e] = ab.x + ab.y * en.omega;
                cr[ch][e] = r;
              }
            }
          }
        }
      }
    }
  }

  // Start: FISTA/ISTA take z^(1) = c^(0) (the warm start, or zero), ADMM z - v = 0;
  // the owned rows' DFT_rows goes to xy.
  float2 st[kState ? MAXCH : 1][E];
#pragma unroll
  for (int ch = 0; ch < MAXCH; ++ch) {
    if (ch < nch) {
      const size_t base = static_cast<size_t>(row0 + ch * RPC + rr) * N1;
      float2 v[E];
      if (!kAdmm && a.init) {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = a.init[base + FR::in_index(rt, e)];
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = zero;
      }
      bool ok = true;
#pragma unroll
      for (int e = 0; e < E; ++e) ok = ok && finite2(v[e]);
      if (!ok) __hip_atomic_fetch_or(a.flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if constexpr (kState) {
#pragma unroll
        for (int e = 0; e < E; ++e) st[ch][e] = v[e];
      }
      __syncthreads();   // twiddles in place; the previous chunk is done with the areas
      fft_fwd<FR>(v, rt, tw1, rA, rB, false);
#pragma unroll
      for (int e = 0; e < E; ++e) store_through(a.xy + base + FR::out_index(rt, e), v[e]);
    }
  }
  unsigned epoch = 1;
  if (!resident_sync(a, g, epoch, &s_ok)) return;

  for (int t = 1; t <= a.iters; ++t) {
    // column phase: DFT_cols -> multiplier -> IDFT_cols on the owned columns
#pragma unroll
    for (int ch = 0; ch < MAXCH; ++ch) {
      if (ch < nch) {
        float2* gcol = a.xy + (col0 + ch * CPC + cc);
        float2 v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = gcol[static_cast<size_t>(FC::in_index(ct, e)) * N1];
        __syncthreads();
        fft_fwd<FC>(v, ct, tw2, cA, cB, false, CPC);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const float m = cm[ch][e];
          const float2 r = cr[ch][e];
          v[e] = make_float2(v[e].x * m + r.x, v[e].y * m + r.y);
        }
        fft_inv_after_fwd<FC>(v, ct, tw2, cA, cB, CPC);
#pragma unroll
        for (int e = 0; e < E; ++e) store_through(gcol + static_cast<size_t>(FC::in_index(ct, e)) * N1, v[e]);
      }
    }
    if (!resident_sync(a, g, ++epoch, &s_ok)) return;

    // row phase: IDFT_rows -> update -> DFT_rows on the owned rows
    const bool last = (t == a.iters);
    const float beta = kFista ? a.beta[t - 1] : 0.f;
#pragma unroll
    for (int ch = 0; ch < MAXCH; ++ch) {
      if (ch < nch) {
        const size_t base = static_cast<size_t>(row0 + ch * RPC + rr) * N1;
        float2 v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = a.xy[base + FR::out_index(rt, e)];
        __syncthreads();
        fft_inv<FR>(v, rt, tw1, rA, rB);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const size_t idx = base + FR::in_index(rt, e);
          if constexpr (MODE == RES_ISTA) {
            const float2 c = shrink(v[e], a.kappa);
            if (last) a.out_c[idx] = c;
            v[e] = c;
          } else if constexpr (kFista) {
            const float2 c = shrink(v[e], a.kappa);
            const float2 cp = st[ch][e];
            st[ch][e] = c;
            if (last) a.out_c[idx] = c;
            v[e] = make_float2(c.x + beta * (c.x - cp.x), c.y + beta * (c.y - cp.y));
          } else {   // ADMM: c = w + IDFT(...) with w applied spectrally, z = S(c + v), v += c - z
            const float2 c = v[e];
            const float2 vv = st[ch][e];
            const float2 z = shrink(cadd(c, vv), a.kappa);
            const float2 vn = csub(cadd(vv, c), z);
            st[ch][e] = vn;
            if (last) {
              a.out_z[idx] = z;
              if (a.out_c) a.out_c[idx] = c;
            }
            v[e] = csub(z, vn);
          }
        }
        if (!last) {
          fft_fwd_after_inv<FR>(v, rt, tw1, rA, rB);
#pragma unroll
          for (int e = 0; e < E; ++e) store_through(a.xy + base + FR::out_index(rt, e), v[e]);
        }
      }
    }
    if (!last) {
      if (!resident_sync(a, g, ++epoch, &s_ok)) return;
    }
  }
}

template <int N1, int N2, int MODE, int NT>
int resident_launch_t(const ResidentArgs& a, int check_only, hipStream_t s) {
  using S = ResidentShape<N1, N2, NT>;
  const int G = a.groups;
  const long per = static_cast<long>(N1) * N2 / G;
  if (per % (S::E * S::NT) != 0 || per / (S::E * S::NT) < 1 || per / (S::E * S::NT) > kResidentMaxChunks) return -1;
  if (S::RPC > N2 || S::CPC > N1 || (N2 / G) % S::RPC != 0 || (N1 / G) % S::CPC != 0) return -1;
  const int spread = a.spread > 1 ? a.spread : 1;
  const auto kfn = k_resident<N1, N2, MODE, NT>;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, S::NT, S::LDS_BYTES) != hipSuccess) return -4;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -4;
  if (static_cast<long>(per_cu) * cus < static_cast<long>(G) * spread) return -1;
  if (check_only) return 0;
  if (!a.xy || !a.tw1 || !a.tw2 || !a.sup_ptr || !a.sup || !a.sup_rhs || !a.sync || !a.flag || a.iters < 1) return -1;
  if (MODE == RES_FISTA && !a.beta) return -1;
  if (MODE != RES_ADMM && (!a.out_c || !a.coef)) return -1;
  if (MODE == RES_ADMM && !a.out_z) return -1;
  void* args[] = {const_cast<ResidentArgs*>(&a)};
  const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kfn), dim3(G * spread), dim3(S::NT), args,
                                                  static_cast<unsigned>(S::LDS_BYTES), s);
  return e == hipSuccess ? 0 : -4;
}

// Launch (check_only: only report whether the shape can be launched co-resident).
// 256 threads when each group gets whole 1024-point chunks, 128 threads when it
// gets one 512-point chunk.
template <int N1, int N2, int MODE>
int resident_launch_m(const ResidentArgs& a, int check_only, hipStream_t s) {
  const int G = a.groups;
  if (G < 1 || G > kResidentMaxGroups || N2 % G != 0 || N1 % G != 0) return -1;
  const long per = static_cast<long>(N1) * N2 / G;
  if (per >= 1024) return resident_launch_t<N1, N2, MODE, 256>(a, check_only, s);
  if (per == 512) return resident_launch_t<N1, N2, MODE, 128>(a, check_only, s);
  return -1;
}

// ---------------------------------------------------------------------------
// Pruned form.  By eq. (21) Omega and DFT2(b) vanish off the support bins, so
// (I - mu G) z + mu b = z + IDFT2(V) with V = m . DFT2(z) + r living on the
// support (m = -mu Omega / L, r = mu S, as the pruned column pass).  ADMM's
// x-update (G + rho I)^-1 (b + rho (z - v)) differs from z - v only on the
// support as well (the inverse is 1 / rho off it); see the ADMM note below.  Group g owns RPC = 1024 / L1 rows (G = L2 / RPC groups of 256
// threads) with z_t and c_{t-1} in registers.  DFT2(z_t) at a support bin
// (k1, k2) is a sum over the rows of DFT_rows(z_t)[l2][k1] e^{-j 2 pi k2 l2 / L2};
// each group publishes the part of that sum over its own rows for every bin
// (nsup values), and after the one grid barrier of an iteration every group
// adds the G parts of every bin in a fixed order.  An iteration:
//   Z_j = sum over groups of the parts; V_j = m_j Z_j + r_j;
//   the owned rows' kept spectra of IDFT2(V): sums over the bins of each kept
//   column with the rows' twiddles (a table built once); IDFT_rows of them
//   (zero off the kept columns); u = z_t + that; c_t = S_kappa(u);
//   z_{t+1} = c_t + beta_t (c_t - c_{t-1}); DFT_rows(z_{t+1}) at the kept
//   columns; this group's parts of DFT2(z_{t+1}) at the bins -> xy; barrier.
// ADMM (eqs. (13)-(15)): with rho << Omega the scaled dual v grows to about
// S / rho on the support modes, far above x, so x formed as (z - v) plus a
// support correction would cancel in FP32.  The dual is therefore split as
// v_t = u_t + IDFT2(Psi_t): Psi (nsup values, the same in every group, since
// every group forms the same sums in the same order) carries the support part
// and u_t = z_{t-1} - z_t the rest.  With Y = DFT2(z_t - u_t) at the bins,
//   V'_j = (S_j - rho Psi_j - Omega_j Y_j / L) / (Omega_j + rho),
//   x_{t+1} = z_t - u_t + IDFT2(V'),  Psi_{t+1} = Psi_t + V',
//   z_{t+1} = S_{tau/rho}(x_{t+1} + v_t) = S_{tau/rho}(z_t + IDFT2(Psi_{t+1})),
//   u_{t+1} = z_t - z_{t+1},
// which is the update of eqs. (13)-(15) rearranged: only small quantities meet
// in a subtraction, and one row transform per iteration remains (x itself is
// formed at the last iteration only).  Registers hold z_t and z_{t-1}; the
// published parts are those of DFT2(2 z_t - z_{t-1}).
// The column transforms of the passes become these sums, so the results agree
// with the pruned passes to FP32 rounding, not element for element.
// ---------------------------------------------------------------------------
template <int N1, int N2, int NT_>
struct ResidentPrunedShape {
  static constexpr int E = kResidentElems;
  static constexpr int NT = NT_;   // 256 or 512 threads per group
  static constexpr int T1 = N1 / E;
  static constexpr int RPC = NT / T1;   // rows per group
  static constexpr int AR1 = fft_areas(N1, E), FA1 = fft_area(N1);
  // dynamic LDS in bytes for ncs kept columns and nsup support bins (ADMM keeps
  // Psi, V' and -rho / (Omega + rho) per bin as well)
  static constexpr size_t lds_bytes(int ncs, int nsup, bool admm) {
    const size_t na = admm ? static_cast<size_t>(nsup) : 0;
    return sizeof(float2) * (static_cast<size_t>(N1) + static_cast<size_t>(RPC) * AR1 * FA1 +
                             static_cast<size_t>(RPC) * nsup + static_cast<size_t>(RPC) * ncs + 2 * static_cast<size_t>(nsup) +
                             2 * na) +
           sizeof(float) * (nsup + na) + sizeof(int) * (static_cast<size_t>(nsup) + 2 * static_cast<size_t>(ncs));
  }
};

template <int N1, int N2, int MODE, int NT_>
__global__ __launch_bounds__(512) void k_resident_pruned(ResidentArgs a) {
  using S = ResidentPrunedShape<N1, N2, NT_>;
  constexpr int E = S::E, NT = S::NT, T1 = S::T1, RPC = S::RPC;
  using FR = Stockham<N1, E, (T1 <= 64)>;
  constexpr bool kFista = (MODE == RES_PRUNED_FISTA);
  constexpr bool kAdmm = (MODE == RES_PRUNED_ADMM);
  constexpr int PB = 16;   // parts loaded per thread and batch
  extern __shared__ float2 lds[];
  __shared__ int s_ok;
  const int ncs = a.ncs, nsup = a.nsup, G = a.groups;
  float2* tw1 = lds;
  float2* area = tw1 + N1;                              // RPC rows x AR1 exchange areas
  float2* cw = area + RPC * S::AR1 * S::FA1;            // [RPC][nsup] e^{+j 2 pi k2_j l2 / L2}, owned rows
  float2* xk = cw + RPC * nsup;                         // [RPC][ncs] owned rows' kept forward spectra
  const int na = kAdmm ? nsup : 0;
  float2* vs = xk + RPC * ncs;                          // [nsup] V_j (ADMM: Psi_{t+1})
  float2* br = vs + nsup;                               // [nsup] r_j
  float2* ps = br + nsup;                               // [na] ADMM: Psi_j
  float2* vd = ps + na;                                 // [na] ADMM: V'_j of the last iteration
  float* bm = reinterpret_cast<float*>(vd + na);        // [nsup] m_j
  float* bq = bm + nsup;                                // [na] ADMM: -rho / (Omega_j + rho)
  int* bslot = reinterpret_cast<int*>(bq + na);         // [nsup] kept slot of bin j
  int* sbeg = bslot + nsup;                             // [ncs] bins of slot s: sbeg[s] .. send[s]
  int* send = sbeg + ncs;

  int g;
  if (!spread_block(a.spread, g)) return;   // whole block exits together
  const int tid = threadIdx.x;
  const int rr = tid / T1, rt = tid - (tid / T1) * T1;
  const int row = g * RPC + rr;
  float2* rA = area + S::AR1 * rr * S::FA1;
  float2* rB = rA + (S::AR1 - 1) * S::FA1;
  const size_t base = static_cast<size_t>(row) * N1;
  const float2 zero = make_float2(0.f, 0.f);
  // [2][G][nsup] parts of DFT2(z) at the bins, one row block per group, in the
  // buffer of the iteration's parity: a group can refill a buffer only after the
  // next barrier, which every reader of its previous contents has passed
  float2* const parts = a.xy;
  const size_t pstride = static_cast<size_t>(G) * nsup;

  for (int j = tid; j < N1; j += NT) tw1[j] = a.tw1[j];
  {
    const float cb = kAdmm ? -a.scale / a.rho : a.coef[0].y;   // -1 / L (ADMM), -mu / L
    for (int s2 = tid; s2 < ncs; s2 += NT) {
      const int k1 = a.scol[s2];
      const int j0 = k1 >= 0 ? a.sup_ptr[k1] : 0, j1 = k1 >= 0 ? a.sup_ptr[k1 + 1] : 0;
      sbeg[s2] = j0;
      send[s2] = j1;
      for (int j = j0; j < j1; ++j) {
        const SupEntry en = a.sup[j];
        bslot[j] = s2;
        if constexpr (kAdmm) {
          const float d = 1.f / (en.omega + a.rho);
          const float2 r = a.sup_rhs[j];
          bm[j] = cb * en.omega * d;
          br[j] = make_float2(r.x * d, r.y * d);
          bq[j] = -a.rho * d;
          ps[j] = zero;
        } else {
          bm[j] = cb * en.omega;
          br[j] = a.sup_rhs[j];
        }
        for (int r2 = 0; r2 < RPC; ++r2) {
          const float2 w = a.tw2[(en.k2 * (g * RPC + r2)) & (N2 - 1)];
          cw[r2 * nsup + j] = make_float2(w.x, -w.y);
        }
      }
    }
  }
  int myslot[E];
#pragma unroll
  for (int e = 0; e < E; ++e) myslot[e] = a.colslot[FR::out_index(rt, e)];

  // this group's parts of DFT2(v) at the bins, from the kept forward row spectra
  // v[] of its rows (forward-output layout); the block meets inside
  auto publish = [&](const float2* v, float2* part) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (myslot[e] >= 0) xk[rr * ncs + myslot[e]] = v[e];
    __syncthreads();
    for (int j = tid; j < nsup; j += NT) {
      const int sl = bslot[j];
      float2 acc = zero;
      for (int r2 = 0; r2 < RPC; ++r2) {
        const float2 x = xk[r2 * ncs + sl];
        const float2 w = cw[r2 * nsup + j];   // conj: forward
        acc = make_float2(acc.x + x.x * w.x + x.y * w.y, acc.y + x.y * w.x - x.x * w.y);
      }
      store_through(part + static_cast<size_t>(g) * nsup + j, acc);
    }
  };

  // z_1 = c_0 (warm start or zero), c_{-1} = c_0 as the passes take it; ADMM
  // starts from z = v = 0 (u = 0, Psi = 0) and keeps z_t, z_{t-1} in z[], cp[]
  float2 z[E], cp[E];
  {
    float2 v[E];
    if (a.init && !kAdmm) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = a.init[base + FR::in_index(rt, e)];
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = zero;
    }
    bool ok = true;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      ok = ok && finite2(v[e]);
      z[e] = v[e];
      cp[e] = v[e];
    }
    if (!ok) __hip_atomic_fetch_or(a.flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();   // twiddles and bin tables in place
    fft_fwd<FR>(v, rt, tw1, rA, rB, false);
    publish(v, parts + pstride);   // read at iteration 1
  }
  unsigned epoch = 1;
  if (!resident_sync<false>(a, g, epoch, &s_ok)) return;

  constexpr int W = NT / 64;   // waves per group
  static_assert(S::RPC * S::AR1 * S::FA1 >= W * 64, "the wave sums of the parts fit the exchange areas");
  const int lane = tid & 63, wv = tid >> 6;
  float2* const red = area;   // [W][64] wave sums of the parts, between the barrier and the row IFFT
  const float kappa = a.kappa;
  for (int t = 1; t <= a.iters; ++t) {
    const float beta = kFista ? a.beta[t - 1] : 0.f;
    const bool last = (t == a.iters);
    float2* const part = parts + (t & 1) * pstride;
    // Z_j: lane l of wave w adds the parts of groups w, w + W, ... at bin j0 + l in order
    // (each load of a wave reads 64 consecutive bins of one group's part), then the W
    // wave sums are added in wave order
    for (int j0 = 0; j0 < nsup; j0 += 64) {
      const int j = j0 + lane;
      const int jj = j < nsup ? j : nsup - 1;
      float2 acc = zero;
      for (int g0 = wv; g0 < G; g0 += PB * W) {
        float2 pv[PB];
#pragma unroll
        for (int k = 0; k < PB; ++k) {
          const int gg = g0 + k * W;
          pv[k] = zero;
          if (gg < G) pv[k] = load_coherent(part + static_cast<size_t>(gg) * nsup + jj);   // none past G
        }
#pragma unroll
        for (int k = 0; k < PB; ++k) acc = cadd(acc, pv[k]);
      }
      red[wv * 64 + lane] = acc;
      __syncthreads();
      if (tid < 64 && j < nsup) {
        acc = red[lane];
        for (int w2 = 1; w2 < W; ++w2) acc = cadd(acc, red[w2 * 64 + lane]);
        if constexpr (kAdmm) {
          const float2 p0 = ps[j];
          const float2 vp = make_float2(br[j].x + bq[j] * p0.x + bm[j] * acc.x, br[j].y + bq[j] * p0.y + bm[j] * acc.y);
          const float2 pn = cadd(p0, vp);
          ps[j] = pn;
          vs[j] = pn;
          if (last) vd[j] = vp;
        } else {
          vs[j] = make_float2(acc.x * bm[j] + br[j].x, acc.y * bm[j] + br[j].y);
        }
      }
      if (j0 + 64 < nsup) __syncthreads();   // red is refilled for the next 64 bins
    }
    __syncthreads();
    // the owned rows' kept spectra of IDFT2(V) at this thread's positions
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      float2 acc = zero;
      if (myslot[e] >= 0) {
        const int s2 = myslot[e];
        for (int j = sbeg[s2]; j < send[s2]; ++j) acc = cadd(acc, cmul(vs[j], cw[rr * nsup + j]));
      }
      v[e] = acc;
    }
    fft_inv<FR>(v, rt, tw1, rA, rB);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if constexpr (kAdmm) {   // v[] = IDFT2(Psi_{t+1}): z_{t+1} = S(z_t + v[])
        const float2 zo = z[e];
        const float2 zz = shrink(cadd(zo, v[e]), kappa);
        if (last) a.out_z[base + FR::in_index(rt, e)] = zz;
        // at the end cp[] keeps z_t - u_t, the spatial part of x_{t+1}
        cp[e] = last ? make_float2(2.f * zo.x - cp[e].x, 2.f * zo.y - cp[e].y) : zo;
        z[e] = zz;
        v[e] = make_float2(2.f * zz.x - zo.x, 2.f * zz.y - zo.y);   // z_{t+1} - u_{t+1}
      } else {
        const float2 u = cadd(z[e], v[e]);
        const float2 c = shrink(u, kappa);
        if (last) a.out_c[base + FR::in_index(rt, e)] = c;
        const float2 zn = kFista ? make_float2(c.x + beta * (c.x - cp[e].x), c.y + beta * (c.y - cp[e].y)) : c;
        cp[e] = c;
        z[e] = zn;
        v[e] = zn;
      }
    }
    if (last) {
      if constexpr (kAdmm) {
        if (a.out_c) {   // x_T = z_{T-1} - u_{T-1} + IDFT2(V'_T)
#pragma unroll
          for (int e = 0; e < E; ++e) {
            float2 acc = zero;
            if (myslot[e] >= 0) {
              const int s2 = myslot[e];
              for (int j = sbeg[s2]; j < send[s2]; ++j) acc = cadd(acc, cmul(vd[j], cw[rr * nsup + j]));
            }
            v[e] = acc;
          }
          fft_inv<FR>(v, rt, tw1, rA, rB, true);
#pragma unroll
          for (int e = 0; e < E; ++e) a.out_c[base + FR::in_index(rt, e)] = cadd(cp[e], v[e]);
        }
      }
      break;
    }
    fft_fwd_after_inv<FR>(v, rt, tw1, rA, rB);
    publish(v, parts + ((t + 1) & 1) * pstride);
    if (!resident_sync<false>(a, g, ++epoch, &s_ok)) return;
  }
}

template <int N1, int N2, int MODE, int NT>
int resident_launch_pt(const ResidentArgs& a, int check_only, hipStream_t s) {
  using S = ResidentPrunedShape<N1, N2, NT>;
  if (S::RPC < 1 || S::RPC > N2 || N2 % S::RPC != 0) return -1;
  const int G = N2 / S::RPC;
  if (a.groups != G || G > kResidentMaxGroups) return -1;
  if (a.ncs < 1 || a.ncs > N1 / 2 || a.nsup < 1) return -1;
  const size_t shm = S::lds_bytes(a.ncs, a.nsup, MODE == RES_PRUNED_ADMM);
  if (shm > 65536) return -1;
  const int spread = a.spread > 1 ? a.spread : 1;
  const auto kfn = k_resident_pruned<N1, N2, MODE, NT>;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, S::NT, shm) != hipSuccess) return -4;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -4;
  if (static_cast<long>(per_cu) * cus < static_cast<long>(G) * spread) return -1;
  if (check_only) return 0;
  if (!a.xy || !a.tw1 || !a.tw2 || !a.sup_ptr || !a.sup || !a.sup_rhs || !a.sync || !a.flag || !a.scol ||
      !a.colslot || a.iters < 1)
    return -1;
  if (MODE == RES_PRUNED_FISTA && !a.beta) return -1;
  if (MODE != RES_PRUNED_ADMM && (!a.coef || !a.out_c)) return -1;
  if (MODE == RES_PRUNED_ADMM && (!a.out_z || !(a.rho > 0.f))) return -1;
  void* args[] = {const_cast<ResidentArgs*>(&a)};
  const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kfn), dim3(G * spread), dim3(S::NT), args,
                                                  static_cast<unsigned>(shm), s);
  return e == hipSuccess ? 0 : -4;
}

// Groups of 256 or 512 threads, told apart by the group count the caller asks
// for (N2 L1 / 1024 or N2 L1 / 2048).
template <int N1, int N2, int MODE>
int resident_launch_p(const ResidentArgs& a, int check_only, hipStream_t s) {
  constexpr int T1 = N1 / kResidentElems;
  if (256 / T1 >= 1 && N2 % (256 / T1) == 0 && a.groups == N2 / (256 / T1))
    return resident_launch_pt<N1, N2, MODE, 256>(a, check_only, s);
  if constexpr (512 / T1 >= 1 && 512 / T1 <= N2) {
    if (N2 % (512 / T1) == 0 && a.groups == N2 / (512 / T1)) return resident_launch_pt<N1, N2, MODE, 512>(a, check_only, s);
  }
  return -1;
}

template <int N1, int N2>
int resident_launch_nn(int mode, const ResidentArgs& a, int check_only, hipStream_t s) {
  switch (mode) {
    case RES_ISTA: return resident_launch_m<N1, N2, RES_ISTA>(a, check_only, s);
    case RES_FISTA: return resident_launch_m<N1, N2, RES_FISTA>(a, check_only, s);
    case RES_ADMM: return resident_launch_m<N1, N2, RES_ADMM>(a, check_only, s);
    case RES_PRUNED_ISTA: return resident_launch_p<N1, N2, RES_PRUNED_ISTA>(a, check_only, s);
    case RES_PRUNED_FISTA: return resident_launch_p<N1, N2, RES_PRUNED_FISTA>(a, check_only, s);
    case RES_PRUNED_ADMM: return resident_launch_p<N1, N2, RES_PRUNED_ADMM>(a, check_only, s);
    default: return -1;
  }
}

}  // namespace bccb
