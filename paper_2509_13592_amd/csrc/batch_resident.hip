// Persistent whole-solve FISTA over the batch's support-column classes: one scene
// per workgroup at a time, taken from a queue (see batch_resident.h).
#include "batch_resident.h"
#include "passes.h"

namespace bccb {

namespace {

constexpr int kMaxThreads = 1024;

// The thread's index within its group, as a value the compiler cannot prove loop
// invariant: the transforms' LDS and twiddle addresses are then formed inside each
// row's work instead of all being hoisted out of the row loop into registers.
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Accesses through the global address space: the class table hands out plain
// pointers, and accesses through them would otherwise be flat ones (which also
// count against the LDS wait counter and hold up the row's exchanges).
struct alignas(8) P2 {
  float x, y;
};
template <class T>
__device__ __forceinline__ T ldg(const T* p, size_t i) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ((const __attribute__((address_space(1))) T*)p)[i];
#else
  return p[i];   // the host pass only parses device code
#endif
}
template <class T>
__device__ __forceinline__ void stg(T* p, size_t i, T v) {
#if defined(__HIP_DEVICE_COMPILE__)
  ((__attribute__((address_space(1))) T*)p)[i] = v;
#else
  p[i] = v;
#endif
}
__device__ __forceinline__ float2 ldg2(const float2* p, size_t i) {
  const P2 v = ldg(reinterpret_cast<const P2*>(p), i);
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void stg2(float2* p, size_t i, float2 v) {
  stg(reinterpret_cast<P2*>(p), i, P2{v.x, v.y});
}

// The complex soft threshold of passes.h (zero for |z| <= k, z (1 - k/|z|) above),
// formed without a branch: the reciprocal square root is taken for every element
// and the factor selected, so a row's lanes never split over the two cases.
__device__ __forceinline__ float sq_abs(float2 z) { return __builtin_fmaf(z.x, z.x, z.y * z.y); }
__device__ __forceinline__ float2 shrink_sel(float2 z, float k) {
  const float a2 = sq_abs(z);
  const float f = 1.f - k * __builtin_amdgcn_rsqf(a2);
  const float m = a2 > k * k ? f : 0.f;
  return make_float2(z.x * m, z.y * m);
}

// acc += a b as four fused multiply-adds (one rounding per product term)
__device__ __forceinline__ void cmac(float2& acc, float2 a, float2 b) {
  acc.x = __builtin_fmaf(a.x, b.x, acc.x);
  acc.x = __builtin_fmaf(-a.y, b.y, acc.x);
  acc.y = __builtin_fmaf(a.x, b.y, acc.y);
  acc.y = __builtin_fmaf(a.y, b.x, acc.y);
}

// dst[kq[e]] = the DFT of the row x at the bin F::out_index(t, e), for the kept bins
// (kq[e] >= 0) this thread holds; x holds the row's elements t + T e of thread t of the
// group, `tot` nonzeros in the row, `before` of them with lower threads.  Direct sums over
// the nonzeros where the row has at most N / 8 of them, the row FFT above that (x is
// overwritten).  Uses the group's exchange areas A, B.
template <class F, int N, int E>
__device__ __forceinline__ void kept_forward(float2 (&x)[E], int tot, int before, int t, const int (&kq)[E],
                                             const float2* stw, float2* sa, float2* sb, float2* dst) {
  constexpr int DIRECT = SparseRow<N>::CAP;
  const float2 zero = make_float2(0.f, 0.f);
  if (tot > DIRECT) {
    fft_fwd<F>(x, t, stw, sa, sb, true);
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (kq[e] >= 0) dst[kq[e]] = x[e];
  } else if (tot == 0) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (kq[e] >= 0) dst[kq[e]] = zero;
  } else {
    lds_sync<true>();   // the group's last use of its areas is done
    int* zpos = reinterpret_cast<int*>(sb);
    int o = before;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (x[e].x != 0.f || x[e].y != 0.f) {
        sa[o] = x[e];
        zpos[o] = F::in_index(t, e);
        ++o;
      }
    }
    lds_sync<true>();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (kq[e] >= 0) {
        const int kk = F::out_index(t, e);
        float2 acc = zero;
        for (int q = 0; q < tot; ++q) {
          const float2 w = stw[(kk * zpos[q]) & (N - 1)];   // e^{-j 2 pi k l / N}
          acc = cadd(acc, cmul(sa[q], w));
        }
        dst[kq[e]] = acc;
      }
    }
  }
}

// Every iteration of one scene's FISTA solve (eqs. (10)-(12)).  The workgroup is cut
// into groups of T = N / E threads (inside one wavefront), each owning the kept
// columns q = g, g + G, ... in the column pass and the rows r = g, g + G, ... in the
// row pass; a group's exchanges order only its wavefront.
//
// The kept columns are held in the order of their spectral column k1 modulo E = 4
// (qoff[j] .. qoff[j + 1] - 1 hold k1 = j mod 4): thread t of a row owns the elements
// l = t + T e, and the inverse row transform of a row with only the kept bins,
//   u(t + T e) = sum_q X_q w^{k1_q t} i^{k1_q e}      (w = e^{j 2 pi / N}),
// is then four sums S_j = sum over the q of class j of X_q w^{k1_q t} followed by one
// 4-point transform, with the per-thread twiddles w^{k1_q t} read from LDS.
//
// A carrying launch of a class with kkt_sum checks the KKT conditions at its last
// iterate c_t inside the same workgroup once the state is saved: c_t's kept row spectra
// (from the rows it wrote to the outputs) go to X, one more column pass turns them into
// those of mu (b - G c_t), and a row pass of class sums forms the sum of e^2 over the
// scene (the conditions of the separate KKT row kernel; each term in FP32, the sum in FP64).
template <int N, int E, bool KKT>
__device__ void solve_scene(const ResidentClass& c, int k, const float* beta, int it0, int steps, int carry,
                            float2* lds) {
  static_assert(E == 4, "the row inverse is a 4-point transform of four class sums");
  using F = Stockham<N, E, true>;
  constexpr int T = F::T;
  static_assert(T <= 64 && 64 % T == 0, "a transform inside one wavefront");
  constexpr int FA = fft_area(N);
  constexpr int CAP = N / kResidentSlotDiv;     // slots per row of the stored iterate
  constexpr int SPT = (CAP + T - 1) / T;
  const int G = static_cast<int>(blockDim.x) / T;
  const int g = static_cast<int>(threadIdx.x) / T;
  const int t0 = static_cast<int>(threadIdx.x) - g * T;
  const int ncs = c.ncs, xs = c.xs;
  float2* X = lds;                       // kept row spectra [N][xs], kept column q at q
  float2* stw = X + N * xs;              // twiddles [N]
  float2* sa = stw + N + 2 * g * FA;     // the group's exchange areas A, B
  float2* sb = sa + FA;
  float2* tw2 = stw + N + 2 * G * FA;    // [ncs][T]: w^{k1_q t}, conjugated table entries
  int* cntl = reinterpret_cast<int*>(tw2 + ncs * T);   // [3][N] nonzeros of the row of c_t (> CAP: dense)
  int* qpos = cntl + 3 * N;              // [ncs] slot -> kept-column position q (-1: padding)
  int* qk1 = qpos + ncs;                 // [ncs] q -> spectral column k1
  int* qsl = qk1 + ncs;                  // [ncs] q -> slot
  int* qoff = qsl + ncs;                 // [5] class bounds of q
  const float2 zero = make_float2(0.f, 0.f);
  const bool kkt = KKT && carry && c.kkt_sum != nullptr;   // the launch ends with the KKT check

  const float kappa = c.kmul * ldg(c.kscale, k);
  const float cb = ldg2(c.coef, static_cast<size_t>(k) * c.coef_stride).y;
  const int* scol = c.scol + static_cast<size_t>(k) * c.scol_stride;
  const int* sptr = c.sup_ptr + static_cast<size_t>(k) * c.sup_ptr_stride;
  const float2* srhs = c.sup_rhs + static_cast<size_t>(k) * c.rhs_stride;
  float2* out = c.out_base ? c.out_base + static_cast<size_t>(k) * N * N : c.desc[k].out;

  // the kept columns by class; twiddles
  for (int j = threadIdx.x; j < N; j += blockDim.x) stw[j] = c.tw[j];
  if (threadIdx.x == 0) {
    int q = 0;
    for (int j = 0; j < 4; ++j) {
      qoff[j] = q;
      for (int s = 0; s < ncs; ++s) {
        const int k1 = ldg(scol, s);
        if (j == 0) qpos[s] = -1;
        if (k1 >= 0 && (k1 & 3) == j) {
          qpos[s] = q;
          qk1[q] = k1;
          qsl[q] = s;
          ++q;
        }
      }
    }
    qoff[4] = q;
  }
  __syncthreads();
  const int nq = qoff[4];
  if (carry) {
    // z's kept spectra (slot order in memory) and the iterates' row counts of the last launch
    for (int j = threadIdx.x; j < N * nq; j += blockDim.x) {
      const int r = j / nq, q = j - (j / nq) * nq;
      X[r * xs + q] = ldg2(c.xkeep, (static_cast<size_t>(k) * N + r) * ncs + qsl[q]);
    }
    for (int j = threadIdx.x; j < 3 * N; j += blockDim.x)
      cntl[j] = ldg(c.buf[j / N].cnt, static_cast<size_t>(k) * N + (j - (j / N) * N));
  } else {
    // z_1 = 0: zero kept spectra; c_0 = c_{-1} = 0: empty rows
    for (int j = threadIdx.x; j < N * xs; j += blockDim.x) X[j] = zero;
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
      cntl[j] = 0;
      cntl[2 * N + j] = 0;
    }
  }
  for (int j = threadIdx.x; j < nq * T; j += blockDim.x) {
    const float2 w = stw[(qk1[j / T] * (j % T)) & (N - 1)];
    tw2[j] = make_float2(w.x, -w.y);   // e^{+j 2 pi k1 t / N}
  }
  int kq[E];   // kept-column position of each spectral bin this thread holds after a forward row transform
  {
    const int* cs = c.colslot + static_cast<size_t>(k) * c.colslot_stride;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int sl = ldg(cs, F::out_index(t0, e));
      kq[e] = sl >= 0 ? qpos[sl] : -1;
    }
  }
  const int o1 = qoff[1], o2 = qoff[2], o3 = qoff[3];
  __syncthreads();

  // column pass over the kept columns: X[:, q] = IDFT_cols(m . DFT_cols(X[:, q]) + r),
  // m = b Omega_j and r = rhs_j on the column's support bins, m = r = 0 elsewhere
  auto column_pass = [&]() __attribute__((always_inline)) {
    for (int q = g; q < nq; q += G) {
      const int k1 = qk1[q];
      const int t = opaque(t0);
      float2 v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = X[F::in_index(t, e) * xs + q];
      fft_fwd<F>(v, t, stw, sa, sb, true);
      float2 src[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        src[e] = v[e];
        v[e] = zero;
      }
      const int j0 = ldg(sptr, k1), j1 = ldg(sptr, k1 + 1);
      for (int j = j0; j < j1; ++j) {
        const SupEntry en = ldg(c.sup, j);
        const float2 r = ldg2(srhs, j);
        const float m = cb * en.omega;
#pragma unroll
        for (int e = 0; e < E; ++e)
          if (F::out_index(t, e) == en.k2) v[e] = make_float2(src[e].x * m + r.x, src[e].y * m + r.y);
      }
      fft_inv_after_fwd<F>(v, t, stw, sa, sb);
#pragma unroll
      for (int e = 0; e < E; ++e) X[F::in_index(t, e) * xs + q] = v[e];
    }
  };
  // u = IDFT_rows(X) of the row xr at this thread's elements t + T e
  auto row_inverse = [&](const float2* xr, int t, float2 (&v)[E]) __attribute__((always_inline)) {
    const float2* wt = tw2 + t;
    float2 S[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) S[j] = zero;
#pragma unroll 4
    for (int q = 0; q < o1; ++q) cmac(S[0], xr[q], wt[q * T]);
#pragma unroll 4
    for (int q = o1; q < o2; ++q) cmac(S[1], xr[q], wt[q * T]);
#pragma unroll 4
    for (int q = o2; q < o3; ++q) cmac(S[2], xr[q], wt[q * T]);
#pragma unroll 4
    for (int q = o3; q < nq; ++q) cmac(S[3], xr[q], wt[q * T]);
    const float2 a = cadd(S[0], S[2]), b = make_float2(S[0].x - S[2].x, S[0].y - S[2].y);
    const float2 cc = cadd(S[1], S[3]), d = make_float2(S[1].x - S[3].x, S[1].y - S[3].y);
    v[0] = cadd(a, cc);                              // i^0
    v[1] = make_float2(b.x - d.y, b.y + d.x);        // S0 + i S1 - S2 - i S3
    v[2] = make_float2(a.x - cc.x, a.y - cc.y);      // S0 - S1 + S2 - S3
    v[3] = make_float2(b.x + d.y, b.y - d.x);        // S0 - i S1 - S2 + i S3
  };

  for (int it = it0 + 1; it <= it0 + steps; ++it) {
    column_pass();
    __syncthreads();

    // row pass: z_t = c_{t-1} + beta_{t-1} (c_{t-1} - c_{t-2}); c_t = S_kappa(z_t + IDFT_rows(X));
    // X = DFT_rows(c_t + beta_t (c_t - c_{t-1})) on the kept columns
    const int i0 = it % 3, i1 = (it - 1) % 3, i2 = (it + 1) % 3;
    const float bt = beta[it], bp = beta[it - 1];
    const bool fin = it == it0 + steps;   // the launch's last iteration: c_t goes to the outputs
    const bool last = fin && !carry;      // ... and nothing after it is needed
    const SlotBuf b0 = c.buf[i0], b1 = c.buf[i1], b2 = c.buf[i2];
    for (int r = g; r < N; r += G) {
      const int t = opaque(t0);
      const size_t prow = static_cast<size_t>(k) * N + r;
      const size_t base = prow * N;
      float2* xr = X + r * xs;
      const int n1 = cntl[i1 * N + r], n2 = cntl[i2 * N + r];
      // u = IDFT_rows(X) at this thread's elements t + T e
      float2 v[E];
      row_inverse(xr, t, v);
      float2 p1[E];
      bool cold = false;   // c_t and z_{t+1} vanish on the row
      if (n1 == 0 && n2 == 0) {
        // z_t = 0 on the row: c_t = S_kappa(u).  Where no element of the rows of this
        // wavefront in this branch exceeds the threshold, the rows stay empty and the
        // threshold, counts and forward sums are skipped
        bool hot = false;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          p1[e] = zero;
          hot = hot || sq_abs(v[e]) > kappa * kappa;   // the threshold's own test
        }
        cold = !__any(hot);
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = cold ? zero : shrink_sel(v[e], kappa);
      } else {
        // dense rows straight into registers; slot rows scattered into zeroed areas
        const bool full1 = n1 > CAP, full2 = n2 > CAP;
        float2 p2[E];
        unsigned short q1[SPT], q2[SPT];
        float2 w1[SPT], w2[SPT];
        if (full1) {
#pragma unroll
          for (int e = 0; e < E; ++e) p1[e] = ldg2(b1.dense, base + F::in_index(t, e));
        }
        if (full2) {
#pragma unroll
          for (int e = 0; e < E; ++e) p2[e] = ldg2(b2.dense, base + F::in_index(t, e));
        }
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
          const int j = t + T * q;
          q1[q] = q2[q] = 0;
          w1[q] = w2[q] = zero;
          if (!full1 && j < n1) {
            q1[q] = ldg(b1.sidx, prow * CAP + j);
            w1[q] = ldg2(b1.sval, prow * CAP + j);
          }
          if (!full2 && j < n2) {
            q2[q] = ldg(b2.sidx, prow * CAP + j);
            w2[q] = ldg2(b2.sval, prow * CAP + j);
          }
        }
        lds_sync<true>();   // the group's last use of its areas is done
        if (!full1) {
#pragma unroll
          for (int e = 0; e < E; ++e) sb[F::in_index(t, e)] = zero;
        }
        if (!full2) {
#pragma unroll
          for (int e = 0; e < E; ++e) sa[F::in_index(t, e)] = zero;
        }
        lds_sync<true>();
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
          const int j = t + T * q;
          if (!full1 && j < n1) sb[q1[q] < N ? q1[q] : N - 1] = w1[q];
          if (!full2 && j < n2) sa[q2[q] < N ? q2[q] : N - 1] = w2[q];
        }
        lds_sync<true>();
        if (!full1) {
#pragma unroll
          for (int e = 0; e < E; ++e) p1[e] = sb[F::in_index(t, e)];
        }
        if (!full2) {
#pragma unroll
          for (int e = 0; e < E; ++e) p2[e] = sa[F::in_index(t, e)];
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const float2 z = make_float2(p1[e].x + bp * (p1[e].x - p2[e].x), p1[e].y + bp * (p1[e].y - p2[e].y));
          v[e] = shrink_sel(cadd(z, v[e]), kappa);
        }
      }

      if (fin) {
#pragma unroll
        for (int e = 0; e < E; ++e) stg2(out, static_cast<size_t>(r) * N + F::in_index(t, e), v[e]);
        if (last) continue;   // uniform over the workgroup
      }
      if (cold) {
        if (t == 0) cntl[i0 * N + r] = 0;
#pragma unroll
        for (int e = 0; e < E; ++e)
          if (kq[e] >= 0) xr[kq[e]] = zero;
        continue;
      }
      // z_{t+1} = c_t + beta_t (c_t - c_{t-1}); one scan counts the nonzeros of both rows
      // (with c_{t-1} = 0 on the row, z_{t+1} = c_t + beta_t c_t has the same nonzeros)
      float2 zn[E];
      int mine = 0;
      if (n1 == 0) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          zn[e] = make_float2(__builtin_fmaf(bt, v[e].x, v[e].x), __builtin_fmaf(bt, v[e].y, v[e].y));
          mine += (v[e].x != 0.f || v[e].y != 0.f) ? (1 << 16) + 1 : 0;
        }
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          zn[e] = make_float2(v[e].x + bt * (v[e].x - p1[e].x), v[e].y + bt * (v[e].y - p1[e].y));
          mine += (v[e].x != 0.f || v[e].y != 0.f) ? 1 : 0;
          mine += (zn[e].x != 0.f || zn[e].y != 0.f) ? (1 << 16) : 0;
        }
      }
      int tot2, before2;
      row_prefix<T>(mine, t, nullptr, tot2, before2);
      const int total = tot2 & 0xffff, before = before2 & 0xffff;
      const int ztot = tot2 >> 16, zbefore = before2 >> 16;
      if (t == 0) cntl[i0 * N + r] = total;
      // c_t: slots while the row has at most CAP nonzeros, the dense row otherwise
      if (total > CAP) {
#pragma unroll
        for (int e = 0; e < E; ++e) stg2(b0.dense, base + F::in_index(t, e), v[e]);
      } else if (total > 0) {
        int o = before;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          if (v[e].x != 0.f || v[e].y != 0.f) {
            stg(b0.sidx, prow * CAP + o, static_cast<unsigned short>(F::in_index(t, e)));
            stg2(b0.sval, prow * CAP + o, v[e]);
            ++o;
          }
        }
      }
      // X = DFT_rows(z_{t+1}) on the kept columns: direct sums over its nonzeros when it has
      // at most N/8 of them (none for most rows once the iterate is sparse), else the row FFT
      kept_forward<F, N, E>(zn, ztot, zbefore, t, kq, stw, sa, sb, xr);
    }
    __syncthreads();
  }
  if (carry) {
    // the next launch continues from z's kept spectra and the row counts
    for (int j = threadIdx.x; j < N * nq; j += blockDim.x) {
      const int r = j / nq, q = j - (j / nq) * nq;
      stg2(c.xkeep, (static_cast<size_t>(k) * N + r) * ncs + qsl[q], X[r * xs + q]);
    }
    for (int j = threadIdx.x; j < 3 * N; j += blockDim.x)
      stg(c.buf[j / N].cnt, static_cast<size_t>(k) * N + (j - (j / N) * N), cntl[j]);
  }
  if (kkt) {
    // X = kept spectra of c_t, read back from the outputs (rows with nonzeros only) ...
    const int* nc = cntl + ((it0 + steps) % 3) * N;   // the row counts of c_t
    __syncthreads();   // the state is saved: X is free
    for (int r = g; r < N; r += G) {
      const int t = opaque(t0);
      float2 x[E];
      int mine = 0;
#pragma unroll
      for (int e = 0; e < E; ++e) x[e] = zero;
      if (nc[r] > 0) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          x[e] = ldg2(out, static_cast<size_t>(r) * N + F::in_index(t, e));
          mine += (x[e].x != 0.f || x[e].y != 0.f) ? 1 : 0;
        }
      }
      int tot, before;
      row_prefix<T>(mine, t, nullptr, tot, before);
      kept_forward<F, N, E>(x, tot, before, t, kq, stw, sa, sb, X + r * xs);
    }
    __syncthreads();
    // ... -> kept spectra of mu (b - G c_t); then per element g = b - G c_t and e^2,
    // summed over the scene
    column_pass();
    __syncthreads();
    // per element in FP32 (g itself comes from FP32 sums, with errors of the order of those
    // of these few operations), summed in FP64
    const float tau = ldg(c.kscale, k), sc = c.kkt_scale;
    double acc = 0.0;
    for (int r = g; r < N; r += G) {
      const int t = opaque(t0);
      float2 v[E];
      row_inverse(X + r * xs, t, v);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        // c_t as this thread stored it to the outputs in the last row pass
        const float2 cv = nc[r] > 0 ? ldg2(out, static_cast<size_t>(r) * N + F::in_index(t, e)) : zero;
        const float gr = sc * v[e].x, gi = sc * v[e].y;
        const float a2 = sq_abs(cv);
        // c != 0: e = g - tau c / |c|; c = 0: |e| = max(|g| - tau, 0); both formed, one kept
        const float rc = a2 > 0.f ? __builtin_amdgcn_rsqf(a2) : 0.f;
        const float er = gr - tau * cv.x * rc, ei = gi - tau * cv.y * rc;
        const float dd = __builtin_fmaxf(__builtin_sqrtf(__builtin_fmaf(gr, gr, gi * gi)) - tau, 0.f);
        const float e2 = a2 > 0.f ? __builtin_fmaf(er, er, ei * ei) : dd * dd;
        acc += static_cast<double>(e2);
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __syncthreads();   // every row is done with X
    double* red = reinterpret_cast<double*>(X);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sum = 0.0;
      for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) sum += red[w];
      stg(c.kkt_sum, static_cast<size_t>(k), sum);
    }
  }
  if (carry) __syncthreads();   // LDS is reused by the next scene
}

template <bool KKT>
__global__ __launch_bounds__(kMaxThreads) void k_scene_fista(const ResidentClass* cls, int ncls, int total,
                                                             const float* beta, int it0, int steps, int carry,
                                                             int* queue) {
  extern __shared__ float2 lds[];
  __shared__ int item;
  for (;;) {
    if (threadIdx.x == 0) item = atomicAdd(queue, 1);
    __syncthreads();
    const int q = __builtin_amdgcn_readfirstlane(item);   // uniform: the class table is read with scalar loads
    __syncthreads();   // every thread has read the item before thread 0 takes the next
    if (q >= total) return;   // uniform: every wave leaves together, the queue only grows
    int ci = 0;
    while (ci + 1 < ncls && q >= cls[ci + 1].first) ++ci;
    const ResidentClass& c = cls[ci];
    const int k = c.scene_map ? c.scene_map[q - c.first] : q - c.first;
    switch (c.N) {
      case 32: solve_scene<32, kResidentE, KKT>(c, k, beta, it0, steps, carry, lds); break;
      case 64: solve_scene<64, kResidentE, KKT>(c, k, beta, it0, steps, carry, lds); break;
      case 128: solve_scene<128, kResidentE, KKT>(c, k, beta, it0, steps, carry, lds); break;
      case 256: solve_scene<256, kResidentE, KKT>(c, k, beta, it0, steps, carry, lds); break;
      default: break;
    }
  }
}

}  // namespace

int launch_scene_fista(const ResidentClass* cls, int ncls, int total, const float* beta, int it0, int steps,
                       int carry, int check, int* queue, int nthreads, int blocks, size_t lds, hipStream_t s) {
  if (!cls || ncls < 1 || total < 1 || !beta || it0 < 0 || steps < 1 || (carry != 0 && carry != 1) || !queue)
    return -1;
  if ((check != 0 && check != 1) || (check && !carry)) return -1;
  if (nthreads < 64 || nthreads > kMaxThreads || nthreads % 64 != 0 || blocks < 1) return -1;
  const void* fn = check ? reinterpret_cast<const void*>(k_scene_fista<true>)
                         : reinterpret_cast<const void*>(k_scene_fista<false>);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
    return -2;
  if (check)
    hipLaunchKernelGGL(k_scene_fista<true>, dim3(blocks), dim3(nthreads), lds, s, cls, ncls, total, beta, it0, steps,
                       carry, queue);
  else
    hipLaunchKernelGGL(k_scene_fista<false>, dim3(blocks), dim3(nthreads), lds, s, cls, ncls, total, beta, it0,
                       steps, carry, queue);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int scene_fista_occupancy(int nthreads, size_t lds, int check) {
  int nb = 0;
  const void* fn = check ? reinterpret_cast<const void*>(k_scene_fista<true>)
                         : reinterpret_cast<const void*>(k_scene_fista<false>);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
    return 0;
  hipError_t rc;
  if (check) rc = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_scene_fista<true>, nthreads, lds);
  else rc = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_scene_fista<false>, nthreads, lds);
  return rc == hipSuccess ? nb : 0;
}

}  // namespace bccb
