// Dense "regular" baseline: the explicit L x L iteration matrix.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <vector>

#include "bccb.h"
#include "kernels.h"
#include "plan_internal.h"
#include "plan_math.h"

using namespace bccb;

struct bccb_dense_s {
  bccb_plan_t plan = nullptr;
  int kind = 0;
  float rho = 0.f;
  long L = 0;
  float2* d_R = nullptr;        // [L][L]
  float2* d_x[2] = {nullptr, nullptr};
  float2* d_rhs = nullptr;
  float2* d_state = nullptr;
  float2* d_col = nullptr;
};

namespace {

void dense_free(bccb_dense_s* d) {
  if (!d) return;
  for (void* p : {static_cast<void*>(d->d_R), static_cast<void*>(d->d_x[0]), static_cast<void*>(d->d_x[1]),
                  static_cast<void*>(d->d_rhs), static_cast<void*>(d->d_state), static_cast<void*>(d->d_col)})
    if (p) (void)hipFree(p);
  delete d;
}

}  // namespace

extern "C" {

int bccb_dense_create(bccb_plan_t p, int kind, float rho, bccb_dense_t* out) {
  if (!p || !out || (kind != 0 && kind != 1)) return BCCB_E_INVALID;
  if (kind == 1 && (!(rho > 0.f) || !std::isfinite(rho))) return BCCB_E_INVALID;
  *out = nullptr;
  if (p->emb) return BCCB_E_UNSUPPORTED;
  const long L = p->L;
  if (L % 8 != 0) return BCCB_E_UNSUPPORTED;
  // first column of the iteration matrix, FP64 on the host
  const std::vector<cd> r = gram_first_column_plan(p);
  std::vector<float2> col(L);
  if (kind == 0) {
    for (long i = 0; i < L; ++i) {
      const cd v = (i == 0 ? cd(1.0, 0.0) : cd(0.0, 0.0)) - p->mu * r[i];
      col[i] = make_float2(static_cast<float>(v.real()), static_cast<float>(v.imag()));
    }
  } else {
    // (G + rho I)^-1 is the BCCB with spectrum 1/(Omega + rho) (Sec. III-A (ii));
    // its first column is IDFT2 of that spectrum
    std::vector<cd> om = eigenvalues_eq21(r, p->L1, p->L2);
    for (cd& v : om) v = 1.0 / (cd(v.real(), 0.0) + static_cast<double>(rho));
    for (int l2 = 0; l2 < p->L2; ++l2) host_dft(&om[static_cast<size_t>(l2) * p->L1], p->L1, +1);
    std::vector<cd> tmp(p->L2);
    for (int l1 = 0; l1 < p->L1; ++l1) {
      for (int l2 = 0; l2 < p->L2; ++l2) tmp[l2] = om[static_cast<size_t>(l2) * p->L1 + l1];
      host_dft(tmp.data(), p->L2, +1);
      for (int l2 = 0; l2 < p->L2; ++l2) om[static_cast<size_t>(l2) * p->L1 + l1] = tmp[l2];
    }
    for (long i = 0; i < L; ++i) {
      const cd v = om[i] / static_cast<double>(L);
      col[i] = make_float2(static_cast<float>(v.real()), static_cast<float>(v.imag()));
    }
  }
  bccb_dense_s* d = new (std::nothrow) bccb_dense_s();
  if (!d) return BCCB_E_NOMEM;
  d->plan = p;
  d->kind = kind;
  d->rho = rho;
  d->L = L;
  int rc = BCCB_OK;
  auto dal = [&](float2** ptr, size_t n) {
    if (rc == BCCB_OK && hipMalloc(reinterpret_cast<void**>(ptr), n * sizeof(float2)) != hipSuccess) {
      *ptr = nullptr;
      rc = BCCB_E_NOMEM;
    }
  };
  dal(&d->d_R, static_cast<size_t>(L) * static_cast<size_t>(L));
  dal(&d->d_x[0], L);
  dal(&d->d_x[1], L);
  dal(&d->d_rhs, L);
  dal(&d->d_state, L);
  dal(&d->d_col, L);
  if (rc == BCCB_OK && hipMemcpy(d->d_col, col.data(), L * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess)
    rc = BCCB_E_DEVICE;
  if (rc == BCCB_OK) rc = kern(launch_dense_build(d->d_col, p->L1, p->L2, d->d_R, p->stream));
  if (rc == BCCB_OK && hipStreamSynchronize(p->stream) != hipSuccess) rc = BCCB_E_DEVICE;
  if (rc != BCCB_OK) {
    (void)hipGetLastError();  // clear a failed allocation
    dense_free(d);
    return rc;
  }
  *out = d;
  return BCCB_OK;
}

int bccb_dense_destroy(bccb_dense_t d) {
  if (d) (void)hipStreamSynchronize(d->plan->stream);
  dense_free(d);
  return BCCB_OK;
}

int bccb_dense_apply(bccb_dense_t d, const bccb_c32* x, bccb_c32* y) {
  if (!d || !x || !y || static_cast<const void*>(x) == static_cast<const void*>(y)) return BCCB_E_INVALID;
  DenseArgs a;
  a.R = d->d_R;
  a.x = reinterpret_cast<const float2*>(x);
  a.out = reinterpret_cast<float2*>(y);
  a.L = d->L;
  BCCB_TRY(kern(launch_dense_gemv(0, a, d->plan->stream)));
  BCCB_HIP(hipStreamSynchronize(d->plan->stream));
  return BCCB_OK;
}

int lasso_solve_dense(bccb_dense_t d, int solver, const bccb_c32* y, float tau, int iters, bccb_c32* out) {
  if (!d || !y || !out || iters < 0 || !(tau >= 0.f) || !std::isfinite(tau)) return BCCB_E_INVALID;
  if (solver < 0 || solver > 2 || (solver == 2) != (d->kind == 1)) return BCCB_E_INVALID;
  bccb_plan_s* p = d->plan;
  hipStream_t s = p->stream;
  BCCB_TRY(begin_call(p));
  const long L = d->L;
  if (solver == 2) {
    // w = (G + rho I)^-1 b with the dense matrix itself
    BCCB_TRY(adjoint_into(p, reinterpret_cast<const float2*>(y), 1.f, d->d_x[1]));
    DenseArgs a;
    a.R = d->d_R;
    a.x = d->d_x[1];
    a.out = d->d_rhs;
    a.L = L;
    BCCB_TRY(kern(launch_dense_gemv(0, a, s)));
  } else {
    BCCB_TRY(adjoint_into(p, reinterpret_cast<const float2*>(y), static_cast<float>(p->mu), d->d_rhs));
  }
  BCCB_TRY(kern(launch_fill(d->d_state, L, s)));
  BCCB_TRY(kern(launch_fill(d->d_x[0], L, s)));
  double alpha = 1.0;
  int cur = 0;
  float2* o = reinterpret_cast<float2*>(out);
  for (int t = 1; t <= iters; ++t) {
    DenseArgs a;
    a.R = d->d_R;
    a.x = d->d_x[cur];
    a.out = d->d_x[cur ^ 1];
    a.rhs = d->d_rhs;
    a.state = d->d_state;
    a.L = L;
    if (solver == 2) {
      a.kappa = tau / d->rho;
      a.rho = d->rho;
      a.out_z = (t == iters) ? o : nullptr;
    } else {
      const double an = (1.0 + std::sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0;
      a.kappa = static_cast<float>(p->mu * tau);
      a.beta = solver == 1 ? static_cast<float>((alpha - 1.0) / an) : 0.f;
      alpha = an;
    }
    BCCB_TRY(kern(launch_dense_gemv(solver == 2 ? 2 : 1, a, s)));
    cur ^= 1;
  }
  if (iters == 0) {
    BCCB_TRY(kern(launch_fill(o, L, s)));
  } else if (solver != 2) {
    BCCB_TRY(kern(launch_copy(o, d->d_state, L, s)));
  }
  return end_call(p);
}

}  // extern "C"
