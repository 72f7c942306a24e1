// FP64 entry points: D_s^H y, the eq. (23) product and ISTA / FISTA / ADMM in complex128
// through the FP64 passes (passes_f64.hip), for results at the level of the paper's FP64
// comparison (Table I).  The plan's FP64 buffers (eigenvalues from eq. (21) in FP64, twiddles,
// three work grids: 56 bytes per grid point) are allocated on the first FP64 call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "passes_f64.h"
#include "plan_internal.h"

namespace bccb {

namespace {

template <typename T>
int dalloc64(T** p, size_t n) {
  *p = nullptr;
  return hipMalloc(reinterpret_cast<void**>(p), (n ? n : 1) * sizeof(T)) == hipSuccess ? BCCB_OK : BCCB_E_NOMEM;
}

int k64(int rc) { return rc == 0 ? BCCB_OK : (rc == -1 ? BCCB_E_UNSUPPORTED : BCCB_E_DEVICE); }

// FP64 state of a plan (first call): Omega by eq. (21) in FP64 with the bins no element folds
// onto (FP64 rounding of ~1e-12 of the maximum) set to exact zeros, as the FP32 grid is built
int ensure_f64(bccb_plan_s* p) {
  if (p->d_omega64) return BCCB_OK;
  if (p->emb) return BCCB_E_UNSUPPORTED;
  const std::vector<cd> om = eigenvalues_eq21(gram_first_column_plan(p), p->L1, p->L2);
  double omax = 0.0;
  for (const cd& v : om) omax = std::max(omax, v.real());
  std::vector<double> om64(p->L);
  for (long i = 0; i < p->L; ++i) om64[i] = std::fabs(om[i].real()) > 1e-9 * omax ? om[i].real() : 0.0;
  std::vector<double2> t1(p->L1), t2(p->L2);
  const std::vector<cd> w1 = unit_roots(p->L1), w2 = unit_roots(p->L2);
  for (int j = 0; j < p->L1; ++j) t1[j] = make_double2(w1[j].real(), w1[j].imag());
  for (int j = 0; j < p->L2; ++j) t2[j] = make_double2(w2[j].real(), w2[j].imag());
  int rc = dalloc64(&p->d_omega64, p->L);
  if (rc == BCCB_OK) rc = dalloc64(&p->d_tw1_64, p->L1);
  if (rc == BCCB_OK) rc = dalloc64(&p->d_tw2_64, p->L2);
  if (rc == BCCB_OK) rc = dalloc64(&p->d_xy64, p->L);
  if (rc == BCCB_OK) rc = dalloc64(&p->d_rhs64, p->L);
  if (rc == BCCB_OK) rc = dalloc64(&p->d_state64, p->L);
  if (rc == BCCB_OK &&
      (hipMemcpy(p->d_omega64, om64.data(), p->L * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(p->d_tw1_64, t1.data(), p->L1 * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(p->d_tw2_64, t2.data(), p->L2 * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess))
    rc = BCCB_E_DEVICE;
  if (rc != BCCB_OK) {
    for (void* q : {static_cast<void*>(p->d_omega64), static_cast<void*>(p->d_tw1_64), static_cast<void*>(p->d_tw2_64),
                    static_cast<void*>(p->d_xy64), static_cast<void*>(p->d_rhs64), static_cast<void*>(p->d_state64)})
      if (q) (void)hipFree(q);
    p->d_omega64 = nullptr;
    p->d_tw1_64 = p->d_tw2_64 = p->d_xy64 = p->d_rhs64 = p->d_state64 = nullptr;
  }
  return rc;
}

int row64(bccb_plan_s* p, RowArgs64 a) {
  a.tw = p->d_tw1_64;
  a.nrows = p->L2;
  a.rows_per_scene = p->L2;
  return k64(launch_row64(p->L1, a, p->stream));
}

int col64(bccb_plan_s* p, int mode, double2* xy, double ca, double cb, double scale, double rho) {
  ColArgs64 a;
  a.mode = mode;
  a.xy = xy;
  a.omega = p->d_omega64;
  a.tw = p->d_tw2_64;
  a.L1 = p->L1;
  a.ca = ca;
  a.cb = cb;
  a.scale = scale;
  a.rho = rho;
  return k64(launch_col64(p->L2, a, p->stream));
}

// dst = scale * D_s^H y: the snapshot scattered onto the spectral grid with (-1)^(m1+m2),
// then the unnormalised inverse 2D DFT (as the FP32 adjoint)
int adjoint64(bccb_plan_s* p, const double2* y, double scale, double2* dst) {
  BCCB_TRY(k64(launch_scatter64(y, p->d_sensor_of, p->M1, p->M2, p->L1, p->L2, scale, p->d_xy64, p->d_flag,
                                p->stream)));
  BCCB_TRY(col64(p, COL64_INV, p->d_xy64, 0.0, 0.0, 1.0, 0.0));
  RowArgs64 a;
  a.mode = ROW64_INV;
  a.xy = p->d_xy64;
  a.dst = dst;
  a.scale = 1.0;
  return row64(p, a);
}

int check64(bccb_plan_s* p, const void* y, const void* out, double tau, int iters) {
  if (!p || !y || !out) return BCCB_E_INVALID;
  if (!(tau >= 0.0) || !std::isfinite(tau) || iters < 0) return BCCB_E_INVALID;
  return ensure_f64(p);
}

int prox_grad64(bccb_plan_s* p, int mode, const double2* y, double tau, int iters, const double2* c0, double2* out) {
  BCCB_TRY(check64(p, y, out, tau, iters));
  BCCB_TRY(begin_call(p));
  BCCB_TRY(adjoint64(p, y, p->mu, p->d_rhs64));
  // z^(1) = c^(0); the output holds c^(t-1) between passes
  RowArgs64 f;
  f.mode = ROW64_FWD;
  f.xy = p->d_xy64;
  f.src = c0;
  f.flag = p->d_flag;
  BCCB_TRY(row64(p, f));
  if (c0 && c0 != out) BCCB_TRY(k64(launch_copy64(out, c0, p->L, p->stream)));
  else if (!c0) BCCB_TRY(k64(launch_fill64(out, p->L, p->stream)));
  const double invL = 1.0 / static_cast<double>(p->L);
  double alpha = 1.0;
  for (int t = 1; t <= iters; ++t) {
    BCCB_TRY(col64(p, COL64_AFFINE, p->d_xy64, invL, -p->mu * invL, 1.0, 0.0));   // (1 - mu Omega) / L
    const double alpha_next = (1.0 + std::sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0;
    RowArgs64 a;
    a.mode = mode;
    a.xy = p->d_xy64;
    a.rhs = p->d_rhs64;
    a.state = out;
    a.out_c = out;
    a.kappa = p->mu * tau;
    a.beta = (alpha - 1.0) / alpha_next;
    a.last = (t == iters);
    alpha = alpha_next;
    BCCB_TRY(row64(p, a));
  }
  return end_call(p);
}

}  // namespace

}  // namespace bccb

using namespace bccb;

extern "C" {

int bccb_adjoint_f64(bccb_plan_t p, const bccb_c64* y, bccb_c64* b) {
  BCCB_TRY(check64(p, y, b, 0.0, 0));
  BCCB_TRY(begin_call(p));
  BCCB_TRY(adjoint64(p, reinterpret_cast<const double2*>(y), 1.0, reinterpret_cast<double2*>(b)));
  return end_call(p);
}

int bccb_gram_apply_f64(bccb_plan_t p, const bccb_c64* x, bccb_c64* gx) {
  BCCB_TRY(check64(p, x, gx, 0.0, 0));
  BCCB_TRY(begin_call(p));
  RowArgs64 f;
  f.mode = ROW64_FWD;
  f.xy = p->d_xy64;
  f.src = reinterpret_cast<const double2*>(x);
  f.flag = p->d_flag;
  BCCB_TRY(row64(p, f));
  BCCB_TRY(col64(p, COL64_AFFINE, p->d_xy64, 0.0, 1.0 / static_cast<double>(p->L), 1.0, 0.0));   // Omega / L
  RowArgs64 b;
  b.mode = ROW64_INV;
  b.xy = p->d_xy64;
  b.dst = reinterpret_cast<double2*>(gx);
  BCCB_TRY(row64(p, b));
  return end_call(p);
}

int lasso_solve_ista_f64(bccb_plan_t p, const bccb_c64* y, double tau, int iters, const bccb_c64* c0, bccb_c64* c_out) {
  return prox_grad64(p, ROW64_ISTA, reinterpret_cast<const double2*>(y), tau, iters,
                     reinterpret_cast<const double2*>(c0), reinterpret_cast<double2*>(c_out));
}

int lasso_solve_fista_f64(bccb_plan_t p, const bccb_c64* y, double tau, int iters, const bccb_c64* c0,
                          bccb_c64* c_out) {
  return prox_grad64(p, ROW64_FISTA, reinterpret_cast<const double2*>(y), tau, iters,
                     reinterpret_cast<const double2*>(c0), reinterpret_cast<double2*>(c_out));
}

int lasso_solve_admm_f64(bccb_plan_t p, const bccb_c64* y, double tau, double rho, int iters, bccb_c64* z_out,
                         bccb_c64* c_out) {
  BCCB_TRY(check64(p, y, z_out, tau, iters));
  if (!(rho > 0.0) || !std::isfinite(rho)) return BCCB_E_INVALID;
  BCCB_TRY(begin_call(p));
  double2* zo = reinterpret_cast<double2*>(z_out);
  double2* co = reinterpret_cast<double2*>(c_out);
  // w = (G + rho I)^-1 D_s^H y = IDFT2(S / (Omega + rho)), unnormalised (DFT2(b) = L S)
  BCCB_TRY(k64(launch_scatter64(reinterpret_cast<const double2*>(y), p->d_sensor_of, p->M1, p->M2, p->L1, p->L2, 1.0,
                                p->d_xy64, p->d_flag, p->stream)));
  {
    // S is spectral already: divide by Omega + rho in place, then the inverse transforms
    ColArgs64 a;
    a.mode = COL64_INV;
    a.xy = p->d_xy64;
    a.omega = p->d_omega64;
    a.tw = p->d_tw2_64;
    a.L1 = p->L1;
    BCCB_TRY(k64(launch_spectral_div64(p->d_xy64, p->d_omega64, rho, p->L, p->stream)));
    BCCB_TRY(k64(launch_col64(p->L2, a, p->stream)));
    RowArgs64 r;
    r.mode = ROW64_INV;
    r.xy = p->d_xy64;
    r.dst = p->d_rhs64;
    BCCB_TRY(row64(p, r));
  }
  BCCB_TRY(k64(launch_fill64(p->d_state64, p->L, p->stream)));   // v^(0) = 0
  BCCB_TRY(k64(launch_fill64(p->d_xy64, p->L, p->stream)));      // DFT_rows(z^(0) - v^(0)) = 0
  if (iters == 0) {
    BCCB_TRY(k64(launch_fill64(zo, p->L, p->stream)));
    if (co) BCCB_TRY(k64(launch_fill64(co, p->L, p->stream)));
  }
  const double scale = rho / static_cast<double>(p->L);
  for (int t = 1; t <= iters; ++t) {
    BCCB_TRY(col64(p, COL64_ADMM, p->d_xy64, 0.0, 0.0, scale, rho));   // rho (G + rho I)^-1 (z - v)
    RowArgs64 a;
    a.mode = ROW64_ADMM;
    a.xy = p->d_xy64;
    a.rhs = p->d_rhs64;
    a.state = p->d_state64;
    a.out_z = zo;
    a.out_c = co;
    a.kappa = tau / rho;
    a.last = (t == iters);
    BCCB_TRY(row64(p, a));
  }
  return end_call(p);
}

}  // extern "C"
