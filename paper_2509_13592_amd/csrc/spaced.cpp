// Plans on a zero-padded circulant embedding: uniform harmonic grids at a general element
// spacing gamma_i (the Toeplitz Gram of Sec. III-A, eq. (16)) and grid lengths that are not
// powers of two.
//
// The Gram of such a grid is block Toeplitz with Toeplitz blocks (embed_math.h); placed in
// the leading A1 x A2 window of a P1 x P2 grid (P_i powers of two >= 2 A_i - 1) it is the
// window of a BCCB, so every product G x is the P1 x P2 product IDFT2(Omega_e . DFT2(x_pad))
// of eq. (23) cropped to the window.  ISTA and FISTA run the plan's ordinary row and column
// passes on the padded grid with Omega_e as the spectrum and the row pass holding every
// element outside the window at zero, which makes each padded iteration exactly the
// iteration on the window (the padded iterate is zero outside it, and the crop of
// (I - mu C_e) x_pad is (I - mu G) x).  ADMM needs (G + rho I)^-1 as a product: at
// gamma = 1/2 it is the BCCB with spectrum 1/(Omega + rho) (Sec. III-A (ii)), whose first
// column is again embedded; for gamma != 1/2 the inverse of a Toeplitz matrix is not Toeplitz
// and ADMM is not offered.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "embed_math.h"
#include "plan_internal.h"
#include "spaced_api.h"
#include "spaced_kernels.h"

namespace bccb {

namespace {

template <typename T>
int dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T)) == hipSuccess ? BCCB_OK : BCCB_E_NOMEM;
}

template <typename T>
int upload(T* d, const T* h, size_t n) {
  return hipMemcpy(d, h, n * sizeof(T), hipMemcpyHostToDevice) == hipSuccess ? BCCB_OK : BCCB_E_DEVICE;
}

std::vector<float2> to_c64(const std::vector<cdx>& v) {
  std::vector<float2> out(v.size());
  for (size_t i = 0; i < v.size(); ++i)
    out[i] = make_float2(static_cast<float>(v[i].real()), static_cast<float>(v[i].imag()));
  return out;
}

bool pow2(int L) { return L > 0 && (L & (L - 1)) == 0; }

// Row pass arguments over the padded grid with the coefficient window set.
RowArgs window_args(const bccb_plan_s* p) {
  RowArgs a;
  a.act_cols = p->A1;
  a.act_rows = p->A2;
  return a;
}

// b = scale * D_s^H y into the padded grid (zero outside the window) or the caller's grid.
int adjoint_to(bccb_plan_s* p, const float2* y, float scale, float2* out, bool padded) {
  const int cols = padded ? p->L1 : p->A1, rows = padded ? p->L2 : p->A2;
  return kern(launch_sep_adjoint(y, p->d_sensor_of, p->d_W1, p->d_W2, p->M1, p->M2, p->A1, p->A2, scale,
                                 p->d_emb_u, cols, rows, cols, out, p->d_flag, p->stream));
}

// The column pass over the padded grid with an explicit spectrum (the Gram's or the ADMM one).
int col_pass_spectrum(bccb_plan_s* p, int mode, float2* xy, const float* omega, const float2* coef, hipStream_t s) {
  ColArgs a;
  a.xy = xy;
  a.omega = omega;
  a.coef = coef;
  a.tw = p->d_tw2;
  a.L1 = p->L1;
  a.nscenes = 1;
  a.scale = 1.f;
  return kern(launch_col(p->L2, p->cfg_col, mode, a, s));
}

// Eigenvalues of the embedding of (G + rho I)^-1 (circulant plans), built once per rho.
int ensure_rho(bccb_plan_s* p, float rho) {
  if (p->emb_rho == rho) return BCCB_OK;
  const std::vector<double> om =
      shifted_inverse_embedding_spectrum(p->emb_omega, p->A1, p->A2, static_cast<double>(rho), p->L1, p->L2);
  std::vector<float> om32(om.size());
  for (size_t i = 0; i < om.size(); ++i) om32[i] = static_cast<float>(om[i]);
  BCCB_HIP(hipStreamSynchronize(p->stream));
  BCCB_TRY(upload(p->d_omega_rho, om32.data(), om32.size()));
  p->emb_rho = rho;
  drop_graph(p);   // a captured ADMM loop read the previous spectrum's coefficients
  return BCCB_OK;
}

}  // namespace

int spaced_adjoint(bccb_plan_s* p, const float2* y, float2* b) {
  BCCB_TRY(begin_call(p));
  BCCB_TRY(adjoint_to(p, y, 1.f, b, false));
  return end_call(p);
}

int spaced_adjoint_maxabs(bccb_plan_s* p, const float2* y, double* maxabs) {
  BCCB_TRY(begin_call(p));
  BCCB_TRY(adjoint_to(p, y, 1.f, p->d_rhs, false));
  int nb = 0;
  BCCB_TRY(kern(launch_absmax(p->d_rhs, p->AL, p->d_red, &nb, p->stream)));
  BCCB_HIP(hipMemcpyAsync(p->h_red, p->d_red, nb * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  const int rc = end_call(p);
  double m = 0.0;
  for (int i = 0; i < nb; ++i) m = p->h_red[i] > m ? p->h_red[i] : m;
  *maxabs = m;
  return rc;
}

// G x: pad, row DFT, column pass with Omega_e / L, row IDFT, crop.
static int gram_into(bccb_plan_s* p, const float2* x, float2* gx_user) {
  BCCB_TRY(kern(launch_pad(x, p->A1, p->A2, p->L1, p->L2, p->d_emb_c, p->stream)));
  RowArgs f;
  f.xy = p->d_xy;
  f.src = p->d_emb_c;
  f.flag = p->d_flag;
  BCCB_TRY(row_pass(p, ROW_FWD, f));
  BCCB_TRY(col_pass_spectrum(p, COL_FILTER_AFFINE, p->d_xy, p->d_omega, p->d_coef + 1, p->stream));
  RowArgs b;
  b.xy = p->d_xy;
  b.dst = p->d_state;
  BCCB_TRY(row_pass(p, ROW_INV, b));
  return kern(launch_crop(p->d_state, p->A1, p->A2, p->L1, gx_user, p->stream));
}

int spaced_gram_apply(bccb_plan_s* p, const float2* x, float2* gx) {
  BCCB_TRY(begin_call(p));
  BCCB_TRY(gram_into(p, x, gx));
  return end_call(p);
}

int spaced_prox_grad(bccb_plan_s* p, int mode, const float2* y, float tau, int iters, const float2* c0, float2* out) {
  BCCB_TRY(begin_call(p));
  // mu D_s^H y on the padded grid; c^(0) padded into the state buffer; its row DFT starts
  // the first column pass (z^(1) = c^(0))
  BCCB_TRY(adjoint_to(p, y, static_cast<float>(p->mu), p->d_rhs, true));
  BCCB_TRY(kern(launch_pad(c0, p->A1, p->A2, p->L1, p->L2, p->d_emb_c, p->stream)));
  RowArgs f;
  f.xy = p->d_xy;
  f.src = p->d_emb_c;
  f.flag = p->d_flag;
  BCCB_TRY(row_pass(p, ROW_FWD, f));
  const float kappa = static_cast<float>(p->mu * tau);
  if (iters > 0) {
    const unsigned long long key[8] = {static_cast<unsigned long long>(mode), static_cast<unsigned long long>(iters),
                                       reinterpret_cast<unsigned long long>(p->d_emb_c), fbits(kappa), 0, 0, 5, 1};
    BCCB_TRY(run_loop(p, key, [&](hipStream_t s) -> int {
      double alpha = 1.0;
      for (int t = 1; t <= iters; ++t) {
        BCCB_TRY(col_pass_spectrum(p, COL_FILTER_AFFINE, p->d_xy, p->d_omega, p->d_coef, s));
        const double alpha_next = (1.0 + std::sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0;
        RowArgs a = window_args(p);
        a.xy = p->d_xy;
        a.rhs = p->d_rhs;
        a.state = p->d_emb_c;
        a.out_c = p->d_emb_c;
        a.kappa = kappa;
        a.beta = static_cast<float>((alpha - 1.0) / alpha_next);
        a.last = (t == iters);
        alpha = alpha_next;
        BCCB_TRY(row_pass_on(p, p->cfg_row, mode, a, s));
      }
      return BCCB_OK;
    }));
  }
  BCCB_TRY(kern(launch_crop(p->d_emb_c, p->A1, p->A2, p->L1, out, p->stream)));
  return end_call(p);
}

int spaced_admm(bccb_plan_s* p, const float2* y, float tau, float rho, int iters, float2* zo, float2* co) {
  if (!p->emb_circulant) return BCCB_E_UNSUPPORTED;
  BCCB_TRY(ensure_rho(p, rho));
  BCCB_TRY(begin_call(p));
  // w = (G + rho I)^-1 b: b padded, then the product with the embedded inverse (multiplier
  // Omega_rho / L), the window of which is w (outside it the row pass ignores w)
  BCCB_TRY(adjoint_to(p, y, 1.f, p->d_emb_c2, true));
  RowArgs f;
  f.xy = p->d_xy;
  f.src = p->d_emb_c2;
  BCCB_TRY(row_pass(p, ROW_FWD, f));
  const double invL = 1.0 / static_cast<double>(p->L);
  const float2 coef[2] = {make_float2(0.f, static_cast<float>(invL)),
                          make_float2(0.f, static_cast<float>(static_cast<double>(rho) * invL))};
  std::memcpy(p->h_red, coef, sizeof(coef));   // the stream is drained: the pinned buffer is free
  BCCB_HIP(hipMemcpyAsync(p->d_emb_coef, p->h_red, sizeof(coef), hipMemcpyHostToDevice, p->stream));
  BCCB_TRY(col_pass_spectrum(p, COL_FILTER_AFFINE, p->d_xy, p->d_omega_rho, p->d_emb_coef, p->stream));
  RowArgs wi;
  wi.xy = p->d_xy;
  wi.dst = p->d_rhs;
  BCCB_TRY(row_pass(p, ROW_INV, wi));
  // z^(0) = v^(0) = 0
  BCCB_TRY(kern(launch_fill(p->d_state, p->L, p->stream)));
  BCCB_TRY(kern(launch_fill(p->d_xy, p->L, p->stream)));
  BCCB_TRY(kern(launch_fill(p->d_emb_c, p->L, p->stream)));
  BCCB_TRY(kern(launch_fill(p->d_emb_c2, p->L, p->stream)));
  const float kappa = tau / rho;
  if (iters > 0) {
    const unsigned long long key[8] = {static_cast<unsigned long long>(ROW_ADMM), static_cast<unsigned long long>(iters),
                                       reinterpret_cast<unsigned long long>(p->d_emb_c), fbits(kappa),
                                       reinterpret_cast<unsigned long long>(p->d_emb_c2), fbits(rho), 0, 6};
    BCCB_TRY(run_loop(p, key, [&](hipStream_t s) -> int {
      for (int t = 1; t <= iters; ++t) {
        // rho (G + rho I)^-1 (z - v): multiplier rho Omega_rho / L
        BCCB_TRY(col_pass_spectrum(p, COL_FILTER_AFFINE, p->d_xy, p->d_omega_rho, p->d_emb_coef + 1, s));
        RowArgs a = window_args(p);
        a.xy = p->d_xy;
        a.rhs = p->d_rhs;
        a.state = p->d_state;
        a.out_z = p->d_emb_c;
        a.out_c = p->d_emb_c2;
        a.kappa = kappa;
        a.last = (t == iters);
        BCCB_TRY(row_pass_on(p, p->cfg_row, ROW_ADMM, a, s));
      }
      return BCCB_OK;
    }));
  }
  BCCB_TRY(kern(launch_crop(p->d_emb_c, p->A1, p->A2, p->L1, zo, p->stream)));
  if (co) BCCB_TRY(kern(launch_crop(p->d_emb_c2, p->A1, p->A2, p->L1, co, p->stream)));
  return end_call(p);
}

int spaced_objective_kkt(bccb_plan_s* p, const float2* y, float tau, const float2* c, double* objective,
                         double* r_kkt, double* max_e_over_tau) {
  BCCB_TRY(begin_call(p));
  int nb_r = 0, nb_k = 0;
  double* part_r = p->d_red;
  double* part_k = p->d_red + kReduceBlocks;
  // 1/2 ||y - D_s c||^2 through the separable product (eq. (4))
  BCCB_TRY(kern(launch_sep_resid(c, p->A1, p->d_W1, p->d_W2, p->d_sensors, y, p->M, p->M1, p->A1, p->A2,
                                 p->d_emb_u, part_r, &nb_r, p->d_flag, p->stream)));
  // G c (window of the embedded product) into d_tmp, b = D_s^H y into d_rhs, both A1 x A2
  BCCB_TRY(gram_into(p, c, p->d_tmp));
  BCCB_TRY(adjoint_to(p, y, 1.f, p->d_rhs, false));
  BCCB_TRY(kern(launch_kkt(c, p->d_rhs, p->d_tmp, tau, p->AL, part_k, &nb_k, p->stream)));
  BCCB_HIP(hipMemcpyAsync(p->h_red, p->d_red, kReduceBlocks * 5 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  const int rc = end_call(p);
  double rs = 0.0, e2 = 0.0, emax = 0.0, l1 = 0.0, b2 = 0.0;
  for (int i = 0; i < nb_r; ++i) rs += p->h_red[i];
  const double* hk = p->h_red + kReduceBlocks;
  for (int i = 0; i < nb_k; ++i) {
    e2 += hk[4 * i + 0];
    emax = hk[4 * i + 1] > emax ? hk[4 * i + 1] : emax;
    l1 += hk[4 * i + 2];
    b2 += hk[4 * i + 3];
  }
  if (objective) *objective = rs + static_cast<double>(tau) * l1;   // the partials hold 1/2 |r|^2
  if (r_kkt) *r_kkt = b2 > 0.0 ? std::sqrt(e2) / std::sqrt(b2) : std::sqrt(e2);
  if (max_e_over_tau) *max_e_over_tau = tau > 0.f ? emax / tau : emax;
  return rc;
}

}  // namespace bccb

using namespace bccb;

extern "C" int bccb_plan_spaced(const uint8_t* mask, int M1, int M2, int L1, int L2, double gamma1, double gamma2,
                                void* stream, bccb_plan_t* out) {
  if (!out) return BCCB_E_INVALID;
  *out = nullptr;
  if (!mask || M1 < 1 || M2 < 1 || M1 > 4096 || M2 > 4096) return BCCB_E_INVALID;
  if (!(gamma1 > 0.0 && gamma1 <= 1.0) || !(gamma2 > 0.0 && gamma2 <= 1.0)) return BCCB_E_INVALID;
  if (L1 < 2 || L2 < 2 || L1 > 512 || L2 > 512) {
    // the power-of-two half-spacing grids up to 1024 are the ordinary plans
    if (!(gamma1 == 0.5 && gamma2 == 0.5 && pow2(L1) && pow2(L2) && L1 >= 8 && L2 >= 8 && L1 <= 1024 && L2 <= 1024))
      return L1 < 1 || L2 < 1 ? BCCB_E_INVALID : BCCB_E_UNSUPPORTED;
  }
  long M = 0;
  for (long i = 0; i < static_cast<long>(M1) * M2; ++i) M += mask[i] ? 1 : 0;
  if (M == 0) return BCCB_E_INVALID;
  const bool circulant = gamma1 == 0.5 && gamma2 == 0.5;
  if (circulant && pow2(L1) && pow2(L2) && L1 >= 8 && L2 >= 8) return bccb_plan(mask, M1, M2, L1, L2, stream, out);
  if (!circulant && M > 2048) return BCCB_E_UNSUPPORTED;   // the step's M x M eigenproblem

  bccb_plan_s* p = new (std::nothrow) bccb_plan_s();
  if (!p) return BCCB_E_NOMEM;
  p->emb = true;
  p->M1 = M1;
  p->M2 = M2;
  p->A1 = L1;
  p->A2 = L2;
  p->AL = static_cast<long>(L1) * L2;
  p->L1 = embed_length(L1);
  p->L2 = embed_length(L2);
  p->L = static_cast<long>(p->L1) * p->L2;
  p->gamma1 = gamma1;
  p->gamma2 = gamma2;
  p->emb_circulant = circulant;
  p->M = static_cast<int>(M);
  p->stream = static_cast<hipStream_t>(stream);
  p->use_support = 0;
  p->use_prune = 0;
  p->sparse_iterate = 0;
  p->resident_groups = 0;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return BCCB_E_DEVICE;
  }
  p->mask.assign(mask, mask + static_cast<size_t>(M1) * M2);
  std::vector<int> sensor_of(static_cast<size_t>(M1) * M2, -1);
  std::vector<int2> sensors;
  for (int m2 = 0; m2 < M2; ++m2)
    for (int m1 = 0; m1 < M1; ++m1)
      if (mask[static_cast<size_t>(m2) * M1 + m1]) {
        sensor_of[static_cast<size_t>(m2) * M1 + m1] = static_cast<int>(sensors.size());
        sensors.push_back(make_int2(m1, m2));
      }

  // step mu = 1/sigma_max(D_s)^2 (eq. (9)): at gamma = 1/2 the largest eigenvalue of the
  // A1 x A2 BCCB (eq. (21)); otherwise Lanczos on D_s D_s^H
  if (circulant) {
    p->emb_omega = circulant_eigenvalues(mask, M1, M2, L1, L2);
    p->mu = 1.0 / *std::max_element(p->emb_omega.begin(), p->emb_omega.end());
  } else {
    p->mu = 1.0 / gram_max_eigenvalue(mask, M1, M2, L1, L2, gamma1, gamma2);
  }
  const std::vector<double> om = toeplitz_embedding_spectrum(mask, M1, M2, L1, L2, gamma1, gamma2, p->L1, p->L2);
  p->omega32.resize(p->L);
  for (long i = 0; i < p->L; ++i) p->omega32[i] = static_cast<float>(om[i]);
  const std::vector<float2> W1 = to_c64(steering_table(M1, L1, gamma1));
  const std::vector<float2> W2 = to_c64(steering_table(M2, L2, gamma2));
  std::vector<float2> tw1(p->L1), tw2(p->L2);
  {
    const std::vector<cd> w1 = unit_roots(p->L1), w2 = unit_roots(p->L2);
    for (int j = 0; j < p->L1; ++j) tw1[j] = make_float2(static_cast<float>(w1[j].real()), static_cast<float>(w1[j].imag()));
    for (int j = 0; j < p->L2; ++j) tw2[j] = make_float2(static_cast<float>(w2[j].real()), static_cast<float>(w2[j].imag()));
  }
  const double invL = 1.0 / static_cast<double>(p->L);
  const float2 coef[2] = {make_float2(static_cast<float>(invL), static_cast<float>(-p->mu * invL)),
                          make_float2(0.f, static_cast<float>(invL))};
  const size_t nu = std::max(static_cast<size_t>(M2) * L1, static_cast<size_t>(L2) * M1);

  int rc = BCCB_OK;
  if (rc == BCCB_OK) rc = dalloc(&p->d_omega, p->L);
  if (rc == BCCB_OK) rc = dalloc(&p->d_sensor_of, sensor_of.size());
  if (rc == BCCB_OK) rc = dalloc(&p->d_sensors, sensors.size());
  if (rc == BCCB_OK) rc = dalloc(&p->d_tw1, p->L1);
  if (rc == BCCB_OK) rc = dalloc(&p->d_tw2, p->L2);
  if (rc == BCCB_OK) rc = dalloc(&p->d_xy, p->L);
  if (rc == BCCB_OK) rc = dalloc(&p->d_rhs, p->L);
  if (rc == BCCB_OK) rc = dalloc(&p->d_state, p->L);
  if (rc == BCCB_OK) rc = dalloc(&p->d_tmp, p->L);
  if (rc == BCCB_OK) rc = dalloc(&p->d_coef, 2);
  if (rc == BCCB_OK) rc = dalloc(&p->d_red, static_cast<size_t>(kReduceBlocks) * 8);
  if (rc == BCCB_OK) rc = dalloc(&p->d_flag, 1);
  if (rc == BCCB_OK) rc = dalloc(&p->d_W1, W1.size());
  if (rc == BCCB_OK) rc = dalloc(&p->d_W2, W2.size());
  if (rc == BCCB_OK) rc = dalloc(&p->d_emb_u, nu);
  if (rc == BCCB_OK) rc = dalloc(&p->d_emb_c, p->L);
  if (rc == BCCB_OK) rc = dalloc(&p->d_emb_c2, p->L);
  if (rc == BCCB_OK && circulant) rc = dalloc(&p->d_omega_rho, p->L);
  if (rc == BCCB_OK) rc = dalloc(&p->d_emb_coef, 2);
  if (rc == BCCB_OK && hipHostMalloc(reinterpret_cast<void**>(&p->h_red), kReduceBlocks * 8 * sizeof(double)) != hipSuccess)
    rc = BCCB_E_NOMEM;
  if (rc == BCCB_OK && hipHostMalloc(reinterpret_cast<void**>(&p->h_flag), sizeof(int)) != hipSuccess) rc = BCCB_E_NOMEM;
  if (rc == BCCB_OK) rc = upload(p->d_omega, p->omega32.data(), p->omega32.size());
  if (rc == BCCB_OK) rc = upload(p->d_sensor_of, sensor_of.data(), sensor_of.size());
  if (rc == BCCB_OK) rc = upload(p->d_sensors, sensors.data(), sensors.size());
  if (rc == BCCB_OK) rc = upload(p->d_tw1, tw1.data(), tw1.size());
  if (rc == BCCB_OK) rc = upload(p->d_tw2, tw2.data(), tw2.size());
  if (rc == BCCB_OK) rc = upload(p->d_coef, coef, 2);
  if (rc == BCCB_OK) rc = upload(p->d_W1, W1.data(), W1.size());
  if (rc == BCCB_OK) rc = upload(p->d_W2, W2.data(), W2.size());
  if (rc != BCCB_OK) {
    plan_free(p);
    return rc;
  }
  default_config(p);
  *out = p;
  return BCCB_OK;
}

extern "C" int bccb_plan_embedding(bccb_plan_t p, int* P1, int* P2, float* omega_host) {
  if (!p) return BCCB_E_INVALID;
  if (!p->emb) return BCCB_E_UNSUPPORTED;
  if (P1) *P1 = p->L1;
  if (P2) *P2 = p->L2;
  if (omega_host) std::memcpy(omega_host, p->omega32.data(), p->omega32.size() * sizeof(float));
  return BCCB_OK;
}
