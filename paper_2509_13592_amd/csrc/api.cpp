// C ABI of libbccb: argument checks, plans, and the solver drivers that
// enqueue the row/column passes (see include/bccb.h for the contract).
#include "bccb.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "kernels.h"
#include "plan_internal.h"
#include "spaced_api.h"
#include "plan_math.h"

using bccb::ColArgs;
using bccb::RowArgs;

namespace bccb {

bool is_pow2_in_range(int L) { return L >= 8 && L <= 1024 && (L & (L - 1)) == 0; }

int check_geometry(const uint8_t* mask, int M1, int M2, int L1, int L2) {
  if (!mask || M1 < 1 || M2 < 1 || M1 > 4096 || M2 > 4096 || L1 <= 0 || L2 <= 0) return BCCB_E_INVALID;
  if (!is_pow2_in_range(L1) || !is_pow2_in_range(L2)) return BCCB_E_UNSUPPORTED;
  long kept = 0;
  for (long i = 0; i < static_cast<long>(M1) * M2; ++i) kept += mask[i] != 0;
  if (kept == 0) return BCCB_E_INVALID;
  return BCCB_OK;
}

template <typename T>
static int dmalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  if (hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return BCCB_E_NOMEM;
  }
  return BCCB_OK;
}

static void dfree(void* p) {
  if (p) (void)hipFree(p);
}

void plan_free(bccb_plan_s* p) {
  if (!p) return;
  drop_graph(p);
  dfree(p->d_W1);
  dfree(p->d_W2);
  dfree(p->d_emb_u);
  dfree(p->d_emb_c);
  dfree(p->d_emb_c2);
  dfree(p->d_omega_rho);
  dfree(p->d_emb_coef);
  dfree(p->d_cand);
  dfree(p->d_ccount);
  dfree(p->d_omega64);
  dfree(p->d_tw1_64);
  dfree(p->d_tw2_64);
  dfree(p->d_xy64);
  dfree(p->d_rhs64);
  dfree(p->d_state64);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  dfree(p->d_omega);
  dfree(p->d_sensor_of);
  dfree(p->d_sensors);
  dfree(p->d_tw1);
  dfree(p->d_tw2);
  dfree(p->d_xy);
  dfree(p->d_rhs);
  dfree(p->d_state);
  dfree(p->d_cnt);
  dfree(p->d_sidx);
  dfree(p->d_sval);
  dfree(p->d_scol);
  dfree(p->d_colslot);
  dfree(p->d_xyc);
  for (int i = 0; i < 3; ++i) {
    dfree(p->d_pcnt[i]);
    dfree(p->d_psidx[i]);
    dfree(p->d_psval[i]);
    dfree(p->d_pdense[i]);
  }
  dfree(p->d_tmp);
  dfree(p->d_beta);
  dfree(p->d_sync);
  dfree(p->d_rpart);
  dfree(p->d_psi);
  dfree(p->d_vlast);
  dfree(p->d_coef);
  dfree(p->d_red);
  dfree(p->d_flag);
  dfree(p->d_sup_ptr);
  dfree(p->d_sup);
  dfree(p->d_src_ptr);
  dfree(p->d_src);
  dfree(p->d_sup_rhs);
  dfree(p->d_sup_desc);
  if (p->h_sup_desc) (void)hipHostFree(p->h_sup_desc);
  if (p->h_red) (void)hipHostFree(p->h_red);
  if (p->h_flag) (void)hipHostFree(p->h_flag);
  delete p;
}


// --- pass helpers on one plan ------------------------------------------------
int row_pass_on(bccb_plan_s* p, const PassCfg& cfg, int mode, RowArgs a, hipStream_t s) {
  a.tw = p->d_tw1;
  a.nrows = p->L2;
  a.rows_per_scene = p->L2;
  return kern(launch_row(p->L1, cfg, mode, a, s));
}

int col_pass_on(bccb_plan_s* p, const PassCfg& cfg, int mode, float2* xy, const float2* coef, float rho,
                float scale, hipStream_t s) {
  ColArgs a;
  a.xy = xy;
  a.sup_ptr = p->d_sup_ptr;
  a.sup = p->d_sup;
  a.sup_rhs = p->d_sup_rhs;
  a.omega = p->d_omega;
  a.coef = coef;
  a.tw = p->d_tw2;
  a.L1 = p->L1;
  a.nscenes = 1;
  a.rho = rho;
  a.scale = scale;
  return kern(launch_col(p->L2, cfg, mode, a, s));
}

int row_pass(bccb_plan_s* p, int mode, RowArgs a) { return row_pass_on(p, p->cfg_row, mode, a, p->stream); }

int col_pass(bccb_plan_s* p, int mode, float2* xy, const float2* coef, float rho, float scale) {
  return col_pass_on(p, p->cfg_col, mode, xy, coef, rho, scale, p->stream);
}

// --- launch shapes -------------------------------------------------------------
bool elems_ok(int N, int E) {
  if (E != 4 && E != 8 && E != 16 && E != 32) return false;
  if (E > N || N / E > 256) return false;
  if (N == 8 && E > 8) return false;
  return true;
}

bool row_shape_ok(int L1, const PassCfg& c, bool sparse_iterate) {
  if (!elems_ok(L1, c.E) || c.rpb < 1) return false;
  const int T = L1 / c.E;
  const long counts = sparse_iterate ? static_cast<long>(c.rpb) * T * 4 : 0;  // per-thread nonzero counts
  return c.rpb * T <= 256 && (static_cast<long>(fft_areas(L1, c.E)) * c.rpb * fft_area(L1) + L1) * 8 + counts <= 65536;
}

bool col_shape_ok(int L1, int L2, const PassCfg& c) {
  if (!elems_ok(L2, c.E) || c.W < 1 || L1 % c.W != 0) return false;
  const int T = L2 / c.E;
  return c.W * T <= 256 && (static_cast<long>(fft_areas(L2, c.E)) * c.W * fft_area(L2) + L2) * 8 <= 65536;
}

bool rowp_shape_ok(int L1, const PassCfg& c, int ncs) {
  if (!elems_ok(L1, c.E) || c.rpb < 1 || ncs < 1 || ncs > L1 / 2) return false;
  const int T = L1 / c.E;
  return c.rpb * T <= 256 && rowp_lds_floats(L1, c.E, c.rpb, ncs) * 8 <= 65536;
}

bool colp_shape_ok(int ncs, int L2, const PassCfg& c) { return ncs >= 1 && col_shape_ok(ncs, L2, c); }

bool pruned_on(const bccb_plan_s* p) { return p->prune_ok && p->use_prune && p->has_support && p->use_support; }

bool resident_on(const bccb_plan_s* p) { return p->resident_groups > 0 && p->has_support && p->use_support; }

// The cooperative solver can run on this plan with G working workgroups, spread
// launched per working one, for all three solvers.
static bool resident_shape_ok(const bccb_plan_s* p, int groups, int spread) {
  if (groups < 1 || groups > kResidentMaxGroups || !(spread == 1 || spread == 2 || spread == 4 || spread == 8))
    return false;
  ResidentArgs a;
  a.groups = groups;
  a.spread = spread;
  for (int m = RES_ISTA; m <= RES_ADMM; ++m)
    if (launch_resident(p->L1, p->L2, m, a, 1, nullptr) != 0) return false;
  return true;
}

// Groups of the pruned cooperative form: rows of 4 block / L1 per group of
// `block` threads (256 or 512), 0 if that does not tile the grid.
static int resident_pruned_groups(const bccb_plan_s* p, int block) {
  const int rpc = 4 * block / p->L1;
  return rpc >= 1 && rpc <= p->L2 && p->L2 % rpc == 0 ? p->L2 / rpc : 0;
}
static int resident_pruned_groups(const bccb_plan_s* p) { return resident_pruned_groups(p, p->resident_block); }

// The solves take the pruned cooperative form when they would take the pruned
// passes otherwise (pruned_on) and that form can be launched with the plan's
// spread and block for all three solvers (cached per spread and block: the
// check queries the occupancy API).
static bool resident_pruned_on(bccb_plan_s* p) {
  if (!pruned_on(p) || !p->d_rpart) return false;
  if (p->res_pruned_spread != p->resident_spread || p->res_pruned_block != p->resident_block) {
    ResidentArgs a;
    a.groups = resident_pruned_groups(p);
    a.spread = p->resident_spread;
    a.ncs = p->ncs;
    a.nsup = p->nsup;
    p->res_pruned_ok = a.groups > 0 && launch_resident(p->L1, p->L2, RES_PRUNED_FISTA, a, 1, nullptr) == 0 &&
                       launch_resident(p->L1, p->L2, RES_PRUNED_ISTA, a, 1, nullptr) == 0 &&
                       launch_resident(p->L1, p->L2, RES_PRUNED_ADMM, a, 1, nullptr) == 0;
    p->res_pruned_spread = p->resident_spread;
    p->res_pruned_block = p->resident_block;
  }
  return p->res_pruned_ok;
}

// FISTA momenta beta_t = (alpha_t - 1) / alpha_{t+1} of eqs. (10)-(12) for t = 1..iters in
// d_beta[t - 1], computed on the host exactly as the two-pass driver does (the
// sequence does not depend on the iteration count, so the table only grows).
static int ensure_beta(bccb_plan_s* p, int iters) {
  if (iters <= p->beta_cap) return BCCB_OK;
  int cap = p->beta_cap > 0 ? p->beta_cap : 1024;
  while (cap < iters) cap = cap > (1 << 29) ? iters : cap * 2;
  std::vector<float> h(cap);
  double alpha = 1.0;
  for (int t = 0; t < cap; ++t) {
    const double alpha_next = (1.0 + std::sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0;
    h[t] = static_cast<float>((alpha - 1.0) / alpha_next);
    alpha = alpha_next;
  }
  BCCB_HIP(hipStreamSynchronize(p->stream));
  dfree(p->d_beta);
  p->d_beta = nullptr;
  p->beta_cap = 0;
  BCCB_TRY(dmalloc(&p->d_beta, static_cast<size_t>(cap)));
  BCCB_HIP(hipMemcpy(p->d_beta, h.data(), static_cast<size_t>(cap) * sizeof(float), hipMemcpyHostToDevice));
  p->beta_cap = cap;
  return BCCB_OK;
}

// Enqueue one cooperative solve on stream s (the right-hand side on the support
// bins already in d_sup_rhs).  mode: RES_ISTA / RES_FISTA (kappa = mu tau; out_c
// receives c^(T)) or RES_ADMM (kappa = tau / rho, scale = rho / L; out_z, out_c),
// each in the pruned form when the plan takes it.
static int resident_enqueue(bccb_plan_s* p, int mode, int iters, float kappa, float rho, float scale,
                            const float2* init, float2* out_c, float2* out_z, hipStream_t s) {
  if (2 * static_cast<long long>(iters) + 1 >= (1ll << 31)) return BCCB_E_UNSUPPORTED;   // barrier epochs
  const bool pruned = resident_pruned_on(p);
  if (pruned) mode = mode == RES_FISTA ? RES_PRUNED_FISTA : (mode == RES_ADMM ? RES_PRUNED_ADMM : RES_PRUNED_ISTA);
  const int groups = pruned ? resident_pruned_groups(p) : p->resident_groups;
  if (mode == RES_FISTA || mode == RES_PRUNED_FISTA) BCCB_TRY(ensure_beta(p, iters));
  // a fresh tag per solve: the sync words keep what earlier solves wrote (all below it)
  const unsigned long long tag = (++p->res_solve) << 32;
  ResidentArgs a;
  a.xy = pruned ? p->d_rpart : p->d_xy;
  a.scol = p->d_scol;
  a.colslot = p->d_colslot;
  a.ncs = p->ncs;
  a.nsup = p->nsup;
  a.init = init;
  a.out_c = out_c;
  a.out_z = out_z;
  a.tw1 = p->d_tw1;
  a.tw2 = p->d_tw2;
  a.beta = p->d_beta;
  a.coef = p->d_coef;
  a.sup_ptr = p->d_sup_ptr;
  a.sup = p->d_sup;
  a.sup_rhs = p->d_sup_rhs;
  a.kappa = kappa;
  a.rho = rho;
  a.scale = scale;
  a.iters = iters;
  a.groups = groups;
  a.spread = p->resident_spread;
  a.sync = p->d_sync;
  a.tag = tag;
  a.flag = p->d_flag;
  a.timeout_ticks = p->wall_ticks_per_s;   // one second per barrier wait
  return kern(launch_resident(p->L1, p->L2, mode, a, 0, s));
}

// Latency-oriented default: E = 4, about one wave per workgroup.
void default_config(bccb_plan_s* p) {
  p->cfg_row.E = 4;
  const int Tr = p->L1 / 4;
  p->cfg_row.rpb = Tr >= 64 ? 1 : 64 / Tr;
  p->cfg_col.E = 4;
  const int Tc = p->L2 / 4;
  int W = Tc >= 64 ? 1 : 64 / Tc;
  if (W > p->L1) W = p->L1;
  p->cfg_col.W = W;
  // A pass of at most 32 workgroups fits one die's 32 CUs: spreading it keeps
  // the scene in that die's L2 between passes.
  if ((p->L2 + p->cfg_row.rpb - 1) / p->cfg_row.rpb <= 32) p->cfg_row.spread = 8;
  if (p->L1 / W <= 32) p->cfg_col.spread = 8;
  p->cfg_rowp = p->cfg_row;
  while (!rowp_shape_ok(p->L1, p->cfg_rowp, p->ncs) && p->cfg_rowp.rpb > 1) p->cfg_rowp.rpb /= 2;
  p->cfg_colp.E = 4;
  p->cfg_colp.W = 1;   // one kept column per workgroup: the most workgroups for a single scene
}

void drop_graph(bccb_plan_s* p) {
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  p->graph_exec = nullptr;
  for (auto& k : p->graph_key) k = 0;
}

// b (or scale*b) = D_s^H y into dst, using p->d_tmp as the spectral scratch.
int adjoint_into(bccb_plan_s* p, const float2* y, float scale, float2* dst) {
  BCCB_TRY(kern(launch_scatter(y, p->d_sensor_of, p->M1, p->M2, p->L1, p->L2, scale, p->d_tmp, p->d_flag,
                               p->stream)));
  BCCB_TRY(col_pass(p, COL_INV, p->d_tmp, nullptr, 0.f, 1.f));
  RowArgs a;
  a.xy = p->d_tmp;
  a.dst = dst;
  a.scale = 1.f;
  return row_pass(p, ROW_INV, a);
}

bool sparse_on(const bccb_plan_s* p) { return p->has_support && p->use_support; }

// Spectral right-hand side on the support bins: scale * (scattered snapshot).
int fill_sup_rhs(bccb_plan_s* p, const float2* y, float scale) {
  SupRhsDesc& d = *p->h_sup_desc;
  d.y = y;
  d.entry_off = 0;
  d.nentries = p->nsup;
  d.rhs_off = 0;
  d.scale = scale;
  BCCB_HIP(hipMemcpyAsync(p->d_sup_desc, p->h_sup_desc, sizeof(SupRhsDesc), hipMemcpyHostToDevice, p->stream));
  return kern(launch_sup_rhs(p->d_sup_desc, 1, p->nsup, p->d_src_ptr, p->d_src, p->d_sup_rhs, p->d_flag, p->stream));
}

int begin_call(bccb_plan_s* p) {
  BCCB_HIP(hipMemsetAsync(p->d_flag, 0, sizeof(int), p->stream));
  return BCCB_OK;
}

// Drain the stream and report a non-finite input seen by any pass.
int end_call(bccb_plan_s* p) {
  BCCB_HIP(hipMemcpyAsync(p->h_flag, p->d_flag, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  BCCB_HIP(hipStreamSynchronize(p->stream));
  if (*p->h_flag & 2) return BCCB_E_DEVICE;   // a grid barrier of the cooperative solver timed out
  return *p->h_flag ? BCCB_E_NONFINITE : BCCB_OK;
}

}  // namespace bccb

using namespace bccb;

extern "C" {

const char* bccb_status_string(int status) {
  switch (status) {
    case BCCB_OK: return "BCCB_OK";
    case BCCB_E_INVALID: return "BCCB_E_INVALID: invalid argument";
    case BCCB_E_UNSUPPORTED: return "BCCB_E_UNSUPPORTED: unsupported size or option";
    case BCCB_E_NOMEM: return "BCCB_E_NOMEM: device allocation failed";
    case BCCB_E_DEVICE: return "BCCB_E_DEVICE: HIP runtime error";
    case BCCB_E_NONFINITE: return "BCCB_E_NONFINITE: NaN or Inf in the input";
    case BCCB_E_SCRATCH: return "BCCB_E_SCRATCH: grid larger than the allocation-free entry point's static array";
    default: return "unknown bccb status";
  }
}

int bccb_plan(const uint8_t* mask, int M1, int M2, int L1, int L2, void* stream, bccb_plan_t* out) {
  if (!out) return BCCB_E_INVALID;
  *out = nullptr;
  BCCB_TRY(check_geometry(mask, M1, M2, L1, L2));

  bccb_plan_s* p = new (std::nothrow) bccb_plan_s();
  if (!p) return BCCB_E_NOMEM;
  p->M1 = M1;
  p->M2 = M2;
  p->L1 = L1;
  p->L2 = L2;
  p->L = static_cast<long>(L1) * L2;
  p->stream = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return BCCB_E_DEVICE;
  }

  // sensors in increasing m1 + m2*M1 (rows of Psi, eq. (6))
  std::vector<int> sensor_of(static_cast<size_t>(M1) * M2, -1);
  std::vector<int2> sensors;
  for (int m2 = 0; m2 < M2; ++m2)
    for (int m1 = 0; m1 < M1; ++m1)
      if (mask[static_cast<size_t>(m2) * M1 + m1]) {
        sensor_of[static_cast<size_t>(m2) * M1 + m1] = static_cast<int>(sensors.size());
        sensors.push_back(make_int2(m1, m2));
      }
  p->M = static_cast<int>(sensors.size());
  p->mask.assign(mask, mask + static_cast<size_t>(M1) * M2);

  // eigenvalues (eq. (21)) in FP64 from the first column of the Gram
  const std::vector<cd> r = gram_first_column(mask, M1, M2, L1, L2);
  const std::vector<cd> om = eigenvalues_eq21(r, L1, L2);
  p->omega32.resize(p->L);
  double omax = 0.0;
  for (long i = 0; i < p->L; ++i) omax = std::max(omax, om[i].real());
  p->mu = 1.0 / omax;  // sigma_max(D_s)^2 = lambda_max(G) = max Omega
  // G is Hermitian PSD, so Omega is real and >= 0; eq. (21) gives L1 L2 times the
  // number of elements folding onto each bin, so bins no element folds onto hold
  // only FP64 rounding (~1e-12 of the maximum) and are stored as exact zeros.
  for (long i = 0; i < p->L; ++i) {
    const double v = om[i].real();
    p->omega32[i] = (std::fabs(v) > 1e-9 * omax) ? static_cast<float>(v) : 0.f;
  }
  // support list by column, with the snapshot entries folding onto each bin
  {
    std::vector<std::vector<int>> bin_src(p->L);
    for (int m = 0; m < p->M; ++m) {
      const int m1 = sensors[m].x, m2 = sensors[m].y;
      const long bin = static_cast<long>(m2 % L2) * L1 + (m1 % L1);
      bin_src[bin].push_back((m << 1) | ((m1 + m2) & 1));
    }
    p->h_sup_ptr.assign(L1 + 1, 0);
    p->h_src_ptr.assign(1, 0);
    for (int k1 = 0; k1 < L1; ++k1) {
      p->h_sup_ptr[k1] = static_cast<int>(p->h_sup.size());
      for (int k2 = 0; k2 < L2; ++k2) {
        const long bin = static_cast<long>(k2) * L1 + k1;
        if (p->omega32[bin] == 0.f && bin_src[bin].empty()) continue;
        p->h_sup.push_back(bccb::SupEntry{k2, p->omega32[bin]});
        for (int c : bin_src[bin]) p->h_src.push_back(c);
        p->h_src_ptr.push_back(static_cast<int>(p->h_src.size()));
      }
    }
    p->h_sup_ptr[L1] = static_cast<int>(p->h_sup.size());
    p->nsup = static_cast<int>(p->h_sup.size());
    p->has_support = p->nsup <= p->L / 4;
    // spectral columns holding support bins (the pruned iteration transforms only these)
    for (int k1 = 0; k1 < L1; ++k1)
      if (p->h_sup_ptr[k1 + 1] > p->h_sup_ptr[k1]) p->h_scol.push_back(k1);
    p->nscol = static_cast<int>(p->h_scol.size());
    p->ncs = (p->nscol + 3) / 4 * 4;
    p->prune_ok = p->has_support && L1 >= 8 && p->nscol >= 1 && p->ncs <= L1 / 2;
    p->h_scol.resize(p->ncs, -1);
  }

  std::vector<float2> tw1(L1), tw2(L2);
  {
    const std::vector<cd> w1 = unit_roots(L1), w2 = unit_roots(L2);
    for (int j = 0; j < L1; ++j) tw1[j] = make_float2(static_cast<float>(w1[j].real()), static_cast<float>(w1[j].imag()));
    for (int j = 0; j < L2; ++j) tw2[j] = make_float2(static_cast<float>(w2[j].real()), static_cast<float>(w2[j].imag()));
  }
  const double invL = 1.0 / static_cast<double>(p->L);
  const float2 coef[2] = {make_float2(static_cast<float>(invL), static_cast<float>(-p->mu * invL)),
                          make_float2(0.f, static_cast<float>(invL))};

  int rc = BCCB_OK;
  if (rc == BCCB_OK) rc = dmalloc(&p->d_omega, p->L);
  if (rc == BCCB_OK) rc = dmalloc(&p->d_sensor_of, sensor_of.size());
  if (rc == BCCB_OK) rc = dmalloc(&p->d_sensors, sensors.size());
  if (rc == BCCB_OK) rc = dmalloc(&p->d_tw1, L1);
  if (rc == BCCB_OK) rc = dmalloc(&p->d_tw2, L2);
  if (rc == BCCB_OK) rc = dmalloc(&p->d_xy, p->L);
  if (rc == BCCB_OK) rc = dmalloc(&p->d_rhs, p->L);
  if (rc == BCCB_OK) rc = dmalloc(&p->d_state, p->L);
  if (rc == BCCB_OK) rc = dmalloc(&p->d_cnt, L2);
  if (rc == BCCB_OK) rc = dmalloc(&p->d_sidx, static_cast<size_t>(L2) * (L1 / 8 > 0 ? L1 / 8 : 1));
  if (rc == BCCB_OK) rc = dmalloc(&p->d_sval, static_cast<size_t>(L2) * (L1 / 8 > 0 ? L1 / 8 : 1));
  // every row starts out dense: no slot is read before the kernel has written it
  if (rc == BCCB_OK && hipMemset(p->d_cnt, 0x7f, L2 * sizeof(int)) != hipSuccess) rc = BCCB_E_DEVICE;
  if (rc == BCCB_OK) rc = dmalloc(&p->d_tmp, p->L);
  if (rc == BCCB_OK && p->prune_ok) {
    const size_t cap = static_cast<size_t>(L2) * (L1 / 8);
    std::vector<int> colslot(L1, -1);
    for (int j = 0; j < p->nscol; ++j) colslot[p->h_scol[j]] = j;
    rc = dmalloc(&p->d_scol, p->ncs);
    if (rc == BCCB_OK) rc = dmalloc(&p->d_colslot, L1);
    if (rc == BCCB_OK) rc = dmalloc(&p->d_xyc, static_cast<size_t>(L2) * p->ncs);
    for (int i = 0; i < 3 && rc == BCCB_OK; ++i) {
      rc = dmalloc(&p->d_pcnt[i], L2);
      if (rc == BCCB_OK) rc = dmalloc(&p->d_psidx[i], cap);
      if (rc == BCCB_OK) rc = dmalloc(&p->d_psval[i], cap);
      if (rc == BCCB_OK) rc = dmalloc(&p->d_pdense[i], p->L);
      // rows start out dense over a zeroed grid: nothing unwritten is ever read
      if (rc == BCCB_OK && (hipMemset(p->d_pcnt[i], 0x7f, L2 * sizeof(int)) != hipSuccess ||
                            hipMemset(p->d_pdense[i], 0, p->L * sizeof(float2)) != hipSuccess))
        rc = BCCB_E_DEVICE;
    }
    if (rc == BCCB_OK) rc = dmalloc(&p->d_psi, p->nsup);
    if (rc == BCCB_OK) rc = dmalloc(&p->d_vlast, p->nsup);
    if (rc == BCCB_OK && (hipMemcpy(p->d_scol, p->h_scol.data(), p->ncs * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
                          hipMemcpy(p->d_colslot, colslot.data(), L1 * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
                          hipMemset(p->d_xyc, 0, static_cast<size_t>(L2) * p->ncs * sizeof(float2)) != hipSuccess))
      rc = BCCB_E_DEVICE;
  }
  if (rc == BCCB_OK) rc = dmalloc(&p->d_coef, 2);
  if (rc == BCCB_OK) rc = dmalloc(&p->d_sync, kResidentSyncWords);
  if (rc == BCCB_OK && hipMemset(p->d_sync, 0, kResidentSyncWords * sizeof(unsigned long long)) != hipSuccess)
    rc = BCCB_E_DEVICE;
  // the pruned cooperative form's per-group parts of DFT2 at the support bins (two
  // buffers, by iteration parity)
  if (rc == BCCB_OK && p->prune_ok && resident_pruned_groups(p, 256) > 0)   // the most groups
    rc = dmalloc(&p->d_rpart, 2 * static_cast<size_t>(resident_pruned_groups(p, 256)) * p->nsup);
  if (rc == BCCB_OK) {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, p->device) != hipSuccess || khz <= 0) khz = 100000;
    p->wall_ticks_per_s = static_cast<long long>(khz) * 1000;
  }
  if (rc == BCCB_OK) rc = dmalloc(&p->d_red, static_cast<size_t>(kReduceBlocks) * 8);
  if (rc == BCCB_OK) rc = dmalloc(&p->d_flag, 1);
  if (rc == BCCB_OK && hipHostMalloc(reinterpret_cast<void**>(&p->h_red), kReduceBlocks * 8 * sizeof(double)) != hipSuccess)
    rc = BCCB_E_NOMEM;
  if (rc == BCCB_OK && hipHostMalloc(reinterpret_cast<void**>(&p->h_flag), sizeof(int)) != hipSuccess) rc = BCCB_E_NOMEM;
  if (rc == BCCB_OK) rc = dmalloc(&p->d_sup_ptr, p->h_sup_ptr.size());
  if (rc == BCCB_OK) rc = dmalloc(&p->d_sup, p->h_sup.size());
  if (rc == BCCB_OK) rc = dmalloc(&p->d_src_ptr, p->h_src_ptr.size());
  if (rc == BCCB_OK) rc = dmalloc(&p->d_src, p->h_src.size());
  if (rc == BCCB_OK) rc = dmalloc(&p->d_sup_rhs, p->h_sup.size());
  if (rc == BCCB_OK) rc = dmalloc(&p->d_sup_desc, 1);
  if (rc == BCCB_OK && hipHostMalloc(reinterpret_cast<void**>(&p->h_sup_desc), sizeof(SupRhsDesc)) != hipSuccess)
    rc = BCCB_E_NOMEM;
  if (rc == BCCB_OK &&
      (hipMemcpy(p->d_sup_ptr, p->h_sup_ptr.data(), p->h_sup_ptr.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
       (p->nsup && hipMemcpy(p->d_sup, p->h_sup.data(), p->h_sup.size() * sizeof(SupEntry), hipMemcpyHostToDevice) != hipSuccess) ||
       hipMemcpy(p->d_src_ptr, p->h_src_ptr.data(), p->h_src_ptr.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
       (!p->h_src.empty() && hipMemcpy(p->d_src, p->h_src.data(), p->h_src.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)))
    rc = BCCB_E_DEVICE;
  if (rc == BCCB_OK) {
    const bool ok =
        hipMemcpy(p->d_omega, p->omega32.data(), p->L * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
        hipMemcpy(p->d_sensor_of, sensor_of.data(), sensor_of.size() * sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
        hipMemcpy(p->d_sensors, sensors.data(), sensors.size() * sizeof(int2), hipMemcpyHostToDevice) == hipSuccess &&
        hipMemcpy(p->d_tw1, tw1.data(), L1 * sizeof(float2), hipMemcpyHostToDevice) == hipSuccess &&
        hipMemcpy(p->d_tw2, tw2.data(), L2 * sizeof(float2), hipMemcpyHostToDevice) == hipSuccess &&
        hipMemcpy(p->d_coef, coef, sizeof(coef), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) rc = BCCB_E_DEVICE;
  }
  if (rc != BCCB_OK) {
    plan_free(p);
    return rc;
  }
  default_config(p);
  *out = p;
  return BCCB_OK;
}

int bccb_plan_destroy(bccb_plan_t plan) {
  if (plan) {
    if (plan->stream) (void)hipStreamSynchronize(plan->stream);
    else (void)hipDeviceSynchronize();
  }
  plan_free(plan);
  return BCCB_OK;
}

int bccb_set_stream(bccb_plan_t plan, void* stream) {
  if (!plan) return BCCB_E_INVALID;
  plan->stream = static_cast<hipStream_t>(stream);
  return BCCB_OK;
}

int bccb_plan_info(bccb_plan_t plan, int* M, double* mu, float* omega_host) {
  if (!plan) return BCCB_E_INVALID;
  if (plan->emb && omega_host) return BCCB_E_UNSUPPORTED;   // see bccb_plan_embedding
  if (M) *M = plan->M;
  if (mu) *mu = plan->mu;
  if (omega_host) std::memcpy(omega_host, plan->omega32.data(), plan->L * sizeof(float));
  return BCCB_OK;
}

int bccb_stream_copy(const void* src, void* dst, size_t bytes, int variant, void* stream) {
  if (!src || !dst || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(src) % 16 != 0 ||
      reinterpret_cast<uintptr_t>(dst) % 16 != 0 || variant < 0 || variant > 63)
    return BCCB_E_INVALID;
  return kern(launch_stream_copy(src, dst, static_cast<long>(bytes / 16), variant, static_cast<hipStream_t>(stream)));
}

int bccb_plan_support_columns(bccb_plan_t plan, int* ncols, int* pruned) {
  if (!plan) return BCCB_E_INVALID;
  if (plan->emb) return BCCB_E_UNSUPPORTED;
  if (ncols) *ncols = plan->nscol;
  if (pruned) *pruned = pruned_on(plan) ? (resident_on(plan) && resident_pruned_on(plan) ? 2 : 1) : 0;
  return BCCB_OK;
}

int bccb_adjoint(bccb_plan_t p, const bccb_c32* y, bccb_c32* b) {
  if (!p || !y || !b) return BCCB_E_INVALID;
  if (p->emb) return spaced_adjoint(p, reinterpret_cast<const float2*>(y), reinterpret_cast<float2*>(b));
  BCCB_TRY(begin_call(p));
  BCCB_TRY(adjoint_into(p, reinterpret_cast<const float2*>(y), 1.f, reinterpret_cast<float2*>(b)));
  return end_call(p);
}

int bccb_adjoint_maxabs(bccb_plan_t p, const bccb_c32* y, double* maxabs) {
  if (!p || !y || !maxabs) return BCCB_E_INVALID;
  if (p->emb) return spaced_adjoint_maxabs(p, reinterpret_cast<const float2*>(y), maxabs);
  BCCB_TRY(begin_call(p));
  BCCB_TRY(adjoint_into(p, reinterpret_cast<const float2*>(y), 1.f, p->d_rhs));
  int nb = 0;
  BCCB_TRY(kern(launch_absmax(p->d_rhs, p->L, p->d_red, &nb, p->stream)));
  BCCB_HIP(hipMemcpyAsync(p->h_red, p->d_red, nb * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  const int rc = end_call(p);
  double m = 0.0;
  for (int i = 0; i < nb; ++i) m = p->h_red[i] > m ? p->h_red[i] : m;
  *maxabs = m;
  return rc;
}

int bccb_gram_apply(bccb_plan_t p, const bccb_c32* x, bccb_c32* gx) {
  if (!p || !x || !gx) return BCCB_E_INVALID;
  if (p->emb) return spaced_gram_apply(p, reinterpret_cast<const float2*>(x), reinterpret_cast<float2*>(gx));
  BCCB_TRY(begin_call(p));
  RowArgs a;
  a.xy = p->d_xy;
  a.src = reinterpret_cast<const float2*>(x);
  BCCB_TRY(row_pass(p, ROW_FWD, a));
  BCCB_TRY(col_pass(p, COL_FILTER_AFFINE, p->d_xy, p->d_coef + 1, 0.f, 1.f));
  RowArgs b;
  b.xy = p->d_xy;
  b.dst = reinterpret_cast<float2*>(gx);
  BCCB_TRY(row_pass(p, ROW_INV, b));
  return end_call(p);
}

static int check_solve(bccb_plan_t p, const bccb_c32* y, float tau, int iters, const void* out) {
  if (!p || !y || !out) return BCCB_E_INVALID;
  if (!(tau >= 0.f) || !std::isfinite(tau) || iters < 0) return BCCB_E_INVALID;
  return BCCB_OK;
}

// Pruned ISTA / FISTA (sparse support, kept columns only).  c_t lives in SlotBuf
// t mod 3; buffer 0's dense rows are the output grid, which holds c_0 at the start.
static SlotBuf pruned_buf(bccb_plan_s* p, int i, float2* out) {
  SlotBuf b;
  b.cnt = p->d_pcnt[i];
  b.sidx = p->d_psidx[i];
  b.sval = p->d_psval[i];
  b.dense = i == 0 ? out : p->d_pdense[i];
  return b;
}

// The pruned column pass's arguments over the plan's kept columns.
static ColArgs pruned_col_args(bccb_plan_s* p) {
  ColArgs c;
  c.xy = p->d_xyc;
  c.sup_ptr = p->d_sup_ptr;
  c.sup = p->d_sup;
  c.sup_rhs = p->d_sup_rhs;
  c.coef = p->d_coef;
  c.tw = p->d_tw2;
  c.L1 = p->L1;
  c.ncols = p->ncs;
  c.ldx = p->ncs;
  c.scol = p->d_scol;
  return c;
}

static int enqueue_pruned(bccb_plan_s* p, int mode, int iters, float kappa, const float2* init, float2* out) {
  hipStream_t st = p->stream;
  const bool fista = (mode == ROW_FISTA);
  if (init && init != out) BCCB_TRY(kern(launch_copy(out, init, p->L, st)));
  else if (!init) BCCB_TRY(kern(launch_fill(out, p->L, st)));
  // c_0 dense in buffer 0, c_{-1} = 0 in buffer 2
  BCCB_TRY(kern(launch_fill_int(p->d_pcnt[0], p->L2, p->L1 + 1, st)));
  BCCB_TRY(kern(launch_fill_int(p->d_pcnt[2], p->L2, 0, st)));
  RowArgs f;
  f.xy = p->d_xyc;
  f.src = out;
  f.flag = p->d_flag;
  f.colslot = p->d_colslot;
  f.ncs = p->ncs;
  BCCB_TRY(row_pass_on(p, p->cfg_rowp, ROW_PRUNED_FWD, f, st));   // kept columns of DFT_rows(z_1 = c_0)
  if (iters == 0) return BCCB_OK;
  const unsigned long long key[8] = {static_cast<unsigned long long>(mode), static_cast<unsigned long long>(iters),
                                     reinterpret_cast<unsigned long long>(out), fbits(kappa), 1, 0, 1, 2};
  BCCB_TRY(run_loop(p, key, [&](hipStream_t s) -> int {
    double alpha = 1.0;
    float beta_prev = 0.f;
    const ColArgs c = pruned_col_args(p);
    for (int t = 1; t <= iters; ++t) {
      BCCB_TRY(kern(launch_col(p->L2, p->cfg_colp, COL_PRUNED_AFFINE, c, s)));
      const double alpha_next = (1.0 + std::sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0;
      const float beta = fista ? static_cast<float>((alpha - 1.0) / alpha_next) : 0.f;
      alpha = alpha_next;
      RowArgs a;
      a.xy = p->d_xyc;
      a.colslot = p->d_colslot;
      a.ncs = p->ncs;
      a.b1 = pruned_buf(p, (t - 1) % 3, out);
      if (fista) a.b2 = pruned_buf(p, (t + 1) % 3, out);   // (t - 2) mod 3
      a.b0 = pruned_buf(p, t % 3, out);
      a.out_c = out;
      a.kappa = kappa;
      a.beta = beta;
      a.beta_prev = beta_prev;
      a.last = (t == iters);
      beta_prev = beta;
      BCCB_TRY(row_pass_on(p, p->cfg_rowp, ROW_PRUNED, a, s));
    }
    return BCCB_OK;
  }));
  return BCCB_OK;
}

// Pruned ADMM passes (sparse support, kept columns only; iters >= 1).  The scaled
// dual is split as v_t = u_t + IDFT2(Psi_t) with u_t = z_{t-1} - z_t and Psi on
// the support bins (eqs. (13)-(15) rearranged, so that x is never formed by
// cancelling the large support part of v; the cooperative form does the same):
// the column pass turns Y = DFT2(z_t - u_t) at the bins into V' and Psi_{t+1} =
// Psi_t + V', and the pruned row pass with beta_prev = 0 and beta = 1 gives
// z_{t+1} = S_{tau/rho}(z_t + IDFT2(Psi_{t+1})) and the next DFT_rows of
// 2 z_{t+1} - z_t.  z_t lives in SlotBuf t mod 3 (buffer 0's dense rows in the
// scratch grid, so the outputs alias no state); x_T = 2 z_{T-1} - z_{T-2} +
// IDFT2(V'_T) is one more column and row pass (beta_prev = 1, kappa = 0).
static int enqueue_pruned_admm(bccb_plan_s* p, int iters, float kappa, float rho, float2* zo, float2* co) {
  hipStream_t st = p->stream;
  auto buf = [&](int i) { return pruned_buf(p, i, p->d_tmp); };
  // z_0 = z_{-1} = 0 (empty rows), Psi_0 = 0, DFT_rows(z_0 - u_0) = 0
  BCCB_TRY(kern(launch_fill_int(p->d_pcnt[0], p->L2, 0, st)));
  BCCB_TRY(kern(launch_fill_int(p->d_pcnt[2], p->L2, 0, st)));
  BCCB_TRY(kern(launch_fill(p->d_psi, p->nsup, st)));
  RowArgs f;
  f.xy = p->d_xyc;
  f.src = nullptr;
  f.flag = p->d_flag;
  f.colslot = p->d_colslot;
  f.ncs = p->ncs;
  BCCB_TRY(row_pass_on(p, p->cfg_rowp, ROW_PRUNED_FWD, f, st));
  ColArgs c = pruned_col_args(p);
  c.psi = p->d_psi;
  c.vlast = p->d_vlast;
  c.rho = rho;
  c.scale = static_cast<float>(1.0 / static_cast<double>(p->L));
  const unsigned long long key[8] = {static_cast<unsigned long long>(ROW_ADMM), static_cast<unsigned long long>(iters),
                                     reinterpret_cast<unsigned long long>(zo), fbits(kappa),
                                     reinterpret_cast<unsigned long long>(co), fbits(rho), 1, 4};
  return run_loop(p, key, [&](hipStream_t s) -> int {
    for (int t = 1; t <= iters; ++t) {
      BCCB_TRY(kern(launch_col(p->L2, p->cfg_colp, COL_PRUNED_ADMM, c, s)));
      RowArgs a;
      a.xy = p->d_xyc;
      a.colslot = p->d_colslot;
      a.ncs = p->ncs;
      a.b1 = buf((t - 1) % 3);
      a.b0 = buf(t % 3);
      a.out_c = zo;
      a.kappa = kappa;
      a.beta = 1.f;
      a.beta_prev = 0.f;
      a.last = (t == iters);
      BCCB_TRY(row_pass_on(p, p->cfg_rowp, ROW_PRUNED, a, s));
    }
    if (co) {
      BCCB_TRY(kern(launch_col(p->L2, p->cfg_colp, COL_PRUNED_EXPAND, c, s)));
      RowArgs a;
      a.xy = p->d_xyc;
      a.colslot = p->d_colslot;
      a.ncs = p->ncs;
      a.b1 = buf((iters - 1) % 3);
      a.b2 = buf((iters + 1) % 3);   // (iters - 2) mod 3
      a.b0 = buf(iters % 3);
      a.out_c = co;
      a.kappa = 0.f;
      a.beta = 0.f;
      a.beta_prev = 1.f;
      a.last = true;
      BCCB_TRY(row_pass_on(p, p->cfg_rowp, ROW_PRUNED, a, s));
    }
    return BCCB_OK;
  });
}

// The iterations of an ISTA (mode ROW_ISTA) or FISTA (ROW_FISTA) solve with
// kappa = mu tau, the right-hand side already in place: the cooperative solver,
// the pruned passes or the full passes, as the plan's configuration selects.
static int enqueue_prox_grad(bccb_plan_s* p, int mode, int iters, float kappa, const float2* init, float2* out) {
  const bool sparse = sparse_on(p);
  if (resident_on(p) && iters > 0)
    return resident_enqueue(p, mode == ROW_FISTA ? RES_FISTA : RES_ISTA, iters, kappa, 0.f, 1.f, init, out, nullptr,
                            p->stream);
  if (pruned_on(p)) return enqueue_pruned(p, mode, iters, kappa, init, out);
  // z^(1) = c^(0): its row DFT starts the first column pass; FISTA keeps c^(t-1) in c_out
  RowArgs f;
  f.xy = p->d_xy;
  f.src = init;
  f.flag = p->d_flag;
  BCCB_TRY(row_pass(p, ROW_FWD, f));
  if (mode == ROW_FISTA || iters == 0) {
    if (init && init != out) BCCB_TRY(kern(launch_copy(out, init, p->L, p->stream)));
    else if (!init) BCCB_TRY(kern(launch_fill(out, p->L, p->stream)));
  }
  // FISTA with the iterate in per-row slots: c^(0) is read densely (all counts "dense")
  const int rmode = (mode == ROW_FISTA && p->sparse_iterate) ? ROW_FISTA_SP : mode;
  if (rmode == ROW_FISTA_SP) BCCB_TRY(kern(launch_fill_int(p->d_cnt, p->L2, p->L1 + 1, p->stream)));
  if (iters > 0) {
    const unsigned long long key[8] = {static_cast<unsigned long long>(rmode), static_cast<unsigned long long>(iters),
                                       reinterpret_cast<unsigned long long>(out), fbits(kappa), 0, 0,
                                       sparse ? 1ull : 0ull, 1};
    BCCB_TRY(run_loop(p, key, [&](hipStream_t s) -> int {
      double alpha = 1.0;
      for (int t = 1; t <= iters; ++t) {
        BCCB_TRY(col_pass_on(p, p->cfg_col, sparse ? COL_SPARSE_AFFINE : COL_FILTER_AFFINE, p->d_xy, p->d_coef,
                             0.f, 1.f, s));
        const double alpha_next = (1.0 + std::sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0;
        RowArgs a;
        a.xy = p->d_xy;
        a.rhs = sparse ? nullptr : p->d_rhs;
        a.state = out;
        a.out_c = out;
        a.cnt = p->d_cnt;
        a.sidx = p->d_sidx;
        a.sval = p->d_sval;
        a.kappa = kappa;
        a.beta = static_cast<float>((alpha - 1.0) / alpha_next);
        a.last = (t == iters);
        alpha = alpha_next;
        BCCB_TRY(row_pass_on(p, p->cfg_row, rmode, a, s));
      }
      return BCCB_OK;
    }));
  }
  return BCCB_OK;
}


// ISTA (mode ROW_ISTA) and FISTA (ROW_FISTA) share one driver.
static int solve_prox_grad(bccb_plan_t p, int mode, const bccb_c32* y, float tau, int iters, const bccb_c32* c0,
                           bccb_c32* c_out) {
  BCCB_TRY(check_solve(p, y, tau, iters, c_out));
  if (p->emb)
    return spaced_prox_grad(p, mode, reinterpret_cast<const float2*>(y), tau, iters, reinterpret_cast<const float2*>(c0),
                            reinterpret_cast<float2*>(c_out));
  float2* out = reinterpret_cast<float2*>(c_out);
  const float2* init = reinterpret_cast<const float2*>(c0);
  BCCB_TRY(begin_call(p));
  const bool sparse = sparse_on(p);
  // mu * D_s^H y: on the support bins of the spectrum (sparse) or as a grid
  if (sparse) BCCB_TRY(fill_sup_rhs(p, reinterpret_cast<const float2*>(y), static_cast<float>(p->mu)));
  else BCCB_TRY(adjoint_into(p, reinterpret_cast<const float2*>(y), static_cast<float>(p->mu), p->d_rhs));
  BCCB_TRY(enqueue_prox_grad(p, mode, iters, static_cast<float>(p->mu * tau), init, out));
  return end_call(p);
}

int lasso_solve_ista(bccb_plan_t p, const bccb_c32* y, float tau, int iters, const bccb_c32* c0, bccb_c32* c_out) {
  return solve_prox_grad(p, ROW_ISTA, y, tau, iters, c0, c_out);
}

int lasso_solve_fista(bccb_plan_t p, const bccb_c32* y, float tau, int iters, const bccb_c32* c0, bccb_c32* c_out) {
  return solve_prox_grad(p, ROW_FISTA, y, tau, iters, c0, c_out);
}

int lasso_solve_admm(bccb_plan_t p, const bccb_c32* y, float tau, float rho, int iters, bccb_c32* z_out,
                     bccb_c32* c_out) {
  BCCB_TRY(check_solve(p, y, tau, iters, z_out));
  if (!(rho > 0.f) || !std::isfinite(rho)) return BCCB_E_INVALID;
  if (p->emb)
    return spaced_admm(p, reinterpret_cast<const float2*>(y), tau, rho, iters, reinterpret_cast<float2*>(z_out),
                       reinterpret_cast<float2*>(c_out));
  float2* zo = reinterpret_cast<float2*>(z_out);
  float2* co = reinterpret_cast<float2*>(c_out);
  BCCB_TRY(begin_call(p));
  const bool sparse = sparse_on(p);
  // w = (G + rho I)^-1 D_s^H y: the scattered snapshot S is already spectral, so
  // w = IDFT2(S / (Omega + rho)) (unnormalised, since DFT2(b) = L S).  With the
  // sparse support S / (Omega + rho) is added in every column pass instead.
  if (sparse) {
    BCCB_TRY(fill_sup_rhs(p, reinterpret_cast<const float2*>(y), 1.f));
  } else {
    BCCB_TRY(kern(launch_scatter(reinterpret_cast<const float2*>(y), p->d_sensor_of, p->M1, p->M2, p->L1, p->L2, 1.f,
                                 p->d_tmp, p->d_flag, p->stream)));
    BCCB_TRY(col_pass(p, COL_MULINV_ADMM, p->d_tmp, nullptr, rho, 1.f));
    RowArgs a;
    a.xy = p->d_tmp;
    a.dst = p->d_rhs;
    BCCB_TRY(row_pass(p, ROW_INV, a));
  }
  if (sparse && resident_on(p) && iters > 0) {
    BCCB_TRY(resident_enqueue(p, RES_ADMM, iters, tau / rho, rho,
                              static_cast<float>(static_cast<double>(rho) / static_cast<double>(p->L)), nullptr, co, zo,
                              p->stream));
    return end_call(p);
  }
  if (sparse && pruned_on(p) && iters > 0) {
    BCCB_TRY(enqueue_pruned_admm(p, iters, tau / rho, rho, zo, co));
    return end_call(p);
  }
  BCCB_TRY(kern(launch_fill(p->d_state, p->L, p->stream)));  // v^(0) = 0
  BCCB_TRY(kern(launch_fill(p->d_xy, p->L, p->stream)));     // DFT_rows(z^(0) - v^(0)) = 0
  if (iters == 0) {
    BCCB_TRY(kern(launch_fill(zo, p->L, p->stream)));
    if (co) BCCB_TRY(kern(launch_fill(co, p->L, p->stream)));
  }
  const float scale = static_cast<float>(static_cast<double>(rho) / static_cast<double>(p->L));
  const float kappa = tau / rho;
  if (iters > 0) {
    const unsigned long long key[8] = {static_cast<unsigned long long>(ROW_ADMM), static_cast<unsigned long long>(iters),
                                       reinterpret_cast<unsigned long long>(zo), fbits(kappa),
                                       reinterpret_cast<unsigned long long>(co), fbits(rho), fbits(scale),
                                       sparse ? 3ull : 1ull};
    BCCB_TRY(run_loop(p, key, [&](hipStream_t s) -> int {
      for (int t = 1; t <= iters; ++t) {
        BCCB_TRY(col_pass_on(p, p->cfg_col, sparse ? COL_SPARSE_ADMM : COL_FILTER_ADMM, p->d_xy, nullptr, rho, scale,
                             s));
        RowArgs a;
        a.xy = p->d_xy;
        a.rhs = sparse ? nullptr : p->d_rhs;
        a.state = p->d_state;
        a.out_z = zo;
        a.out_c = co;
        a.kappa = kappa;
        a.last = (t == iters);
        BCCB_TRY(row_pass_on(p, p->cfg_row, ROW_ADMM, a, s));
      }
      return BCCB_OK;
    }));
  }
  return end_call(p);
}

int bccb_objective_kkt(bccb_plan_t p, const bccb_c32* y, float tau, const bccb_c32* c, double* objective,
                       double* r_kkt, double* max_e_over_tau) {
  if (!p || !y || !c) return BCCB_E_INVALID;
  if (!(tau >= 0.f) || !std::isfinite(tau)) return BCCB_E_INVALID;
  if (p->emb)
    return spaced_objective_kkt(p, reinterpret_cast<const float2*>(y), tau, reinterpret_cast<const float2*>(c),
                                objective, r_kkt, max_e_over_tau);
  const float2* cc = reinterpret_cast<const float2*>(c);
  BCCB_TRY(begin_call(p));
  // spec = DFT2(c); D_s c = (-1)^(m1+m2) spec at the kept elements' bins
  RowArgs f;
  f.xy = p->d_xy;
  f.src = cc;
  f.flag = p->d_flag;
  BCCB_TRY(row_pass(p, ROW_FWD, f));
  BCCB_TRY(col_pass(p, COL_FWD, p->d_xy, nullptr, 0.f, 1.f));
  int nb_r = 0, nb_k = 0;
  double* part_r = p->d_red;
  double* part_k = p->d_red + kReduceBlocks;
  BCCB_TRY(kern(launch_resid(p->d_xy, reinterpret_cast<const float2*>(y), p->d_sensors, p->M, p->L1, p->L2, part_r,
                             &nb_r, p->stream)));
  // G c = IDFT2(Omega/L . spec)
  BCCB_TRY(col_pass(p, COL_MULINV_AFFINE, p->d_xy, p->d_coef + 1, 0.f, 1.f));
  {
    RowArgs a;
    a.xy = p->d_xy;
    a.dst = p->d_state;
    BCCB_TRY(row_pass(p, ROW_INV, a));
  }
  BCCB_TRY(adjoint_into(p, reinterpret_cast<const float2*>(y), 1.f, p->d_rhs));
  BCCB_TRY(kern(launch_kkt(cc, p->d_rhs, p->d_state, tau, p->L, part_k, &nb_k, p->stream)));
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
  if (objective) *objective = 0.5 * rs + static_cast<double>(tau) * l1;
  if (r_kkt) *r_kkt = b2 > 0.0 ? std::sqrt(e2) / std::sqrt(b2) : std::sqrt(e2);
  if (max_e_over_tau) *max_e_over_tau = tau > 0.f ? emax / tau : emax;
  return rc;
}

int bccb_kkt(bccb_plan_t p, const bccb_c32* y, float tau, const bccb_c32* c, double* r_kkt, double* obj) {
  return bccb_objective_kkt(p, y, tau, c, obj, r_kkt, nullptr);
}

int bccb_plan_omega_device(bccb_plan_t p, float* omega_dev) {
  if (!p || !omega_dev) return BCCB_E_INVALID;
  if (p->emb) return BCCB_E_UNSUPPORTED;
  BCCB_HIP(hipMemcpyAsync(omega_dev, p->d_omega, p->L * sizeof(float), hipMemcpyDeviceToDevice, p->stream));
  BCCB_HIP(hipStreamSynchronize(p->stream));
  return BCCB_OK;
}

int bccb_plan_get_config(bccb_plan_t p, bccb_config* cfg) {
  if (!p || !cfg) return BCCB_E_INVALID;
  cfg->row_elems = p->cfg_row.E;
  cfg->row_rows_per_block = p->cfg_row.rpb;
  cfg->col_elems = p->cfg_col.E;
  cfg->col_cols_per_block = p->cfg_col.W;
  cfg->use_graph = p->use_graph;
  cfg->spectral_support = p->use_support;
  cfg->row_spread = p->cfg_row.spread;
  cfg->col_spread = p->cfg_col.spread;
  cfg->sparse_iterate = p->sparse_iterate;
  cfg->support_columns = p->use_prune;
  cfg->prow_elems = p->cfg_rowp.E;
  cfg->prow_rows_per_block = p->cfg_rowp.rpb;
  cfg->pcol_elems = p->cfg_colp.E;
  cfg->pcol_cols_per_block = p->cfg_colp.W;
  cfg->resident_groups = p->resident_groups;
  cfg->resident_spread = p->resident_spread;
  cfg->resident_block = p->resident_block;
  return BCCB_OK;
}

int bccb_plan_set_config(bccb_plan_t p, const bccb_config* cfg) {
  if (!p || !cfg) return BCCB_E_INVALID;
  // padded-embedding plans run the full passes only: their shapes can be set, the other forms not
  if (p->emb && (cfg->sparse_iterate || cfg->resident_groups)) return BCCB_E_UNSUPPORTED;
  PassCfg r, c;
  r.E = cfg->row_elems;
  r.rpb = cfg->row_rows_per_block;
  r.spread = cfg->row_spread;
  c.E = cfg->col_elems;
  c.W = cfg->col_cols_per_block;
  c.spread = cfg->col_spread;
  auto spread_ok = [](int v) { return v == 1 || v == 2 || v == 4 || v == 8; };
  const bool spi = cfg->sparse_iterate != 0;
  if (!row_shape_ok(p->L1, r, spi) || !col_shape_ok(p->L1, p->L2, c) || !spread_ok(r.spread) || !spread_ok(c.spread) ||
      (spi && p->L1 < 8))
    return BCCB_E_INVALID;
  if (!(cfg->resident_block == 0 || cfg->resident_block == 256 || cfg->resident_block == 512)) return BCCB_E_INVALID;
  if (cfg->resident_groups < 0 || (cfg->resident_groups > 0 && (!p->has_support ||
                                     !resident_shape_ok(p, cfg->resident_groups, cfg->resident_spread))))
    return BCCB_E_INVALID;
  PassCfg rp = p->cfg_rowp, cp = p->cfg_colp;
  if (p->prune_ok) {
    rp.E = cfg->prow_elems;
    rp.rpb = cfg->prow_rows_per_block;
    rp.spread = r.spread;
    cp.E = cfg->pcol_elems;
    cp.W = cfg->pcol_cols_per_block;
    cp.spread = c.spread;
    if (!rowp_shape_ok(p->L1, rp, p->ncs) || !colp_shape_ok(p->ncs, p->L2, cp)) return BCCB_E_INVALID;
  }
  p->cfg_rowp = rp;
  p->cfg_colp = cp;
  p->use_prune = cfg->support_columns ? 1 : 0;
  p->cfg_row = r;
  p->cfg_col = c;
  p->use_graph = cfg->use_graph ? 1 : 0;
  p->use_support = cfg->spectral_support ? 1 : 0;
  p->sparse_iterate = spi ? 1 : 0;
  p->resident_groups = cfg->resident_groups;
  p->resident_spread = cfg->resident_groups > 0 ? cfg->resident_spread : 1;
  p->resident_block = cfg->resident_block == 512 ? 512 : 256;
  drop_graph(p);
  return BCCB_OK;
}

// Arguments of the pruned passes over the plan's own buffers (autotuning, profiling):
// c_{t-1}, c_{t-2} from buffers 1 and 2, c_t into buffer 0's private grid.
static RowArgs pruned_work_args(bccb_plan_s* p) {
  RowArgs a;
  a.xy = p->d_xyc;
  a.colslot = p->d_colslot;
  a.ncs = p->ncs;
  a.b1 = pruned_buf(p, 1, nullptr);
  a.b2 = pruned_buf(p, 2, nullptr);
  a.b0 = pruned_buf(p, 0, nullptr);
  a.b0.dense = p->d_pdense[0];
  a.out_c = p->d_tmp;
  a.kappa = 1.f;
  a.beta = 0.5f;
  a.beta_prev = 0.5f;
  return a;
}

int bccb_plan_autotune(bccb_plan_t p, int reps, bccb_config* chosen) {
  if (!p || reps < 1) return BCCB_E_INVALID;   // padded-embedding plans: the full passes' shapes only
  hipStream_t st = p->stream;
  RowArgs a;
  a.xy = p->d_xy;
  a.rhs = sparse_on(p) ? nullptr : p->d_rhs;
  a.state = p->d_state;
  a.cnt = p->d_cnt;
  a.sidx = p->d_sidx;
  a.sval = p->d_sval;
  a.kappa = 1.f;
  a.beta = 0.5f;
  const bool spi = p->sparse_iterate != 0;
  const int rmode = spi ? ROW_FISTA_SP : ROW_FISTA;
  const int cmode = sparse_on(p) ? COL_SPARSE_AFFINE : COL_FILTER_AFFINE;
  const bool pr = p->prune_ok;
  const RowArgs ap = pr ? pruned_work_args(p) : RowArgs();
  const ColArgs cp = pr ? pruned_col_args(p) : ColArgs();
  float best[4] = {1e30f, 1e30f, 1e30f, 1e30f};   // row, col, pruned row, pruned col
  PassCfg br = p->cfg_row, bc = p->cfg_col, brp = p->cfg_rowp, bcp = p->cfg_colp;
  auto consider = [&](float ms, int slot, PassCfg& keep, const PassCfg& cand) -> int {
    if (ms < 0.f) return BCCB_E_DEVICE;
    if (ms < best[slot]) {
      best[slot] = ms;
      keep = cand;
    }
    return BCCB_OK;
  };
  const int Es[4] = {4, 8, 16, 32};
  for (int cand = 0; cand < 8; ++cand) {
    const int spread = cand < 4 ? 1 : 8;
    for (int k = 1; k <= 256; k *= 2) {
      PassCfg r;
      r.E = Es[cand % 4];
      r.rpb = k;
      r.spread = spread;
      if (row_shape_ok(p->L1, r, spi))
        BCCB_TRY(consider(time_launches(st, reps, [&] { return row_pass_on(p, r, rmode, a, st); }), 0, br, r));
      if (pr && rowp_shape_ok(p->L1, r, p->ncs))
        BCCB_TRY(consider(time_launches(st, reps, [&] { return row_pass_on(p, r, ROW_PRUNED, ap, st); }), 2, brp, r));
      PassCfg c;
      c.E = Es[cand % 4];
      c.W = k;
      c.spread = spread;
      if (col_shape_ok(p->L1, p->L2, c))
        BCCB_TRY(consider(time_launches(st, reps, [&] { return col_pass_on(p, c, cmode, p->d_xy, p->d_coef, 0.f, 1.f, st); }),
                          1, bc, c));
      if (pr && colp_shape_ok(p->ncs, p->L2, c))
        BCCB_TRY(consider(time_launches(st, reps, [&] { return kern(launch_col(p->L2, c, COL_PRUNED_AFFINE, cp, st)); }),
                          3, bcp, c));
    }
  }
  p->cfg_row = br;
  p->cfg_col = bc;
  p->cfg_rowp = brp;
  p->cfg_colp = bcp;
  // ISTA / FISTA take whichever pair of passes is faster per iteration
  if (pr && p->use_support) p->use_prune = (best[2] + best[3] < best[0] + best[1]) ? 1 : 0;
  // the cooperative solver (every launchable group count and spread) against
  // those passes, each timed as a FISTA solve of kIt iterations enqueues it
  // (the passes replayed from their captured graph when use_graph is set)
  if (p->has_support && p->use_support) {
    constexpr int kIt = 200;
    const int n = reps / 10 > 1 ? reps / 10 : 1;
    auto solve_ms = [&]() {
      return time_launches(st, n, [&] { return enqueue_prox_grad(p, ROW_FISTA, kIt, 1.f, nullptr, p->d_tmp); });
    };
    const int pass_prune = p->use_prune;
    auto restore = [&]() {
      p->resident_groups = 0;
      p->resident_spread = 1;
      p->resident_block = 256;
      p->use_prune = pass_prune;
    };
    restore();
    float best_ms = solve_ms();
    if (best_ms < 0.f) return BCCB_E_DEVICE;
    int bg = 0, bs = 1, bb = 256, bprune = pass_prune;
    // per spread: the fastest full cooperative group count (ADMM runs that form)
    float full_ms[9];
    int full_g[9];
    for (int i = 0; i < 9; ++i) {
      full_ms[i] = 1e30f;
      full_g[i] = 0;
    }
    bool pruned_done[9][2] = {};
    for (int G = 1; G <= kResidentMaxGroups; G *= 2) {
      for (int sp = 1; sp <= 8; sp *= 8) {
        if (!resident_shape_ok(p, G, sp)) continue;
        // candidates: the full form (pz 0), the pruned form with 256- and 512-thread groups
        for (int cand = 0; cand < (pr ? 3 : 1); ++cand) {
          const int pz = cand > 0 ? 1 : 0;
          const int blk = cand == 2 ? 512 : 256;
          if (pz == 1 && pruned_done[sp][cand - 1]) continue;   // the pruned form's groups do not depend on G
          p->resident_groups = G;
          p->resident_spread = sp;
          p->resident_block = blk;
          p->use_prune = pz;
          if (pz == 1) {
            pruned_done[sp][cand - 1] = true;
            if (!resident_pruned_on(p)) {
              restore();
              continue;
            }
          }
          const float ms = solve_ms();
          restore();
          if (ms < 0.f) return BCCB_E_DEVICE;
          if (pz == 0 && ms < full_ms[sp]) {
            full_ms[sp] = ms;
            full_g[sp] = G;
          }
          if (ms < best_ms) {
            best_ms = ms;
            bg = G;
            bs = sp;
            bb = blk;
            bprune = pz;
          }
        }
      }
    }
    p->resident_groups = bg > 0 ? (full_g[bs] > 0 ? full_g[bs] : bg) : 0;
    p->resident_spread = bg > 0 ? bs : 1;
    p->resident_block = bb;
    p->use_prune = bprune;
  }
  drop_graph(p);
  if (chosen) return bccb_plan_get_config(p, chosen);
  return BCCB_OK;
}

int bccb_profile_resident(bccb_plan_t p, int solver, int iters, int reps, double* ms) {
  if (!p || reps < 1 || iters < 1 || solver < 0 || solver > 2 || !ms) return BCCB_E_INVALID;
  if (p->emb || !resident_on(p)) return BCCB_E_UNSUPPORTED;
  const int mode = solver == 0 ? RES_ISTA : (solver == 1 ? RES_FISTA : RES_ADMM);
  const float scale = static_cast<float>(1.0 / static_cast<double>(p->L));
  const float m = time_launches(p->stream, reps, [&] {
    return mode == RES_ADMM ? resident_enqueue(p, mode, iters, 1.f, 1.f, scale, nullptr, nullptr, p->d_tmp, p->stream)
                            : resident_enqueue(p, mode, iters, 1.f, 0.f, 1.f, nullptr, p->d_tmp, nullptr, p->stream);
  });
  if (m < 0.f) return BCCB_E_DEVICE;
  *ms = m;
  return BCCB_OK;
}

int bccb_profile_passes(bccb_plan_t p, int solver, int reps, double* col_ms, double* row_ms) {
  if (!p || reps < 1 || solver < 0 || solver > 2 || !col_ms || !row_ms) return BCCB_E_INVALID;
  if (p->emb) return BCCB_E_UNSUPPORTED;
  hipEvent_t e0, e1, e2;
  BCCB_HIP(hipEventCreate(&e0));
  BCCB_HIP(hipEventCreate(&e1));
  BCCB_HIP(hipEventCreate(&e2));
  int rc = BCCB_OK;
  RowArgs a;
  a.xy = p->d_xy;
  a.rhs = p->d_rhs;
  a.state = p->d_state;
  a.out_z = p->d_tmp;
  a.out_c = p->d_tmp;
  a.cnt = p->d_cnt;
  a.sidx = p->d_sidx;
  a.sval = p->d_sval;
  a.kappa = 1.f;
  a.beta = 0.5f;
  const int row_mode = solver == 0 ? ROW_ISTA
                                   : (solver == 1 ? (p->sparse_iterate ? ROW_FISTA_SP : ROW_FISTA) : ROW_ADMM);
  const bool sparse = sparse_on(p);
  const int col_mode = solver == 2 ? (sparse ? COL_SPARSE_ADMM : COL_FILTER_ADMM)
                                   : (sparse ? COL_SPARSE_AFFINE : COL_FILTER_AFFINE);
  if (sparse) a.rhs = nullptr;
  const float scale = static_cast<float>(1.0 / static_cast<double>(p->L));
  // a plan whose solves take the pruned passes: time those (ADMM: beta = 1, the
  // column pass updating the support part of the dual)
  const bool pr = pruned_on(p);
  RowArgs ap = pr ? pruned_work_args(p) : RowArgs();
  if (pr && solver != 1) {
    ap.b2 = SlotBuf();
    ap.beta = solver == 2 ? 1.f : 0.f;
    ap.beta_prev = 0.f;
  }
  ColArgs cp = pr ? pruned_col_args(p) : ColArgs();
  if (pr && solver == 2) {
    cp.psi = p->d_psi;
    cp.vlast = p->d_vlast;
    cp.rho = 1.f;
    cp.scale = scale;
  }
  const int pcol_mode = solver == 2 ? COL_PRUNED_ADMM : COL_PRUNED_AFFINE;
  if (hipEventRecord(e0, p->stream) != hipSuccess) rc = BCCB_E_DEVICE;
  for (int i = 0; i < reps && rc == BCCB_OK; ++i)
    rc = pr ? kern(launch_col(p->L2, p->cfg_colp, pcol_mode, cp, p->stream))
            : col_pass(p, col_mode, p->d_xy, p->d_coef, 1.f, scale);
  if (rc == BCCB_OK && hipEventRecord(e1, p->stream) != hipSuccess) rc = BCCB_E_DEVICE;
  for (int i = 0; i < reps && rc == BCCB_OK; ++i)
    rc = pr ? row_pass_on(p, p->cfg_rowp, ROW_PRUNED, ap, p->stream) : row_pass(p, row_mode, a);
  if (rc == BCCB_OK && hipEventRecord(e2, p->stream) != hipSuccess) rc = BCCB_E_DEVICE;
  if (rc == BCCB_OK && hipEventSynchronize(e2) != hipSuccess) rc = BCCB_E_DEVICE;
  float m01 = 0.f, m12 = 0.f;
  if (rc == BCCB_OK && (hipEventElapsedTime(&m01, e0, e1) != hipSuccess ||
                        hipEventElapsedTime(&m12, e1, e2) != hipSuccess))
    rc = BCCB_E_DEVICE;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e2);
  *col_ms = m01 / reps;
  *row_ms = m12 / reps;
  return rc;
}

}  // extern "C"
