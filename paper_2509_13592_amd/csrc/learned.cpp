// Learned unrolled FISTA (forward, backward, Adam) and the KKT-gated solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "batch_resident.h"
#include "bccb.h"
#include "kernels.h"
#include "lista.h"
#include "plan_internal.h"

using namespace bccb;

struct bccb_lista_s {
  bccb_plan_t plan = nullptr;
  int K = 0, cap = 0, train = 0, L1 = 0, L2 = 0;
  long L = 0;
  hipStream_t stream = nullptr;
  std::vector<double> beta;        // FISTA momentum weights of the layers
  double alpha_end = 1.0;          // FISTA alpha after the layers (continuation of the schedule)
  PassCfg rcfg, ccfg;              // forward / FISTA pass shapes
  int bwdE = 16, bwd_rpb = 1, bwd_W = 1, groups = 16;

  float2 *d_b = nullptr, *d_c = nullptr, *d_xy = nullptr, *d_A = nullptr, *d_Z = nullptr;
  float2* d_cprev = nullptr;                    // c_{K-2} of the last forward (momentum continuation)
  float2* d_ring[2] = {nullptr, nullptr};
  float2 *d_U = nullptr, *d_C = nullptr;        // [K][cap][L] (training)
  float2 *d_mulc = nullptr, *d_omp = nullptr;   // [K][L]
  float* d_dscal = nullptr;                     // [K][2]
  float* d_tau = nullptr;                       // [cap]
  float2 *d_coef_fista = nullptr, *d_coef_gram = nullptr;  // [cap]
  double* d_rows = nullptr;                     // [cap * L2 * 2]
  float2 *d_gm_part = nullptr, *d_gm = nullptr; // [groups][L], [L]
  double* d_lg = nullptr;                       // [27][2]
  double *d_sum_part = nullptr, *d_sums = nullptr, *d_sums2 = nullptr, *d_bnorm = nullptr;  // per scene
  double* d_rk = nullptr;                       // [cap] sum e^2 per scene
  SceneDesc* d_desc = nullptr;
  SceneDesc* h_desc = nullptr;
  int* d_map = nullptr;
  int* h_map = nullptr;
  float* h_tau = nullptr;
  double* h_tmp = nullptr;
  int* d_flag = nullptr;
  int* h_flag = nullptr;
  int batch = 0;                                // batch of the last training forward
  bool have_acts = false;
  // spectral right-hand sides of the fallback FISTA on the plan's support bins
  float2* d_sup_rhs = nullptr;                  // [cap][nsup]
  SupRhsDesc* d_sdesc = nullptr;                // [cap]
  SupRhsDesc* h_sdesc = nullptr;                // pinned [cap]
  // pruned fallback (the plan has a kept-column set): kept row spectra [cap][L2][ncs],
  // c_t over three SlotBufs whose dense grids are d_R0, d_xy and d_cprev
  bool prune = false;
  bool kkt_pruned = false;                      // the current solve checks KKT on the kept columns
  float2* d_xyc = nullptr;
  float2* d_xyck = nullptr;                     // kept spectra of the KKT checks [cap][L2][ncs]
  float2* d_R0 = nullptr;
  int* d_pcnt[3] = {nullptr, nullptr, nullptr};
  unsigned short* d_psidx[3] = {nullptr, nullptr, nullptr};
  float2* d_psval[3] = {nullptr, nullptr, nullptr};
  PassCfg rcfgp, ccfgp;
  // pruned learned layers: Omega'_k = Omega + Delta_k (*) Omega lives on the 5x5 dilation of
  // Omega's support; its spectral columns (ncsd, padded), per-column entries and kept spectra
  bool prune_layers = false;
  int ncsd = 0;
  int* d_dscol = nullptr;
  int* d_dcolslot = nullptr;
  int* d_dsup_ptr = nullptr;
  DilEntry* d_dil = nullptr;
  float2* d_xycd = nullptr;                     // [cap][L2][ncsd]
  PassCfg rcfgd, ccfgd;
  // the fallback's iterations as chunks of the persistent whole-solve launch (batch_resident.h):
  // each check interval of the active scenes is one launch carrying the state in d_xyc and
  // the slot buffers' counts
  bool res_ok = false, res_on = false;
  ResidentClass* d_rcls = nullptr;
  int res_threads = 0, res_blocks = 0;
  size_t res_lds = 0;
  int* d_queue = nullptr;
  float* d_rbeta = nullptr;                     // [rbeta_cap] momentum weights of the fallback
  float* h_rbeta = nullptr;                     // pinned
  int rbeta_cap = 0;
};

namespace {

template <typename T>
int dalloc(T** p, size_t n) {
  if (hipMalloc(reinterpret_cast<void**>(p), (n ? n : 1) * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return BCCB_E_NOMEM;
  }
  return BCCB_OK;
}

void lista_free(bccb_lista_s* n) {
  if (!n) return;
  void* ptrs[] = {n->d_b, n->d_c, n->d_cprev, n->d_xy, n->d_A, n->d_Z, n->d_ring[0], n->d_ring[1], n->d_U, n->d_C,
                  n->d_mulc, n->d_omp, n->d_dscal, n->d_tau, n->d_coef_fista, n->d_coef_gram, n->d_rows,
                  n->d_gm_part, n->d_gm, n->d_lg, n->d_sum_part, n->d_sums, n->d_sums2, n->d_bnorm, n->d_rk,
                  n->d_desc, n->d_map, n->d_flag, n->d_sup_rhs, n->d_sdesc};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (void* p : {static_cast<void*>(n->d_rcls), static_cast<void*>(n->d_queue), static_cast<void*>(n->d_rbeta)})
    if (p) (void)hipFree(p);
  if (n->h_rbeta) (void)hipHostFree(n->h_rbeta);
  for (void* p : {static_cast<void*>(n->d_xyc), static_cast<void*>(n->d_R0), static_cast<void*>(n->d_xyck),
                  static_cast<void*>(n->d_dscol), static_cast<void*>(n->d_dcolslot), static_cast<void*>(n->d_dsup_ptr),
                  static_cast<void*>(n->d_dil), static_cast<void*>(n->d_xycd)})
    if (p) (void)hipFree(p);
  for (int i = 0; i < 3; ++i)
    for (void* p : {static_cast<void*>(n->d_pcnt[i]), static_cast<void*>(n->d_psidx[i]), static_cast<void*>(n->d_psval[i])})
      if (p) (void)hipFree(p);
  if (n->h_desc) (void)hipHostFree(n->h_desc);
  if (n->h_map) (void)hipHostFree(n->h_map);
  if (n->h_tau) (void)hipHostFree(n->h_tau);
  if (n->h_tmp) (void)hipHostFree(n->h_tmp);
  if (n->h_flag) (void)hipHostFree(n->h_flag);
  if (n->h_sdesc) (void)hipHostFree(n->h_sdesc);
  delete n;
}

int row(bccb_lista_s* n, int mode, RowArgs a, int nscenes) {
  a.tw = n->plan->d_tw1;
  a.nrows = nscenes * n->L2;
  a.rows_per_scene = n->L2;
  return kern(launch_row(n->L1, n->rcfg, mode, a, n->stream));
}

int col(bccb_lista_s* n, int mode, float2* xy, int nscenes, const float2* coef, const float2* mulc, const int* map) {
  ColArgs a;
  a.xy = xy;
  a.sup_ptr = n->plan->d_sup_ptr;
  a.sup = n->plan->d_sup;
  a.sup_rhs = n->d_sup_rhs;
  a.sup_rhs_stride = n->plan->nsup;
  a.omega = n->plan->d_omega;
  a.omega_stride = 0;
  a.mulc = mulc;
  a.mulc_stride = 0;
  a.coef = coef;
  a.tw = n->plan->d_tw2;
  a.L1 = n->L1;
  a.nscenes = nscenes;
  a.scene_map = map;
  return kern(launch_col(n->L2, n->ccfg, mode, a, n->stream));
}

// b_s = D_s^H y_s for every scene (y contiguous [batch][M]) and tau to the device.
int setup_rhs(bccb_lista_s* n, const bccb_c32* y, const float* tau, int batch) {
  bccb_plan_s* p = n->plan;
  for (int s = 0; s < batch; ++s) {
    if (!(tau[s] >= 0.f) || !std::isfinite(tau[s])) return BCCB_E_INVALID;
    SceneDesc& d = n->h_desc[s];
    d.y = reinterpret_cast<const float2*>(y) + static_cast<size_t>(s) * p->M;
    d.sensor_of = p->d_sensor_of;
    d.out = nullptr;
    d.M1 = p->M1;
    d.M2 = p->M2;
    d.scale = 1.f;
    n->h_tau[s] = tau[s];
  }
  BCCB_HIP(hipMemsetAsync(n->d_flag, 0, sizeof(int), n->stream));
  BCCB_HIP(hipMemcpyAsync(n->d_desc, n->h_desc, batch * sizeof(SceneDesc), hipMemcpyHostToDevice, n->stream));
  BCCB_HIP(hipMemcpyAsync(n->d_tau, n->h_tau, batch * sizeof(float), hipMemcpyHostToDevice, n->stream));
  BCCB_TRY(kern(launch_scatter_batch(n->d_desc, batch, n->L1, n->L2, n->d_xy, n->d_flag, n->stream)));
  BCCB_TRY(col(n, COL_INV, n->d_xy, batch, nullptr, nullptr, nullptr));
  RowArgs a;
  a.xy = n->d_xy;
  a.dst = n->d_b;
  return row(n, ROW_INV, a, batch);
}

int finish(bccb_lista_s* n) {
  BCCB_HIP(hipMemcpyAsync(n->h_flag, n->d_flag, sizeof(int), hipMemcpyDeviceToHost, n->stream));
  BCCB_HIP(hipStreamSynchronize(n->stream));
  return *n->h_flag ? BCCB_E_NONFINITE : BCCB_OK;
}

// The unrolled layers on the current b / tau (c and xy arenas start at zero).
int run_layers(bccb_lista_s* n, const float* params, int batch, bool save) {
  BCCB_TRY(kern(lista_prepare(params, n->plan->d_omega, static_cast<float>(n->plan->mu), n->L1, n->L2, n->K, n->d_mulc,
                              n->d_omp, n->d_dscal, n->stream)));
  BCCB_TRY(kern(launch_fill(n->d_c, static_cast<long>(batch) * n->L, n->stream)));
  BCCB_TRY(kern(launch_fill(n->d_xy, static_cast<long>(batch) * n->L, n->stream)));
  const size_t lay = static_cast<size_t>(n->cap) * n->L;
  for (int k = 0; k < n->K; ++k) {
    BCCB_TRY(col(n, COL_FILTER_CPLX, n->d_xy, batch, nullptr, n->d_mulc + k * n->L, nullptr));
    RowArgs a;
    a.xy = n->d_xy;
    a.rhs = n->d_b;
    a.state = n->d_c;
    a.kscale = n->d_tau;
    a.dscal = n->d_dscal + 2 * k;
    a.beta = static_cast<float>(n->beta[k]);
    a.last = (k == n->K - 1);
    if (a.last) a.out_prev = n->d_cprev;
    if (save) {
      a.save_u = n->d_U + k * lay;
      a.save_c = n->d_C + k * lay;
    }
    BCCB_TRY(row(n, ROW_FISTA, a, batch));
  }
  return BCCB_OK;
}

// The unrolled layers through the pruned passes (inference): the correction
// -mu_k Omega'_k DFT2(z) + mu_k DFT2(b) lives on the dilated support, the identity
// part in the spatial domain; c_k rotates over the fallback's slot buffers.  The
// last layer leaves c_{K-1} in d_c and c_{K-2} in d_cprev, as run_layers does.
int run_layers_pruned(bccb_lista_s* n, const float* params, int batch) {
  hipStream_t s = n->stream;
  bccb_plan_s* pl = n->plan;
  BCCB_TRY(kern(lista_prepare(params, pl->d_omega, static_cast<float>(pl->mu), n->L1, n->L2, n->K, n->d_mulc,
                              n->d_omp, n->d_dscal, s)));
  const long rows = static_cast<long>(batch) * n->L2;
  BCCB_TRY(kern(launch_fill_int(n->d_pcnt[0], rows, 0, s)));   // c_0 = 0
  BCCB_TRY(kern(launch_fill_int(n->d_pcnt[2], rows, 0, s)));   // c_{-1} = 0
  BCCB_TRY(kern(launch_fill(n->d_xycd, rows * n->ncsd, s)));   // DFT_rows(z_1 = 0)
  auto buf = [&](int i) {
    SlotBuf b;
    b.cnt = n->d_pcnt[i];
    b.sidx = n->d_psidx[i];
    b.sval = n->d_psval[i];
    b.dense = i == 0 ? n->d_R0 : (i == 1 ? n->d_xy : n->d_cprev);
    return b;
  };
  for (int k = 0; k < n->K; ++k) {
    ColArgs c;
    c.xy = n->d_xycd;
    c.sup_ptr = n->d_dsup_ptr;
    c.dil = n->d_dil;
    c.sup_rhs = n->d_sup_rhs;
    c.sup_rhs_stride = pl->nsup;
    c.mulc = n->d_mulc + static_cast<size_t>(k) * n->L;
    c.dscal = n->d_dscal + 2 * k;
    c.inv_mu = static_cast<float>(1.0 / pl->mu);
    c.scale = static_cast<float>(1.0 / static_cast<double>(n->L));
    c.tw = pl->d_tw2;
    c.L1 = n->L1;
    c.nscenes = batch;
    c.ncols = n->ncsd;
    c.ldx = n->ncsd;
    c.scol = n->d_dscol;
    BCCB_TRY(kern(launch_col(n->L2, n->ccfgd, COL_PRUNED_CPLX, c, s)));
    RowArgs a;
    a.xy = n->d_xycd;
    a.colslot = n->d_dcolslot;
    a.ncs = n->ncsd;
    a.b0 = buf((k + 1) % 3);
    a.b1 = buf(k % 3);
    a.b2 = buf((k + 2) % 3);
    a.out_c = n->d_c;
    a.kscale = n->d_tau;
    a.dscal = n->d_dscal + 2 * k;
    a.beta = static_cast<float>(n->beta[k]);
    a.beta_prev = k > 0 ? static_cast<float>(n->beta[k - 1]) : 0.f;
    a.last = (k == n->K - 1);
    if (a.last) a.out_prev = n->d_cprev;
    a.tw = pl->d_tw1;
    a.nrows = batch * n->L2;
    a.rows_per_scene = n->L2;
    BCCB_TRY(kern(launch_row(n->L1, n->rcfgd, ROW_PRUNED, a, s)));
  }
  return BCCB_OK;
}

// sum of e^2 (KKT residual terms) per physical scene of the map, into d_rk
int kkt_sums(bccb_lista_s* n, int nact, const int* map) {
  if (n->kkt_pruned) {
    // b - G c on the kept spectral columns: kept row DFT of c, then the pruned
    // column pass with -mu Omega/L and mu S (the fallback's multiplier and
    // right-hand side), so the row kernel scales by 1/mu
    bccb_plan_s* pl = n->plan;
    RowArgs f;
    f.xy = n->d_xyck;
    f.src = n->d_c;
    f.scene_map = map;
    f.colslot = pl->d_colslot;
    f.ncs = pl->ncs;
    f.tw = pl->d_tw1;
    f.nrows = nact * n->L2;
    f.rows_per_scene = n->L2;
    BCCB_TRY(kern(launch_row(n->L1, n->rcfgp, ROW_PRUNED_FWD, f, n->stream)));
    ColArgs c;
    c.xy = n->d_xyck;
    c.sup_ptr = pl->d_sup_ptr;
    c.sup = pl->d_sup;
    c.sup_rhs = n->d_sup_rhs;
    c.sup_rhs_stride = pl->nsup;
    c.coef = n->d_coef_fista;
    c.tw = pl->d_tw2;
    c.L1 = n->L1;
    c.nscenes = nact;
    c.scene_map = map;
    c.ncols = pl->ncs;
    c.ldx = pl->ncs;
    c.scol = pl->d_scol;
    BCCB_TRY(kern(launch_col(n->L2, n->ccfgp, COL_PRUNED_AFFINE, c, n->stream)));
    KktRowArgs k;
    k.gc = n->d_xyck;
    k.c = n->d_c;
    k.tau = n->d_tau;
    k.part = n->d_rows;
    k.scene_map = map;
    k.tw = pl->d_tw1;
    k.nrows = nact * n->L2;
    k.rows_per_scene = n->L2;
    k.colslot = pl->d_colslot;
    k.ncs = pl->ncs;
    k.scale = static_cast<float>(1.0 / pl->mu);
    BCCB_TRY(kern(lista_launch(n->L1, 3, &k, n->bwdE, n->bwd_rpb, 1, n->stream)));
    return kern(rows_to_scene(n->d_rows, n->L2, nact, map, n->d_rk, n->stream));
  }
  RowArgs f;
  f.xy = n->d_A;
  f.src = n->d_c;   // the fallback keeps a dense copy of every check's iterate here
  f.scene_map = map;
  BCCB_TRY(row(n, ROW_FWD, f, nact));
  BCCB_TRY(col(n, COL_FILTER_AFFINE, n->d_A, nact, n->d_coef_gram, nullptr, map));
  KktRowArgs k;
  k.gc = n->d_A;
  k.c = n->d_c;
  k.b = n->d_b;
  k.tau = n->d_tau;
  k.part = n->d_rows;
  k.scene_map = map;
  k.tw = n->plan->d_tw1;
  k.nrows = nact * n->L2;
  k.rows_per_scene = n->L2;
  BCCB_TRY(kern(lista_launch(n->L1, 2, &k, n->bwdE, n->bwd_rpb, 1, n->stream)));
  return kern(rows_to_scene(n->d_rows, n->L2, nact, map, n->d_rk, n->stream));
}

// The persistent launch for the pruned fallback: one class (the plan's square grid), tables
// shared by every scene, the per-scene right-hand sides and thresholds, the active list as
// the scene map, the fallback's slot buffers and kept spectra as the carried state, and the
// dense iterate c as the output.  Leaves res_ok false when the shape does not fit.
int resident_setup(bccb_lista_s* n) {
  bccb_plan_s* pl = n->plan;
  const int N = n->L1;
  if (n->L1 != n->L2 || (N != 32 && N != 64 && N != 128 && N != 256) || pl->ncs < 1) return BCCB_OK;
  ResidentClass r;
  r.N = N;
  r.n = n->cap;
  r.ncs = pl->ncs;
  r.xs = pl->ncs | 1;
  r.colslot = pl->d_colslot;
  r.scol = pl->d_scol;
  r.sup_ptr = pl->d_sup_ptr;
  r.sup = pl->d_sup;
  r.sup_rhs = n->d_sup_rhs;
  r.rhs_stride = pl->nsup;
  r.coef = n->d_coef_fista;
  r.kscale = n->d_tau;
  r.kmul = static_cast<float>(pl->mu);
  r.tw = pl->d_tw1;
  r.out_base = n->d_c;
  r.scene_map = n->d_map;
  r.xkeep = n->d_xyc;
  r.kkt_sum = n->d_rk;   // each chunk's launch ends with the KKT check of its scenes
  r.kkt_scale = static_cast<float>(1.0 / pl->mu);
  float2* dense[3] = {n->d_R0, n->d_xy, n->d_cprev};
  for (int i = 0; i < 3; ++i) {
    r.buf[i].cnt = n->d_pcnt[i];
    r.buf[i].sidx = n->d_psidx[i];
    r.buf[i].sval = n->d_psval[i];
    r.buf[i].dense = dense[i];
  }
  int best = 0;
  for (int nt : {256, 512, 1024}) {
    const long lds = resident_lds_bytes(N, r.ncs, nt);
    const int nb = scene_fista_occupancy(nt, static_cast<size_t>(lds), 1);
    if (nb * (nt / 64) > best) {
      best = nb * (nt / 64);
      n->res_threads = nt;
      n->res_lds = static_cast<size_t>(lds);
      n->res_blocks = nb;
    }
  }
  if (best == 0) return BCCB_OK;
  int dev = 0, cus = 0;
  BCCB_HIP(hipGetDevice(&dev));
  BCCB_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  n->res_blocks *= std::max(cus, 1);
  BCCB_TRY(dalloc(&n->d_rcls, 1));
  BCCB_TRY(dalloc(&n->d_queue, 1));
  BCCB_HIP(hipMemcpy(n->d_rcls, &r, sizeof(ResidentClass), hipMemcpyHostToDevice));
  n->res_ok = n->res_on = true;
  return BCCB_OK;
}

// Momentum weights of the fallback: beta[0] = the weight before its first iteration,
// beta[t] = (alpha_t - 1) / alpha_{t+1} from alpha, for t = 1..iters (the graph loop's schedule).
int resident_betas(bccb_lista_s* n, int iters, double alpha, float beta0) {
  if (iters + 1 > n->rbeta_cap) {
    if (n->d_rbeta) (void)hipFree(n->d_rbeta);
    if (n->h_rbeta) (void)hipHostFree(n->h_rbeta);
    n->d_rbeta = nullptr;
    n->h_rbeta = nullptr;
    n->rbeta_cap = 0;
    BCCB_TRY(dalloc(&n->d_rbeta, iters + 1));
    if (hipHostMalloc(reinterpret_cast<void**>(&n->h_rbeta), (iters + 1) * sizeof(float)) != hipSuccess) {
      n->h_rbeta = nullptr;
      return BCCB_E_NOMEM;
    }
    n->rbeta_cap = iters + 1;
  }
  n->h_rbeta[0] = beta0;
  for (int t = 1; t <= iters; ++t) {
    const double an = (1.0 + std::sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0;
    n->h_rbeta[t] = static_cast<float>((alpha - 1.0) / an);
    alpha = an;
  }
  BCCB_HIP(hipMemcpyAsync(n->d_rbeta, n->h_rbeta, (iters + 1) * sizeof(float), hipMemcpyHostToDevice, n->stream));
  return BCCB_OK;
}

}  // namespace

extern "C" {

int lista_create(bccb_plan_t plan, int layers, int max_batch, int train, bccb_lista_t* out) {
  if (!plan || layers < 1 || layers > 256 || max_batch < 1 || !out) return BCCB_E_INVALID;
  *out = nullptr;
  if (plan->emb) return BCCB_E_UNSUPPORTED;
  bccb_lista_s* n = new (std::nothrow) bccb_lista_s();
  if (!n) return BCCB_E_NOMEM;
  n->plan = plan;
  n->K = layers;
  n->cap = max_batch;
  n->train = train ? 1 : 0;
  n->L1 = plan->L1;
  n->L2 = plan->L2;
  n->L = plan->L;
  n->stream = plan->stream;
  double al = 1.0;
  for (int k = 0; k < layers; ++k) {
    const double an = (1.0 + std::sqrt(1.0 + 4.0 * al * al)) / 2.0;
    n->beta.push_back((al - 1.0) / an);
    al = an;
  }
  n->alpha_end = al;
  // throughput shapes: 16 elements per thread, 256-thread blocks
  n->rcfg.E = n->L1 >= 16 ? 16 : 8;
  n->rcfg.rpb = std::max(1, 256 / (n->L1 / n->rcfg.E));
  while (!row_shape_ok(n->L1, n->rcfg) && n->rcfg.rpb > 1) n->rcfg.rpb /= 2;
  n->ccfg.E = n->L2 >= 16 ? 16 : 8;
  n->ccfg.W = std::min(n->L1, std::max(1, 256 / (n->L2 / n->ccfg.E)));
  while (!col_shape_ok(n->L1, n->L2, n->ccfg) && n->ccfg.W > 1) n->ccfg.W /= 2;
  n->bwdE = n->L1 >= 16 ? 16 : 8;
  {
    const int T = n->L1 / n->bwdE;
    n->bwd_rpb = std::max(1, 128 / T);
    while (n->bwd_rpb > 1 && ((static_cast<long>(n->bwd_rpb) * fft_area(n->L1) + n->L1) * 8 +
                              static_cast<long>(n->bwd_rpb) * T * 16 > 65536))
      n->bwd_rpb /= 2;
    const int Tc = n->L2 / (n->L2 >= 16 ? 16 : 8);
    n->bwd_W = std::min(n->L1, std::max(1, 128 / Tc));
    while (n->bwd_W > 1 && (static_cast<long>(n->bwd_W) * fft_area(n->L2) + n->L2) * 8 > 65536) n->bwd_W /= 2;
  }
  n->groups = std::max(1, std::min(64, 512 / std::max(1, n->L1 / n->bwd_W)));

  const size_t pts = static_cast<size_t>(max_batch) * n->L;
  int rc = BCCB_OK;
  if (rc == BCCB_OK) rc = dalloc(&n->d_b, pts);
  if (rc == BCCB_OK) rc = dalloc(&n->d_c, pts);
  if (rc == BCCB_OK) rc = dalloc(&n->d_cprev, pts);
  if (rc == BCCB_OK) rc = dalloc(&n->d_xy, pts);
  if (rc == BCCB_OK) rc = dalloc(&n->d_A, pts);
  if (rc == BCCB_OK && train) rc = dalloc(&n->d_Z, pts);
  if (rc == BCCB_OK && train) rc = dalloc(&n->d_ring[0], pts);
  if (rc == BCCB_OK && train) rc = dalloc(&n->d_ring[1], pts);
  if (rc == BCCB_OK && train) rc = dalloc(&n->d_U, pts * layers);
  if (rc == BCCB_OK && train) rc = dalloc(&n->d_C, pts * layers);
  if (rc == BCCB_OK) rc = dalloc(&n->d_mulc, static_cast<size_t>(layers) * n->L);
  if (rc == BCCB_OK) rc = dalloc(&n->d_omp, static_cast<size_t>(layers) * n->L);
  if (rc == BCCB_OK) rc = dalloc(&n->d_dscal, 2 * layers);
  if (rc == BCCB_OK) rc = dalloc(&n->d_tau, max_batch);
  if (rc == BCCB_OK) rc = dalloc(&n->d_coef_fista, max_batch);
  if (rc == BCCB_OK) rc = dalloc(&n->d_coef_gram, max_batch);
  if (rc == BCCB_OK) rc = dalloc(&n->d_rows, static_cast<size_t>(max_batch) * n->L2 * 2);
  if (rc == BCCB_OK && train) rc = dalloc(&n->d_gm_part, static_cast<size_t>(n->groups) * n->L);
  if (rc == BCCB_OK && train) rc = dalloc(&n->d_gm, n->L);
  if (rc == BCCB_OK) rc = dalloc(&n->d_lg, 64);
  if (rc == BCCB_OK) rc = dalloc(&n->d_sum_part, static_cast<size_t>(max_batch) * kSumBlocksPerScene * 2);
  if (rc == BCCB_OK) rc = dalloc(&n->d_sums, static_cast<size_t>(max_batch) * 2);
  if (rc == BCCB_OK) rc = dalloc(&n->d_sums2, static_cast<size_t>(max_batch) * 2);
  if (rc == BCCB_OK) rc = dalloc(&n->d_bnorm, static_cast<size_t>(max_batch) * 2);
  if (rc == BCCB_OK) rc = dalloc(&n->d_rk, max_batch);
  if (rc == BCCB_OK) rc = dalloc(&n->d_desc, max_batch);
  if (rc == BCCB_OK) rc = dalloc(&n->d_map, max_batch);
  if (rc == BCCB_OK) rc = dalloc(&n->d_flag, 1);
  if (rc == BCCB_OK && sparse_on(plan)) {
    rc = dalloc(&n->d_sup_rhs, static_cast<size_t>(max_batch) * plan->nsup);
    if (rc == BCCB_OK) rc = dalloc(&n->d_sdesc, max_batch);
    if (rc == BCCB_OK && hipHostMalloc(reinterpret_cast<void**>(&n->h_sdesc), max_batch * sizeof(SupRhsDesc)) != hipSuccess)
      rc = BCCB_E_NOMEM;
  }
  if (rc == BCCB_OK && plan->prune_ok && sparse_on(plan)) {
    // pruned fallback FISTA: kept row spectra, slot buffers, one more dense grid
    const size_t rows = static_cast<size_t>(max_batch) * n->L2;
    rc = dalloc(&n->d_xyc, rows * plan->ncs);
    if (rc == BCCB_OK) rc = dalloc(&n->d_xyck, rows * plan->ncs);
    if (rc == BCCB_OK) rc = dalloc(&n->d_R0, pts);
    for (int i = 0; i < 3 && rc == BCCB_OK; ++i) {
      rc = dalloc(&n->d_pcnt[i], rows);
      // L1/8 slots per row for the passes, L1/kResidentSlotDiv for the persistent launch
      if (rc == BCCB_OK) rc = dalloc(&n->d_psidx[i], rows * (n->L1 / kResidentSlotDiv));
      if (rc == BCCB_OK) rc = dalloc(&n->d_psval[i], rows * (n->L1 / kResidentSlotDiv));
    }
    n->prune = rc == BCCB_OK;
    n->rcfgp.E = n->L1 >= 16 ? 16 : 8;
    n->rcfgp.rpb = std::max(1, 256 / (n->L1 / n->rcfgp.E));
    while (!rowp_shape_ok(n->L1, n->rcfgp, plan->ncs) && n->rcfgp.rpb > 1) n->rcfgp.rpb /= 2;
    n->ccfgp.E = n->L2 >= 16 ? 16 : 8;
    n->ccfgp.W = std::min(plan->ncs, std::max(1, 256 / (n->L2 / n->ccfgp.E)));
    while (!colp_shape_ok(plan->ncs, n->L2, n->ccfgp) && n->ccfgp.W > 1) n->ccfgp.W /= 2;
  }
  if (rc == BCCB_OK && n->prune) {
    // the learned layers' support: every bin within the 5x5 box of a support bin of Omega
    const int L1 = n->L1, L2 = n->L2;
    std::vector<int> orig(static_cast<size_t>(n->L), -2);   // -2: off, -1: dilated only, >= 0: plan entry
    for (int k1 = 0; k1 < L1; ++k1)
      for (int j = plan->h_sup_ptr[k1]; j < plan->h_sup_ptr[k1 + 1]; ++j) {
        const int k2 = plan->h_sup[j].k2;
        for (int a = -2; a <= 2; ++a)
          for (int b = -2; b <= 2; ++b) {
            const long bin = static_cast<long>(((k2 + a) % L2 + L2) % L2) * L1 + ((k1 + b) % L1 + L1) % L1;
            if (orig[bin] == -2) orig[bin] = -1;
          }
      }
    for (int k1 = 0; k1 < L1; ++k1)
      for (int j = plan->h_sup_ptr[k1]; j < plan->h_sup_ptr[k1 + 1]; ++j)
        orig[static_cast<long>(plan->h_sup[j].k2) * L1 + k1] = j;
    std::vector<int> scol, colslot(L1, -1), sptr(L1 + 1, 0);
    std::vector<DilEntry> dil;
    for (int k1 = 0; k1 < L1; ++k1) {
      sptr[k1] = static_cast<int>(dil.size());
      for (int k2 = 0; k2 < L2; ++k2) {
        const int o = orig[static_cast<long>(k2) * L1 + k1];
        if (o != -2) dil.push_back(DilEntry{k2, o});
      }
      if (static_cast<int>(dil.size()) > sptr[k1]) {
        colslot[k1] = static_cast<int>(scol.size());
        scol.push_back(k1);
      }
    }
    sptr[L1] = static_cast<int>(dil.size());
    n->ncsd = (static_cast<int>(scol.size()) + 3) / 4 * 4;
    scol.resize(n->ncsd, -1);
    if (n->ncsd <= L1 / 2) {
      const size_t rows = static_cast<size_t>(max_batch) * L2;
      rc = dalloc(&n->d_dscol, scol.size());
      if (rc == BCCB_OK) rc = dalloc(&n->d_dcolslot, L1);
      if (rc == BCCB_OK) rc = dalloc(&n->d_dsup_ptr, sptr.size());
      if (rc == BCCB_OK) rc = dalloc(&n->d_dil, dil.size());
      if (rc == BCCB_OK) rc = dalloc(&n->d_xycd, rows * n->ncsd);
      if (rc == BCCB_OK &&
          (hipMemcpy(n->d_dscol, scol.data(), scol.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
           hipMemcpy(n->d_dcolslot, colslot.data(), L1 * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
           hipMemcpy(n->d_dsup_ptr, sptr.data(), sptr.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
           hipMemcpy(n->d_dil, dil.data(), dil.size() * sizeof(DilEntry), hipMemcpyHostToDevice) != hipSuccess))
        rc = BCCB_E_DEVICE;
      n->rcfgd = n->rcfgp;
      while (!rowp_shape_ok(L1, n->rcfgd, n->ncsd) && n->rcfgd.rpb > 1) n->rcfgd.rpb /= 2;
      n->ccfgd = n->ccfgp;
      n->ccfgd.W = std::min(n->ncsd, std::max(1, 256 / (L2 / n->ccfgd.E)));
      while (!colp_shape_ok(n->ncsd, L2, n->ccfgd) && n->ccfgd.W > 1) n->ccfgd.W /= 2;
      n->prune_layers = rc == BCCB_OK && rowp_shape_ok(L1, n->rcfgd, n->ncsd) && colp_shape_ok(n->ncsd, L2, n->ccfgd);
    }
  }
  if (rc == BCCB_OK && (hipHostMalloc(reinterpret_cast<void**>(&n->h_desc), max_batch * sizeof(SceneDesc)) != hipSuccess ||
                        hipHostMalloc(reinterpret_cast<void**>(&n->h_map), max_batch * sizeof(int)) != hipSuccess ||
                        hipHostMalloc(reinterpret_cast<void**>(&n->h_tau), max_batch * sizeof(float)) != hipSuccess ||
                        hipHostMalloc(reinterpret_cast<void**>(&n->h_tmp), max_batch * 2 * sizeof(double)) != hipSuccess ||
                        hipHostMalloc(reinterpret_cast<void**>(&n->h_flag), sizeof(int)) != hipSuccess))
    rc = BCCB_E_NOMEM;
  if (rc == BCCB_OK) {
    const float invL = static_cast<float>(1.0 / static_cast<double>(n->L));
    std::vector<float2> cf(max_batch, make_float2(invL, static_cast<float>(-plan->mu / static_cast<double>(n->L))));
    std::vector<float2> cg(max_batch, make_float2(0.f, invL));
    if (hipMemcpy(n->d_coef_fista, cf.data(), cf.size() * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(n->d_coef_gram, cg.data(), cg.size() * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess)
      rc = BCCB_E_DEVICE;
  }
  if (rc == BCCB_OK && n->prune) rc = resident_setup(n);
  if (rc != BCCB_OK) {
    lista_free(n);
    return rc;
  }
  *out = n;
  return BCCB_OK;
}

int lista_set_resident(bccb_lista_t n, int on) {
  if (!n || (on != 0 && on != 1)) return BCCB_E_INVALID;
  if (on == 1 && !n->res_ok) return BCCB_E_UNSUPPORTED;
  n->res_on = on == 1;
  return BCCB_OK;
}

int lista_destroy(bccb_lista_t n) {
  if (n) (void)hipStreamSynchronize(n->stream);
  lista_free(n);
  return BCCB_OK;
}

int lista_forward(bccb_lista_t n, const float* params, const bccb_c32* y, const float* tau, int batch,
                  bccb_c32* c_out) {
  if (!n || !params || !y || !tau || batch < 1 || batch > n->cap) return BCCB_E_INVALID;
  BCCB_TRY(setup_rhs(n, y, tau, batch));
  BCCB_TRY(run_layers(n, params, batch, n->train != 0));
  if (c_out)
    BCCB_TRY(kern(launch_copy(reinterpret_cast<float2*>(c_out), n->d_c, static_cast<long>(batch) * n->L, n->stream)));
  n->batch = batch;
  n->have_acts = n->train != 0;
  return finish(n);
}

int lista_backward(bccb_lista_t n, const float* params, const bccb_c32* labels, float* grad, double* loss) {
  if (!n || !params || !labels || !grad) return BCCB_E_INVALID;
  if (!n->have_acts) return BCCB_E_INVALID;
  const int B = n->batch;
  const long L = n->L;
  const size_t lay = static_cast<size_t>(n->cap) * L;
  const float2* lab = reinterpret_cast<const float2*>(labels);
  hipStream_t s = n->stream;
  const float2* cK = n->d_C + (n->K - 1) * lay;
  // ||c*||^2 and ||c_{K-1} - c*||^2 per scene
  BCCB_TRY(kern(scene_sums(lab, cK, L, B, n->d_sum_part, n->d_sums, s)));
  BCCB_HIP(hipMemcpyAsync(n->h_tmp, n->d_sums, B * 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  std::vector<double> ln(B);
  BCCB_HIP(hipStreamSynchronize(s));
  double total = 0.0;
  for (int i = 0; i < B; ++i) {
    ln[i] = n->h_tmp[2 * i];
    if (!(ln[i] > 0.0)) return BCCB_E_INVALID;  // an all-zero label has no relative error
    total += n->h_tmp[2 * i + 1] / ln[i];
  }
  if (loss) *loss = total / B;
  // norms packed as [B] for the loss gradient (even entries of d_sums2 hold them)
  BCCB_HIP(hipMemcpyAsync(n->d_bnorm, ln.data(), B * sizeof(double), hipMemcpyHostToDevice, s));
  BCCB_HIP(hipStreamSynchronize(s));
  for (int j = n->K - 1; j >= 0; --j) {
    ListaBwdRowArgs r;
    r.A_in = (j == n->K - 1) ? nullptr : n->d_A;
    r.zbar_store = (j == n->K - 1) ? nullptr : n->d_ring[(j + 1) & 1];
    r.zbar2 = (j + 2 <= n->K - 1) ? n->d_ring[j & 1] : nullptr;
    r.U = n->d_U + j * lay;
    r.Cm1 = j >= 1 ? n->d_C + (j - 1) * lay : nullptr;
    r.Cm2 = j >= 2 ? n->d_C + (j - 2) * lay : nullptr;
    r.b = n->d_b;
    r.cout = (j == n->K - 1) ? cK : nullptr;
    r.label = (j == n->K - 1) ? lab : nullptr;
    r.norm_label = n->d_bnorm;
    r.tau = n->d_tau;
    r.dscal = n->d_dscal + 2 * j;
    r.beta_j = static_cast<float>(n->beta[j]);
    r.beta_j1 = (j + 1 < n->K) ? static_cast<float>(n->beta[j + 1]) : 0.f;
    r.beta_jm1 = j >= 1 ? static_cast<float>(n->beta[j - 1]) : 0.f;
    r.loss_scale = 2.f / static_cast<float>(B);
    r.Aout = n->d_A;
    r.Zout = n->d_Z;
    r.part = n->d_rows;
    r.tw = n->plan->d_tw1;
    r.nrows = B * n->L2;
    r.rows_per_scene = n->L2;
    BCCB_TRY(kern(lista_launch(n->L1, 0, &r, n->bwdE, n->bwd_rpb, 1, s)));
    ListaBwdColArgs c;
    c.A = n->d_A;
    c.Z = n->d_Z;
    c.mulc = n->d_mulc + j * L;
    c.gm_part = n->d_gm_part;
    c.tw = n->plan->d_tw2;
    c.L1 = n->L1;
    c.nscenes = B;
    c.groups = n->groups;
    BCCB_TRY(kern(lista_launch(n->L2, 1, &c, n->L2 >= 16 ? 16 : 8, n->bwd_W, n->groups, s)));
    BCCB_TRY(kern(lista_layer_grad(n->d_gm_part, n->groups, n->d_gm, n->d_omp + j * L, n->plan->d_omega, n->L1,
                                   n->L2, n->d_dscal + 2 * j, params + j * kListaPerLayer, n->d_rows, B, n->d_tau,
                                   n->d_lg, static_cast<float>(n->plan->mu), grad + j * kListaPerLayer, s)));
  }
  BCCB_HIP(hipStreamSynchronize(s));
  return BCCB_OK;
}

int lista_autotune(bccb_lista_t n, int reps) {
  if (!n || reps < 1) return BCCB_E_INVALID;
  if (!n->prune) return BCCB_OK;   // the full passes keep the layers' shapes
  hipStream_t s = n->stream;
  bccb_plan_s* pl = n->plan;
  const int nb = n->cap;
  const long rows = static_cast<long>(nb) * n->L2;
  // c_{t-1}, c_{t-2} in slot form (a few entries per row), c_t into buffer 0
  BCCB_TRY(kern(launch_fill(n->d_xyc, rows * pl->ncs, s)));
  BCCB_TRY(kern(launch_fill_int(n->d_pcnt[0], rows, 0, s)));
  BCCB_TRY(kern(launch_fill_int(n->d_pcnt[1], rows, 4, s)));
  BCCB_TRY(kern(launch_fill_int(n->d_pcnt[2], rows, 4, s)));
  RowArgs a;
  a.xy = n->d_xyc;
  a.colslot = pl->d_colslot;
  a.ncs = pl->ncs;
  SlotBuf b[3];
  for (int i = 0; i < 3; ++i) {
    b[i].cnt = n->d_pcnt[i];
    b[i].sidx = n->d_psidx[i];
    b[i].sval = n->d_psval[i];
  }
  b[0].dense = n->d_R0;
  b[1].dense = n->d_xy;
  b[2].dense = n->d_cprev;
  a.b0 = b[0];
  a.b1 = b[1];
  a.b2 = b[2];
  a.out_c = n->d_c;
  a.kscale = n->d_tau;
  a.kappa = static_cast<float>(pl->mu);
  a.beta = a.beta_prev = 0.5f;
  a.tw = pl->d_tw1;
  a.nrows = nb * n->L2;
  a.rows_per_scene = n->L2;
  ColArgs c;
  c.xy = n->d_xyc;
  c.sup_ptr = pl->d_sup_ptr;
  c.sup = pl->d_sup;
  c.sup_rhs = n->d_sup_rhs;
  c.sup_rhs_stride = pl->nsup;
  c.coef = n->d_coef_fista;
  c.tw = pl->d_tw2;
  c.L1 = n->L1;
  c.nscenes = nb;
  c.ncols = pl->ncs;
  c.ldx = pl->ncs;
  c.scol = pl->d_scol;
  float best_r = 1e30f, best_c = 1e30f;
  PassCfg br = n->rcfgp, bc = n->ccfgp;
  const int Es[4] = {4, 8, 16, 32};
  for (int E : Es) {
    for (int k = 1; k <= 256; k *= 2) {
      PassCfg r;
      r.E = E;
      r.rpb = k;
      if (rowp_shape_ok(n->L1, r, pl->ncs)) {
        const float ms = time_launches(s, reps, [&] { return kern(launch_row(n->L1, r, ROW_PRUNED, a, s)); });
        if (ms < 0.f) return BCCB_E_DEVICE;
        if (ms < best_r) { best_r = ms; br = r; }
      }
      PassCfg w;
      w.E = E;
      w.W = k;
      if (colp_shape_ok(pl->ncs, n->L2, w)) {
        const float ms = time_launches(s, reps, [&] { return kern(launch_col(n->L2, w, COL_PRUNED_AFFINE, c, s)); });
        if (ms < 0.f) return BCCB_E_DEVICE;
        if (ms < best_c) { best_c = ms; bc = w; }
      }
    }
  }
  n->rcfgp = br;
  n->ccfgp = bc;
  // the pruned learned layers run the same two kernels over the dilated column
  // set: they take the tuned E, with rows / columns per block cut down to fit it
  if (n->prune_layers) {
    PassCfg rd = br, cd = bc;
    while (!rowp_shape_ok(n->L1, rd, n->ncsd) && rd.rpb > 1) rd.rpb /= 2;
    cd.W = std::min(n->ncsd, cd.W);
    while (!colp_shape_ok(n->ncsd, n->L2, cd) && cd.W > 1) cd.W /= 2;
    if (rowp_shape_ok(n->L1, rd, n->ncsd)) n->rcfgd = rd;
    if (colp_shape_ok(n->ncsd, n->L2, cd)) n->ccfgd = cd;
  }
  return BCCB_OK;
}

int lista_adam(float* params, const float* grad, float* m, float* v, int cnt, int step, float lr, float beta1,
               float beta2, float eps, const float* lr_scale, void* stream) {
  if (!params || !grad || !m || !v || cnt < 1 || step < 1) return BCCB_E_INVALID;
  const float bc1 = static_cast<float>(1.0 - std::pow(static_cast<double>(beta1), step));
  const float bc2 = static_cast<float>(1.0 - std::pow(static_cast<double>(beta2), step));
  return kern(launch_adam(params, grad, m, v, cnt, lr, beta1, beta2, eps, bc1, bc2, lr_scale,
                          static_cast<hipStream_t>(stream)));
}

int lista_solve(bccb_lista_t n, const float* params, const bccb_c32* y, const float* tau, int batch,
                double kkt_target, int check_every, int max_iters, int restart, bccb_c32* c_out, int* iters_out,
                double* rkkt_out) {
  if (!n || !y || !tau || !c_out || batch < 1 || batch > n->cap || check_every < 1 || max_iters < 0 ||
      !(kkt_target > 0.0))
    return BCCB_E_INVALID;
  hipStream_t s = n->stream;
  BCCB_TRY(setup_rhs(n, y, tau, batch));
  const bool sparse = n->d_sup_rhs != nullptr;
  // the pruned passes (kept spectral columns, iterates in slot buffers) when the plan allows them
  const bool pruned = sparse && n->prune && pruned_on(n->plan);
  if (sparse) {
    // mu * D_s^H y of every scene on the support bins of its spectrum
    bccb_plan_s* p = n->plan;
    for (int i = 0; i < batch; ++i) {
      SupRhsDesc& d = n->h_sdesc[i];
      d.y = reinterpret_cast<const float2*>(y) + static_cast<size_t>(i) * p->M;
      d.entry_off = 0;
      d.nentries = p->nsup;
      d.rhs_off = static_cast<long>(i) * p->nsup;
      d.scale = static_cast<float>(p->mu);
    }
    BCCB_HIP(hipMemcpyAsync(n->d_sdesc, n->h_sdesc, batch * sizeof(SupRhsDesc), hipMemcpyHostToDevice, s));
    BCCB_TRY(kern(launch_sup_rhs(n->d_sdesc, batch, p->nsup, p->d_src_ptr, p->d_src, n->d_sup_rhs, n->d_flag, s)));
  }
  n->kkt_pruned = pruned;
  // ||b_s||^2
  BCCB_TRY(kern(scene_sums(n->d_b, nullptr, n->L, batch, n->d_sum_part, n->d_sums, s)));
  std::vector<double> bn(batch), rk(batch, 0.0), r0(batch, 0.0);
  std::vector<int> used(batch, 0);
  BCCB_HIP(hipMemcpyAsync(n->h_tmp, n->d_sums, batch * 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  BCCB_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < batch; ++i) bn[i] = n->h_tmp[2 * i];
  // d_map always holds the current active list (uploaded whenever it changes;
  // every upload is followed by a stream synchronisation before h_map is reused)
  auto upload = [&](const std::vector<int>& act) -> int {
    const int na = static_cast<int>(act.size());
    for (int i = 0; i < na; ++i) n->h_map[i] = act[i];
    if (na) BCCB_HIP(hipMemcpyAsync(n->d_map, n->h_map, na * sizeof(int), hipMemcpyHostToDevice, s));
    return BCCB_OK;
  };
  // r_KKT of the active scenes from the sums in d_rk
  auto read_residuals = [&](const std::vector<int>& act, std::vector<double>& r) -> int {
    BCCB_HIP(hipMemcpyAsync(n->h_tmp, n->d_rk, batch * sizeof(double), hipMemcpyDeviceToHost, s));
    BCCB_HIP(hipStreamSynchronize(s));
    for (int i : act) r[i] = bn[i] > 0.0 ? std::sqrt(n->h_tmp[i] / bn[i]) : std::sqrt(n->h_tmp[i]);
    return BCCB_OK;
  };
  auto residuals = [&](const std::vector<int>& act, std::vector<double>& r) -> int {
    BCCB_TRY(kkt_sums(n, static_cast<int>(act.size()), n->d_map));
    return read_residuals(act, r);
  };
  std::vector<int> act(batch);
  for (int i = 0; i < batch; ++i) act[i] = i;
  BCCB_TRY(upload(act));
  // residual of the zero start, the reference every warm start must beat
  BCCB_TRY(kern(launch_fill(n->d_c, static_cast<long>(batch) * n->L, s)));
  BCCB_TRY(residuals(act, r0));
  if (params) {
    if (pruned && n->prune_layers) BCCB_TRY(run_layers_pruned(n, params, batch));
    else BCCB_TRY(run_layers(n, params, batch, false));
    BCCB_TRY(residuals(act, rk));
  } else {
    rk = r0;
  }
  {
    // A network output that is non-finite (e.g. corrupted weights) or farther
    // from stationarity than zero is discarded: that scene's fallback restarts
    // from zero, so the gate never does worse than plain FISTA.
    std::vector<int> keep;
    for (int i : act) {
      if (!std::isfinite(rk[i]) || rk[i] > r0[i]) {
        BCCB_TRY(kern(launch_fill(n->d_c + static_cast<size_t>(i) * n->L, n->L, s)));
        rk[i] = r0[i];
        restart = 1;  // the discarded scene starts over, so the shared momentum does too
      }
      if (!(rk[i] <= kkt_target)) keep.push_back(i);
    }
    act.swap(keep);
  }
  // Continuing the unrolled FISTA: z = c_{K-1} + beta_{K-1} (c_{K-1} - c_{K-2}) and the
  // alpha schedule resumes after the K layers; restarting: z = c_{K-1}, alpha = 1.
  const bool carry = params && !restart;
  int done_iters = 0;
  double alpha = carry ? n->alpha_end : 1.0;
  bccb_plan_s* pl = n->plan;
  auto pbuf = [&](int i) {
    SlotBuf b;
    b.cnt = n->d_pcnt[i];
    b.sidx = n->d_psidx[i];
    b.sval = n->d_psval[i];
    b.dense = i == 0 ? n->d_R0 : (i == 1 ? n->d_xy : n->d_cprev);
    return b;
  };
  int tp = 0;   // pruned iterations so far: c_t lives in buffer tp mod 3
  float beta_prev = 0.f;
  if (!act.empty() && max_iters > 0) {
    // warm start: z = current c (network output or zeros) or its momentum continuation
    const int na = static_cast<int>(act.size());
    BCCB_TRY(upload(act));
    RowArgs f;
    f.xy = n->d_xy;
    f.src = n->d_c;
    f.scene_map = n->d_map;
    if (carry) {
      BCCB_TRY(kern(launch_momentum(n->d_A, n->d_c, n->d_cprev, static_cast<float>(n->beta[n->K - 1]), n->L, na,
                                    n->d_map, s)));
      f.src = n->d_A;
    }
    if (pruned) {
      // c_0 (dense, buffer 0) = the current c; c_{-1} (buffer 2) = c_{K-2} of the layers or none
      const long rows = static_cast<long>(batch) * n->L2;
      BCCB_TRY(kern(launch_copy(n->d_R0, n->d_c, static_cast<long>(batch) * n->L, s)));
      BCCB_TRY(kern(launch_fill_int(n->d_pcnt[0], rows, n->L1 + 1, s)));
      BCCB_TRY(kern(launch_fill_int(n->d_pcnt[2], rows, carry ? n->L1 + 1 : 0, s)));
      beta_prev = carry ? static_cast<float>(n->beta[n->K - 1]) : 0.f;
      f.xy = n->d_xyc;
      f.colslot = pl->d_colslot;
      f.ncs = pl->ncs;
      f.tw = pl->d_tw1;
      f.nrows = na * n->L2;
      f.rows_per_scene = n->L2;
      BCCB_TRY(kern(launch_row(n->L1, n->rcfgp, ROW_PRUNED_FWD, f, s)));
    } else {
      BCCB_TRY(row(n, ROW_FWD, f, na));
    }
  }
  const bool resident = pruned && n->res_on && !act.empty() && max_iters > 0;
  if (resident) BCCB_TRY(resident_betas(n, max_iters, alpha, beta_prev));
  while (!act.empty() && done_iters < max_iters) {
    const int na = static_cast<int>(act.size());
    const int steps = std::min(check_every, max_iters - done_iters);
    if (resident) {
      // the check interval of every active scene in one persistent launch (iterations
      // tp + 1 .. tp + steps, the state carried in d_xyc and the slot counts, c_t to d_c),
      // ending with each scene's KKT sum in d_rk
      BCCB_TRY(kern(launch_fill_int(n->d_queue, 1, 0, s)));
      BCCB_TRY(kern(launch_scene_fista(n->d_rcls, 1, na, n->d_rbeta, tp, steps, 1, 1, n->d_queue, n->res_threads,
                                       std::min(n->res_blocks, na), n->res_lds, s)));
      tp += steps;
    }
    for (int t = 0; t < steps && !resident; ++t) {
      const double an = (1.0 + std::sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0;
      const float beta = static_cast<float>((alpha - 1.0) / an);
      alpha = an;
      if (pruned) {
        ColArgs c;
        c.xy = n->d_xyc;
        c.sup_ptr = pl->d_sup_ptr;
        c.sup = pl->d_sup;
        c.sup_rhs = n->d_sup_rhs;
        c.sup_rhs_stride = pl->nsup;
        c.coef = n->d_coef_fista;
        c.tw = pl->d_tw2;
        c.L1 = n->L1;
        c.nscenes = na;
        c.scene_map = n->d_map;
        c.ncols = pl->ncs;
        c.ldx = pl->ncs;
        c.scol = pl->d_scol;
        BCCB_TRY(kern(launch_col(n->L2, n->ccfgp, COL_PRUNED_AFFINE, c, s)));
        ++tp;
        RowArgs a;
        a.xy = n->d_xyc;
        a.colslot = pl->d_colslot;
        a.ncs = pl->ncs;
        a.b0 = pbuf(tp % 3);
        a.b1 = pbuf((tp - 1) % 3);
        a.b2 = pbuf((tp + 1) % 3);
        a.out_c = n->d_c;
        a.keep_c = (t + 1 == steps) ? n->d_c : nullptr;   // dense c_t for the check and the output
        a.kscale = n->d_tau;
        a.kappa = static_cast<float>(pl->mu);
        a.beta = beta;
        a.beta_prev = beta_prev;
        a.scene_map = n->d_map;
        a.tw = pl->d_tw1;
        a.nrows = na * n->L2;
        a.rows_per_scene = n->L2;
        beta_prev = beta;
        BCCB_TRY(kern(launch_row(n->L1, n->rcfgp, ROW_PRUNED, a, s)));
        continue;
      }
      BCCB_TRY(col(n, sparse ? COL_SPARSE_AFFINE : COL_FILTER_AFFINE, n->d_xy, na, n->d_coef_fista, nullptr,
                   n->d_map));
      RowArgs a;
      a.xy = n->d_xy;
      a.rhs = sparse ? nullptr : n->d_b;
      a.rhs_scale = static_cast<float>(n->plan->mu);
      a.state = n->d_c;
      a.kscale = n->d_tau;
      a.kappa = static_cast<float>(n->plan->mu);
      a.beta = beta;
      a.scene_map = n->d_map;
      BCCB_TRY(row(n, ROW_FISTA, a, na));
    }
    done_iters += steps;
    for (int i : act) used[i] = done_iters;
    if (resident) BCCB_TRY(read_residuals(act, rk));
    else BCCB_TRY(residuals(act, rk));
    std::vector<int> keep;
    for (int i : act)
      if (!(rk[i] <= kkt_target)) keep.push_back(i);
    if (keep.size() != act.size()) {
      act.swap(keep);
      BCCB_TRY(upload(act));
      BCCB_HIP(hipStreamSynchronize(s));
    }
  }
  BCCB_TRY(kern(launch_copy(reinterpret_cast<float2*>(c_out), n->d_c, static_cast<long>(batch) * n->L, s)));
  n->kkt_pruned = false;
  const int rc = finish(n);
  if (iters_out)
    for (int i = 0; i < batch; ++i) iters_out[i] = used[i];
  if (rkkt_out)
    for (int i = 0; i < batch; ++i) rkkt_out[i] = rk[i];
  if (rc != BCCB_OK) return rc;
  return act.empty() ? BCCB_OK : BCCB_W_NOT_CONVERGED;
}

}  // extern "C"
