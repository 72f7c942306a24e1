// Batched solves of many independent snapshots with uneven grids and masks.
//
// Scenes are grouped by grid size into classes; each class owns contiguous
// arenas so one row-pass launch and one column-pass launch per class cover all
// of its scenes per iteration, and the per-scene quantities (eigenvalues,
// step, threshold, snapshot and output pointers) are read from per-scene
// device arrays.  The whole iteration loop of a solve is one captured hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <numeric>
#include <vector>

#include "batch_layout.h"
#include "batch_resident.h"
#include "bccb.h"
#include "kernels.h"
#include "plan_internal.h"

using namespace bccb;

namespace {

struct BatchClass {
  int L1 = 0, L2 = 0, n = 0;
  long L = 0;
  std::vector<int> scenes;        // batch scene indices in arena order
  PassCfg cfg_row, cfg_col;
  const float2* tw1 = nullptr;    // twiddles, borrowed from a plan of the class
  const float2* tw2 = nullptr;
  float* d_omega = nullptr;       // [n][L]
  float2* d_coef = nullptr;       // [n] (1/L, -mu_s/L)
  float* d_kscale = nullptr;      // [n] mu_s * tau_s
  float2* d_xy = nullptr;         // [n][L]
  float2* d_rhs = nullptr;        // [n][L] mu_s * b_s
  float2* d_c = nullptr;          // [n][L] FISTA c^(t-1) -> c^(t)
  // pruned iteration (every scene has a kept-column set): kept row spectra
  // [n][L2][ncs], per-scene maps, c_t rotating over three SlotBufs [n][L2] / [n][L]
  bool can_prune = false, prune = false;
  int ncs = 0;
  float2* d_xyc = nullptr;
  int* d_scol = nullptr;          // [n][ncs] kept slot -> spectral column (-1 = padding)
  int* d_colslot = nullptr;       // [n][L1] spectral column -> kept slot (-1 = not kept)
  int* d_pcnt[3] = {nullptr, nullptr, nullptr};
  unsigned short* d_psidx[3] = {nullptr, nullptr, nullptr};
  float2* d_psval[3] = {nullptr, nullptr, nullptr};
  float2* d_pdense[3] = {nullptr, nullptr, nullptr};
  PassCfg cfg_rowp, cfg_colp;
  // FISTA iterate in per-row slots while the row is sparse (ROW_FISTA_SP)
  bool sp_iter = false;
  int* d_cnt = nullptr;           // [n][L2]
  unsigned short* d_sidx = nullptr;  // [n][L2][L1/8]
  float2* d_sval = nullptr;       // [n][L2][L1/8]
  SceneDesc* d_desc = nullptr;    // [n]
  // sparse spectral support of every scene, concatenated (see bccb_plan_s)
  bool sparse = false;
  int max_entries = 0;
  std::vector<int> entry_off;     // per scene
  int* d_sup_ptr = nullptr;       // [n][L1 + 1] global entry offsets
  SupEntry* d_sup = nullptr;
  int* d_src_ptr = nullptr;
  int* d_src = nullptr;
  float2* d_sup_rhs = nullptr;    // [total entries]
  SupRhsDesc* d_sdesc = nullptr;  // [n]
  SupRhsDesc* h_sdesc = nullptr;  // pinned [n]
};

}  // namespace

struct bccb_batch_s {
  int n = 0;
  hipStream_t stream = nullptr;
  std::vector<bccb_plan_t> plans;
  std::vector<BatchClass> cls;
  SceneDesc* h_desc = nullptr;    // pinned [n], class-arena order
  float* h_kscale = nullptr;      // pinned [n], class-arena order
  int* d_flag = nullptr;
  int* h_flag = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_iters = -1;
  // whole solves in one persistent launch (batch_resident.h), when every class is a
  // square support-column class of 32..256 points whose workgroup state fits in LDS
  bool res_ok = false, res_on = false;
  ResidentClass* d_rcls = nullptr;
  int res_ncls = 0, res_threads = 0, res_blocks = 0;
  size_t res_lds = 0;
  int* d_queue = nullptr;
  float* d_beta = nullptr;        // [beta_cap] momentum weights of the last iteration count
  float* h_beta = nullptr;        // pinned
  int beta_cap = 0;
};

namespace {

void batch_free(bccb_batch_s* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (BatchClass& c : b->cls) {
    for (void* p : {static_cast<void*>(c.d_omega), static_cast<void*>(c.d_coef), static_cast<void*>(c.d_kscale),
                    static_cast<void*>(c.d_xy), static_cast<void*>(c.d_rhs), static_cast<void*>(c.d_c),
                    static_cast<void*>(c.d_desc), static_cast<void*>(c.d_sup_ptr), static_cast<void*>(c.d_sup),
                    static_cast<void*>(c.d_src_ptr), static_cast<void*>(c.d_src), static_cast<void*>(c.d_sup_rhs),
                    static_cast<void*>(c.d_sdesc), static_cast<void*>(c.d_cnt), static_cast<void*>(c.d_sidx),
                    static_cast<void*>(c.d_sval)})
      if (p) (void)hipFree(p);
    if (c.h_sdesc) (void)hipHostFree(c.h_sdesc);
    for (void* p : {static_cast<void*>(c.d_xyc), static_cast<void*>(c.d_scol), static_cast<void*>(c.d_colslot)})
      if (p) (void)hipFree(p);
    for (int i = 0; i < 3; ++i)
      for (void* p : {static_cast<void*>(c.d_pcnt[i]), static_cast<void*>(c.d_psidx[i]),
                      static_cast<void*>(c.d_psval[i]), static_cast<void*>(c.d_pdense[i])})
        if (p) (void)hipFree(p);
  }
  if (b->d_flag) (void)hipFree(b->d_flag);
  if (b->h_flag) (void)hipHostFree(b->h_flag);
  for (void* p : {static_cast<void*>(b->d_rcls), static_cast<void*>(b->d_queue), static_cast<void*>(b->d_beta)})
    if (p) (void)hipFree(p);
  if (b->h_beta) (void)hipHostFree(b->h_beta);
  if (b->h_desc) (void)hipHostFree(b->h_desc);
  if (b->h_kscale) (void)hipHostFree(b->h_kscale);
  delete b;
}

template <typename T>
int dalloc(T** p, size_t n) {
  if (hipMalloc(reinterpret_cast<void**>(p), (n ? n : 1) * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return BCCB_E_NOMEM;
  }
  return BCCB_OK;
}

// Throughput-oriented default: E = 16 (fewest LDS exchanges), 256-thread blocks.
void default_batch_cfg(BatchClass& c) {
  c.cfg_row.E = c.L1 >= 16 ? 16 : 8;
  int Tr = c.L1 / c.cfg_row.E;
  c.cfg_row.rpb = std::max(1, 256 / Tr);
  while (!row_shape_ok(c.L1, c.cfg_row) && c.cfg_row.rpb > 1) c.cfg_row.rpb /= 2;
  c.cfg_col.E = c.L2 >= 16 ? 16 : 8;
  int Tc = c.L2 / c.cfg_col.E;
  c.cfg_col.W = std::min(c.L1, std::max(1, 256 / Tc));
  while (!col_shape_ok(c.L1, c.L2, c.cfg_col) && c.cfg_col.W > 1) c.cfg_col.W /= 2;
}

void default_pruned_cfg(BatchClass& c) {
  c.cfg_rowp.E = c.L1 >= 16 ? 16 : 8;
  const int Tr = c.L1 / c.cfg_rowp.E;
  c.cfg_rowp.rpb = std::max(1, 256 / Tr);
  while (!rowp_shape_ok(c.L1, c.cfg_rowp, c.ncs) && c.cfg_rowp.rpb > 1) c.cfg_rowp.rpb /= 2;
  c.cfg_colp.E = c.L2 >= 16 ? 16 : 8;
  const int Tc = c.L2 / c.cfg_colp.E;
  c.cfg_colp.W = std::min(c.ncs, std::max(1, 256 / Tc));
  while (!colp_shape_ok(c.ncs, c.L2, c.cfg_colp) && c.cfg_colp.W > 1) c.cfg_colp.W /= 2;
}

SlotBuf class_buf(const BatchClass& c, int i) {
  SlotBuf b;
  b.cnt = c.d_pcnt[i];
  b.sidx = c.d_psidx[i];
  b.sval = c.d_psval[i];
  b.dense = c.d_pdense[i];
  return b;
}

// Pruned-pass arguments over the class arenas: c_{t-1} in buffer i1, c_{t-2} in i2 (-1: none), c_t into i0.
RowArgs class_pruned_args(const BatchClass& c, int i0, int i1, int i2) {
  RowArgs a;
  a.xy = c.d_xyc;
  a.colslot = c.d_colslot;
  a.colslot_stride = c.L1;
  a.ncs = c.ncs;
  a.b0 = class_buf(c, i0);
  a.b1 = class_buf(c, i1);
  if (i2 >= 0) a.b2 = class_buf(c, i2);
  a.out_c = c.d_c;
  a.kscale = c.d_kscale;
  a.kappa = 1.f;
  return a;
}

int class_colp(const BatchClass& c, const PassCfg& cfg, hipStream_t s) {
  ColArgs a;
  a.xy = c.d_xyc;
  a.sup_ptr = c.d_sup_ptr;
  a.sup_ptr_stride = c.L1 + 1;
  a.sup = c.d_sup;
  a.sup_rhs = c.d_sup_rhs;
  a.coef = c.d_coef;
  a.tw = c.tw2;
  a.L1 = c.L1;
  a.nscenes = c.n;
  a.ncols = c.ncs;
  a.ldx = c.ncs;
  a.scol = c.d_scol;
  a.scol_stride = c.ncs;
  return kern(launch_col(c.L2, cfg, COL_PRUNED_AFFINE, a, s));
}

int class_row(const BatchClass& c, const PassCfg& cfg, int mode, RowArgs a, hipStream_t s) {
  a.tw = c.tw1;
  a.nrows = c.n * c.L2;
  a.rows_per_scene = c.L2;
  return kern(launch_row(c.L1, cfg, mode, a, s));
}

int class_col(const BatchClass& c, const PassCfg& cfg, int mode, float2* xy, float scale, hipStream_t s) {
  ColArgs a;
  a.xy = xy;
  a.sup_ptr = c.d_sup_ptr;
  a.sup_ptr_stride = c.L1 + 1;
  a.sup = c.d_sup;
  a.sup_rhs = c.d_sup_rhs;
  a.omega = c.d_omega;
  a.omega_stride = c.L;
  a.coef = c.d_coef;
  a.tw = c.tw2;
  a.L1 = c.L1;
  a.nscenes = c.n;
  a.scale = scale;
  return kern(launch_col(c.L2, cfg, mode, a, s));
}

// The iterations of one size class on stream s (classes share no buffers, so
// each can run its whole loop independently of the others).
int fista_loop_class(BatchClass& c, int iters, hipStream_t s) {
  double alpha = 1.0;
  float beta_prev = 0.f;
  for (int t = 1; t <= iters; ++t) {
    const double alpha_next = (1.0 + std::sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0;
    const float beta = static_cast<float>((alpha - 1.0) / alpha_next);
    alpha = alpha_next;
    {
      if (c.prune) {
        BCCB_TRY(class_colp(c, c.cfg_colp, s));
        RowArgs a = class_pruned_args(c, t % 3, (t - 1) % 3, (t + 1) % 3);
        a.beta = beta;
        a.beta_prev = beta_prev;
        a.last = (t == iters);
        BCCB_TRY(class_row(c, c.cfg_rowp, ROW_PRUNED, a, s));
        beta_prev = beta;
        continue;
      }
      BCCB_TRY(class_col(c, c.cfg_col, c.sparse ? COL_SPARSE_AFFINE : COL_FILTER_AFFINE, c.d_xy, 1.f, s));
      RowArgs a;
      a.xy = c.d_xy;
      a.rhs = c.sparse ? nullptr : c.d_rhs;
      a.state = c.d_c;
      a.out_c = c.d_c;
      a.cnt = c.d_cnt;
      a.sidx = c.d_sidx;
      a.sval = c.d_sval;
      a.kscale = c.d_kscale;
      a.kappa = 1.f;
      a.beta = beta;
      a.last = (t == iters);
      BCCB_TRY(class_row(c, c.cfg_row, c.sp_iter ? ROW_FISTA_SP : ROW_FISTA, a, s));
    }
    beta_prev = beta;
  }
  return BCCB_OK;
}

// The iterations of every class, one class after the other on stream s.
int fista_loop(bccb_batch_s* b, int iters, hipStream_t s) {
  for (BatchClass& c : b->cls) BCCB_TRY(fista_loop_class(c, iters, s));
  return BCCB_OK;
}

// The persistent whole-solve path: class table in queue order (larger grids first, so
// the last scenes taken are the short ones), and the workgroup size that keeps the most
// waves resident per compute unit.  Leaves res_ok false when some class does not fit.
int resident_setup(bccb_batch_s* b) {
  b->res_ok = b->res_on = false;
  std::vector<int> order(b->cls.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->cls[x].L > b->cls[y].L; });
  std::vector<ResidentClass> table;
  int first = 0;
  for (int ci : order) {
    const BatchClass& c = b->cls[ci];
    const bool len_ok = c.L1 == 32 || c.L1 == 64 || c.L1 == 128 || c.L1 == 256;
    if (!c.can_prune || c.L1 != c.L2 || !len_ok || c.ncs < 1) return BCCB_OK;
    ResidentClass r;
    r.N = c.L1;
    r.n = c.n;
    r.ncs = c.ncs;
    r.xs = c.ncs | 1;   // odd stride: a column's elements fall in different banks
    r.first = first;
    r.colslot = c.d_colslot;
    r.scol = c.d_scol;
    r.sup_ptr = c.d_sup_ptr;
    r.colslot_stride = c.L1;
    r.scol_stride = c.ncs;
    r.sup_ptr_stride = c.L1 + 1;   // entry offsets into the class's concatenated support
    r.sup = c.d_sup;
    r.sup_rhs = c.d_sup_rhs;
    r.coef = c.d_coef;
    r.kscale = c.d_kscale;
    r.tw = c.tw1;
    r.desc = c.d_desc;
    for (int i = 0; i < 3; ++i) r.buf[i] = class_buf(c, i);
    table.push_back(r);
    first += c.n;
  }
  if (table.empty()) return BCCB_OK;
  int best_waves = 0;
  for (int nt : {256, 512, 1024}) {
    long lds = 0;
    for (const ResidentClass& r : table) lds = std::max(lds, resident_lds_bytes(r.N, r.ncs, nt));
    const int nb = scene_fista_occupancy(nt, static_cast<size_t>(lds), 0);
    if (nb * (nt / 64) > best_waves) {
      best_waves = nb * (nt / 64);
      b->res_threads = nt;
      b->res_lds = static_cast<size_t>(lds);
      b->res_blocks = nb;
    }
  }
  if (best_waves == 0) return BCCB_OK;
  int dev = 0, cus = 0;
  BCCB_HIP(hipGetDevice(&dev));
  BCCB_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  b->res_blocks = std::max(1, std::min(first, b->res_blocks * std::max(cus, 1)));
  b->res_ncls = static_cast<int>(table.size());
  BCCB_TRY(dalloc(&b->d_rcls, table.size()));
  BCCB_TRY(dalloc(&b->d_queue, 1));
  BCCB_HIP(hipMemcpy(b->d_rcls, table.data(), table.size() * sizeof(ResidentClass), hipMemcpyHostToDevice));
  b->res_ok = b->res_on = true;
  return BCCB_OK;
}

// beta_t = (alpha_t - 1) / alpha_{t+1} for t = 1..iters (beta_0 = 0), as the graph loop forms them
int resident_betas(bccb_batch_s* b, int iters, hipStream_t s) {
  if (iters + 1 > b->beta_cap) {
    if (b->d_beta) (void)hipFree(b->d_beta);
    if (b->h_beta) (void)hipHostFree(b->h_beta);
    b->d_beta = nullptr;
    b->h_beta = nullptr;
    b->beta_cap = 0;
    BCCB_TRY(dalloc(&b->d_beta, iters + 1));
    if (hipHostMalloc(reinterpret_cast<void**>(&b->h_beta), (iters + 1) * sizeof(float)) != hipSuccess) {
      b->h_beta = nullptr;
      return BCCB_E_NOMEM;
    }
    b->beta_cap = iters + 1;
  }
  double alpha = 1.0;
  b->h_beta[0] = 0.f;
  for (int t = 1; t <= iters; ++t) {
    const double alpha_next = (1.0 + std::sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0;
    b->h_beta[t] = static_cast<float>((alpha - 1.0) / alpha_next);
    alpha = alpha_next;
  }
  BCCB_HIP(hipMemcpyAsync(b->d_beta, b->h_beta, (iters + 1) * sizeof(float), hipMemcpyHostToDevice, s));
  return BCCB_OK;
}

}  // namespace

extern "C" {

int bccb_batch_create(const bccb_plan_t* plans, int nscenes, void* stream, bccb_batch_t* out) {
  if (!plans || nscenes < 1 || !out) return BCCB_E_INVALID;
  *out = nullptr;
  for (int i = 0; i < nscenes; ++i) {
    if (!plans[i]) return BCCB_E_INVALID;
    if (plans[i]->emb) return BCCB_E_UNSUPPORTED;   // padded-embedding plans solve one scene at a time
  }
  bccb_batch_s* b = new (std::nothrow) bccb_batch_s();
  if (!b) return BCCB_E_NOMEM;
  b->n = nscenes;
  b->stream = static_cast<hipStream_t>(stream);
  b->plans.assign(plans, plans + nscenes);

  // host tables of every scene (views of the plans), and the size classes
  std::vector<std::pair<int, int>> grids(nscenes);
  std::vector<bccb_layout::SceneTables<SupEntry>> tables(nscenes);
  for (int i = 0; i < nscenes; ++i) {
    const bccb_plan_s* p = plans[i];
    grids[i] = std::make_pair(p->L1, p->L2);
    bccb_layout::SceneTables<SupEntry>& t = tables[i];
    t.L1 = p->L1;
    t.L2 = p->L2;
    t.sparse = sparse_on(p);
    t.sup_ptr = &p->h_sup_ptr;
    t.sup = &p->h_sup;
    t.src_ptr = &p->h_src_ptr;
    t.src = &p->h_src;
    t.prune_ok = p->prune_ok;
    t.nscol = p->nscol;
    t.scol = &p->h_scol;
  }
  for (const bccb_layout::Class& g : bccb_layout::group_by_grid(grids)) {
    BatchClass c;
    c.L1 = g.L1;
    c.L2 = g.L2;
    c.L = static_cast<long>(c.L1) * c.L2;
    c.tw1 = plans[g.scenes[0]]->d_tw1;
    c.tw2 = plans[g.scenes[0]]->d_tw2;
    c.scenes = g.scenes;
    b->cls.push_back(c);
  }
  int rc = BCCB_OK;
  for (BatchClass& c : b->cls) {
    c.n = static_cast<int>(c.scenes.size());
    if (c.n > 65535) rc = BCCB_E_UNSUPPORTED;
    default_batch_cfg(c);
    const size_t pts = static_cast<size_t>(c.n) * c.L;
    c.sparse = true;
    for (int k = 0; k < c.n; ++k) c.sparse = c.sparse && tables[c.scenes[k]].sparse;
    bccb_layout::Class members;
    members.L1 = c.L1;
    members.L2 = c.L2;
    members.scenes = c.scenes;
    if (rc == BCCB_OK && !c.sparse) rc = dalloc(&c.d_omega, pts);  // sparse classes read Omega from the lists
    if (rc == BCCB_OK) rc = dalloc(&c.d_coef, c.n);
    if (rc == BCCB_OK) rc = dalloc(&c.d_kscale, c.n);
    if (rc == BCCB_OK) rc = dalloc(&c.d_xy, pts);
    if (rc == BCCB_OK && !c.sparse) rc = dalloc(&c.d_rhs, pts);
    if (rc == BCCB_OK && c.sparse) {
      bccb_layout::ClassSupport<SupEntry> cs;
      if (!bccb_layout::concat_support(tables, members, &cs)) rc = BCCB_E_INVALID;
      const std::vector<int>& sp = cs.sup_ptr;
      const std::vector<int>& spp = cs.src_ptr;
      const std::vector<int>& src = cs.src;
      const std::vector<SupEntry>& sup = cs.sup;
      c.entry_off = cs.entry_off;
      c.max_entries = cs.max_entries;
      if (rc == BCCB_OK) rc = dalloc(&c.d_sup_ptr, sp.size());
      if (rc == BCCB_OK) rc = dalloc(&c.d_sup, sup.size());
      if (rc == BCCB_OK) rc = dalloc(&c.d_src_ptr, spp.size());
      if (rc == BCCB_OK) rc = dalloc(&c.d_src, src.size());
      if (rc == BCCB_OK) rc = dalloc(&c.d_sup_rhs, sup.size());
      if (rc == BCCB_OK) rc = dalloc(&c.d_sdesc, c.n);
      if (rc == BCCB_OK && hipHostMalloc(reinterpret_cast<void**>(&c.h_sdesc), c.n * sizeof(SupRhsDesc)) != hipSuccess)
        rc = BCCB_E_NOMEM;
      if (rc == BCCB_OK &&
          (hipMemcpy(c.d_sup_ptr, sp.data(), sp.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
           hipMemcpy(c.d_sup, sup.data(), sup.size() * sizeof(SupEntry), hipMemcpyHostToDevice) != hipSuccess ||
           hipMemcpy(c.d_src_ptr, spp.data(), spp.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
           hipMemcpy(c.d_src, src.data(), src.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess))
        rc = BCCB_E_DEVICE;
    }
    if (rc == BCCB_OK) rc = dalloc(&c.d_c, pts);
    if (rc == BCCB_OK) rc = dalloc(&c.d_desc, c.n);
    if (c.L1 >= 8) {
      const size_t rows = static_cast<size_t>(c.n) * c.L2;
      if (rc == BCCB_OK) rc = dalloc(&c.d_cnt, rows);
      if (rc == BCCB_OK) rc = dalloc(&c.d_sidx, rows * (c.L1 / 8));
      if (rc == BCCB_OK) rc = dalloc(&c.d_sval, rows * (c.L1 / 8));
      // every row starts out dense: no slot is read before the kernel has written it
      if (rc == BCCB_OK && hipMemset(c.d_cnt, 0x7f, rows * sizeof(int)) != hipSuccess) rc = BCCB_E_DEVICE;
      c.sp_iter = true;
      while (!row_shape_ok(c.L1, c.cfg_row, true) && c.cfg_row.rpb > 1) c.cfg_row.rpb /= 2;
    }
    bccb_layout::KeptColumns kc;
    c.can_prune = c.sparse && bccb_layout::kept_columns(tables, members, &kc) && kc.ncs <= c.L1 / 2;
    if (c.can_prune) c.ncs = kc.ncs;
    if (rc == BCCB_OK && c.can_prune) {
      const size_t rows = static_cast<size_t>(c.n) * c.L2;
      const std::vector<int>& scol = kc.scol;
      const std::vector<int>& colslot = kc.colslot;
      rc = dalloc(&c.d_xyc, rows * c.ncs);
      if (rc == BCCB_OK) rc = dalloc(&c.d_scol, scol.size());
      if (rc == BCCB_OK) rc = dalloc(&c.d_colslot, colslot.size());
      for (int i = 0; i < 3 && rc == BCCB_OK; ++i) {
        rc = dalloc(&c.d_pcnt[i], rows);
        // L1/8 slots per row for the passes, L1/kResidentSlotDiv for the persistent solve
        if (rc == BCCB_OK) rc = dalloc(&c.d_psidx[i], rows * (c.L1 / kResidentSlotDiv));
        if (rc == BCCB_OK) rc = dalloc(&c.d_psval[i], rows * (c.L1 / kResidentSlotDiv));
        if (rc == BCCB_OK) rc = dalloc(&c.d_pdense[i], pts);
        // rows start out dense over a zeroed grid: nothing unwritten is ever read
        if (rc == BCCB_OK && (hipMemset(c.d_pcnt[i], 0x7f, rows * sizeof(int)) != hipSuccess ||
                              hipMemset(c.d_pdense[i], 0, pts * sizeof(float2)) != hipSuccess))
          rc = BCCB_E_DEVICE;
      }
      if (rc == BCCB_OK && (hipMemcpy(c.d_scol, scol.data(), scol.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
                            hipMemcpy(c.d_colslot, colslot.data(), colslot.size() * sizeof(int),
                                      hipMemcpyHostToDevice) != hipSuccess ||
                            hipMemset(c.d_xyc, 0, rows * c.ncs * sizeof(float2)) != hipSuccess))
        rc = BCCB_E_DEVICE;
      c.prune = true;
      default_pruned_cfg(c);
    }
    if (rc != BCCB_OK) break;
    std::vector<float2> coef(c.n);
    for (int k = 0; k < c.n; ++k) {
      const bccb_plan_s* p = plans[c.scenes[k]];
      coef[k] = make_float2(static_cast<float>(1.0 / static_cast<double>(c.L)),
                            static_cast<float>(-p->mu / static_cast<double>(c.L)));
      if (!c.sparse && hipMemcpyAsync(c.d_omega + static_cast<size_t>(k) * c.L, p->d_omega, c.L * sizeof(float),
                         hipMemcpyDeviceToDevice, b->stream) != hipSuccess) {
        rc = BCCB_E_DEVICE;
        break;
      }
    }
    if (rc == BCCB_OK && hipMemcpy(c.d_coef, coef.data(), c.n * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess)
      rc = BCCB_E_DEVICE;
    if (rc != BCCB_OK) break;
  }
  if (rc == BCCB_OK) rc = resident_setup(b);
  if (rc == BCCB_OK) rc = dalloc(&b->d_flag, 1);
  if (rc == BCCB_OK && (hipHostMalloc(reinterpret_cast<void**>(&b->h_flag), sizeof(int)) != hipSuccess ||
                        hipHostMalloc(reinterpret_cast<void**>(&b->h_desc), nscenes * sizeof(SceneDesc)) != hipSuccess ||
                        hipHostMalloc(reinterpret_cast<void**>(&b->h_kscale), nscenes * sizeof(float)) != hipSuccess))
    rc = BCCB_E_NOMEM;
  if (rc == BCCB_OK && hipStreamSynchronize(b->stream) != hipSuccess) rc = BCCB_E_DEVICE;
  if (rc != BCCB_OK) {
    batch_free(b);
    return rc;
  }
  *out = b;
  return BCCB_OK;
}

int bccb_batch_destroy(bccb_batch_t b) {
  if (b) (void)hipStreamSynchronize(b->stream);
  batch_free(b);
  return BCCB_OK;
}

int bccb_batch_info(bccb_batch_t b, int* nclasses, int* L1, int* L2, int* count) {
  if (!b) return BCCB_E_INVALID;
  if (nclasses) *nclasses = static_cast<int>(b->cls.size());
  for (size_t i = 0; i < b->cls.size(); ++i) {
    if (L1) L1[i] = b->cls[i].L1;
    if (L2) L2[i] = b->cls[i].L2;
    if (count) count[i] = b->cls[i].n;
  }
  return BCCB_OK;
}

int lasso_solve_batch_fista(bccb_batch_t b, const bccb_c32* const* y, const float* tau, int iters,
                            bccb_c32* const* c_out) {
  if (!b || !y || !tau || !c_out || iters < 0) return BCCB_E_INVALID;
  for (int i = 0; i < b->n; ++i) {
    if (!y[i] || !c_out[i] || !(tau[i] >= 0.f) || !std::isfinite(tau[i])) return BCCB_E_INVALID;
  }
  hipStream_t s = b->stream;
  BCCB_HIP(hipMemsetAsync(b->d_flag, 0, sizeof(int), s));
  // per-scene descriptors and thresholds, in class-arena order
  int off = 0;
  for (BatchClass& c : b->cls) {
    for (int k = 0; k < c.n; ++k) {
      const int i = c.scenes[k];
      const bccb_plan_s* p = b->plans[i];
      SceneDesc& d = b->h_desc[off + k];
      d.y = reinterpret_cast<const float2*>(y[i]);
      d.sensor_of = p->d_sensor_of;
      d.out = reinterpret_cast<float2*>(c_out[i]);
      d.M1 = p->M1;
      d.M2 = p->M2;
      d.scale = static_cast<float>(p->mu);
      b->h_kscale[off + k] = static_cast<float>(p->mu * tau[i]);
    }
    BCCB_HIP(hipMemcpyAsync(c.d_desc, b->h_desc + off, c.n * sizeof(SceneDesc), hipMemcpyHostToDevice, s));
    BCCB_HIP(hipMemcpyAsync(c.d_kscale, b->h_kscale + off, c.n * sizeof(float), hipMemcpyHostToDevice, s));
    off += c.n;
  }
  bool resident = b->res_on && iters > 0;
  for (const BatchClass& c : b->cls) resident = resident && c.prune;   // the support-column form is on
  // mu_s * b_s = mu_s * D_s^H y_s for every scene (spectral support bins, or a grid);
  // c^(0) = 0, DFT_rows(z^(1)) = 0 (the persistent launch starts every scene from these itself)
  off = 0;
  for (BatchClass& c : b->cls) {
    if (c.sparse) {
      for (int k = 0; k < c.n; ++k) {
        const bccb_plan_s* p = b->plans[c.scenes[k]];
        SupRhsDesc& d = c.h_sdesc[k];
        d.y = b->h_desc[off + k].y;
        d.entry_off = c.entry_off[k];
        d.nentries = p->nsup;
        d.rhs_off = c.entry_off[k];
        d.scale = static_cast<float>(p->mu);
      }
      BCCB_HIP(hipMemcpyAsync(c.d_sdesc, c.h_sdesc, c.n * sizeof(SupRhsDesc), hipMemcpyHostToDevice, s));
      BCCB_TRY(kern(launch_sup_rhs(c.d_sdesc, c.n, c.max_entries, c.d_src_ptr, c.d_src, c.d_sup_rhs, b->d_flag, s)));
    } else {
      BCCB_TRY(kern(launch_scatter_batch(c.d_desc, c.n, c.L1, c.L2, c.d_xy, b->d_flag, s)));
      BCCB_TRY(class_col(c, c.cfg_col, COL_INV, c.d_xy, 1.f, s));
      RowArgs a;
      a.xy = c.d_xy;
      a.dst = c.d_rhs;
      BCCB_TRY(class_row(c, c.cfg_row, ROW_INV, a, s));
    }
    off += c.n;
    if (resident) continue;
    BCCB_TRY(kern(launch_fill(c.d_c, static_cast<long>(c.n) * c.L, s)));
    BCCB_TRY(kern(launch_fill(c.d_xy, static_cast<long>(c.n) * c.L, s)));
    if (c.sp_iter) BCCB_TRY(kern(launch_fill_int(c.d_cnt, static_cast<long>(c.n) * c.L2, c.L1 + 1, s)));
    if (c.prune) {
      // c_0 = c_{-1} = 0 (empty rows); the kept row spectra of z_1 = 0
      BCCB_TRY(kern(launch_fill_int(c.d_pcnt[0], static_cast<long>(c.n) * c.L2, 0, s)));
      BCCB_TRY(kern(launch_fill_int(c.d_pcnt[2], static_cast<long>(c.n) * c.L2, 0, s)));
      BCCB_TRY(kern(launch_fill(c.d_xyc, static_cast<long>(c.n) * c.L2 * c.ncs, s)));
    }
  }
  if (resident) {
    BCCB_TRY(resident_betas(b, iters, s));
    BCCB_TRY(kern(launch_fill_int(b->d_queue, 1, 0, s)));
    BCCB_TRY(kern(launch_scene_fista(b->d_rcls, b->res_ncls, b->n, b->d_beta, 0, iters, 0, 0, b->d_queue,
                                     b->res_threads, b->res_blocks, b->res_lds, s)));
  } else if (iters > 0) {
    if (!b->exec || b->graph_iters != iters) {
      if (b->exec) (void)hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
      if (!b->cap_stream && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        b->cap_stream = nullptr;
        return BCCB_E_DEVICE;
      }
      BCCB_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
      const int rc = fista_loop(b, iters, b->cap_stream);
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(b->cap_stream, &g);
      if (rc != BCCB_OK || ec != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc != BCCB_OK ? rc : BCCB_E_DEVICE;
      }
      const hipError_t ei = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) {
        b->exec = nullptr;
        return BCCB_E_DEVICE;
      }
      b->graph_iters = iters;
    }
    BCCB_HIP(hipGraphLaunch(b->exec, s));
  }
  if (!resident)
    for (BatchClass& c : b->cls) BCCB_TRY(kern(launch_gather_batch(c.d_desc, c.n, c.L, c.d_c, s)));
  BCCB_HIP(hipMemcpyAsync(b->h_flag, b->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  BCCB_HIP(hipStreamSynchronize(s));
  return *b->h_flag ? BCCB_E_NONFINITE : BCCB_OK;
}

int bccb_batch_autotune(bccb_batch_t b, int reps) {
  if (!b || reps < 1) return BCCB_E_INVALID;
  const int Es[4] = {4, 8, 16, 32};
  for (BatchClass& c : b->cls) {
    float best_r = 1e30f, best_c = 1e30f, best_rp = 1e30f, best_cp = 1e30f;
    PassCfg br = c.cfg_row, bc = c.cfg_col, brp = c.cfg_rowp, bcp = c.cfg_colp;
    for (int E : Es) {
      for (int k = 1; k <= 256; k *= 2) {
        PassCfg r;
        r.E = E;
        r.rpb = k;
        if (row_shape_ok(c.L1, r, c.sp_iter)) {
          RowArgs a;
          a.xy = c.d_xy;
          a.rhs = c.sparse ? nullptr : c.d_rhs;
          a.state = c.d_c;
          a.cnt = c.d_cnt;
          a.sidx = c.d_sidx;
          a.sval = c.d_sval;
          a.kscale = c.d_kscale;
          a.kappa = 1.f;
          a.beta = 0.5f;
          const int mode = c.sp_iter ? ROW_FISTA_SP : ROW_FISTA;
          const float ms = time_launches(b->stream, reps, [&] { return class_row(c, r, mode, a, b->stream); });
          if (ms < 0.f) return BCCB_E_DEVICE;
          if (ms < best_r) { best_r = ms; br = r; }
        }
        if (c.can_prune && rowp_shape_ok(c.L1, r, c.ncs)) {
          // timed on the state most iterations see: rows of c_{t-1}, c_{t-2} in slot form
          const long rows = static_cast<long>(c.n) * c.L2;
          if (kern(launch_fill_int(c.d_pcnt[1], rows, 4, b->stream)) != BCCB_OK ||
              kern(launch_fill_int(c.d_pcnt[2], rows, 4, b->stream)) != BCCB_OK)
            return BCCB_E_DEVICE;
          RowArgs a = class_pruned_args(c, 0, 1, 2);
          a.beta = a.beta_prev = 0.5f;
          const float ms = time_launches(b->stream, reps, [&] { return class_row(c, r, ROW_PRUNED, a, b->stream); });
          if (ms < 0.f) return BCCB_E_DEVICE;
          if (ms < best_rp) { best_rp = ms; brp = r; }
        }
        PassCfg w;
        w.E = E;
        w.W = k;
        if (c.can_prune && colp_shape_ok(c.ncs, c.L2, w)) {
          const float ms = time_launches(b->stream, reps, [&] { return class_colp(c, w, b->stream); });
          if (ms < 0.f) return BCCB_E_DEVICE;
          if (ms < best_cp) { best_cp = ms; bcp = w; }
        }
        if (col_shape_ok(c.L1, c.L2, w)) {
          const int cm = c.sparse ? COL_SPARSE_AFFINE : COL_FILTER_AFFINE;
          const float ms = time_launches(b->stream, reps, [&] { return class_col(c, w, cm, c.d_xy, 1.f, b->stream); });
          if (ms < 0.f) return BCCB_E_DEVICE;
          if (ms < best_c) { best_c = ms; bc = w; }
        }
      }
    }
    c.cfg_row = br;
    c.cfg_col = bc;
    c.cfg_rowp = brp;
    c.cfg_colp = bcp;
  }
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  b->graph_iters = -1;
  return BCCB_OK;
}

int bccb_batch_class_config(bccb_batch_t b, int cls, int* cfg) {
  if (!b || !cfg || cls < 0 || cls >= static_cast<int>(b->cls.size())) return BCCB_E_INVALID;
  const BatchClass& c = b->cls[cls];
  const PassCfg& r = c.prune ? c.cfg_rowp : c.cfg_row;
  const PassCfg& w = c.prune ? c.cfg_colp : c.cfg_col;
  cfg[0] = r.E;
  cfg[1] = r.rpb;
  cfg[2] = w.E;
  cfg[3] = w.W;
  cfg[4] = c.prune ? 1 : 0;
  cfg[5] = c.prune ? c.ncs : c.L1;
  return BCCB_OK;
}

int bccb_batch_set_support_columns(bccb_batch_t b, int on) {
  if (!b || (on != 0 && on != 1)) return BCCB_E_INVALID;
  for (BatchClass& c : b->cls) c.prune = on == 1 && c.can_prune;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  b->graph_iters = -1;
  return BCCB_OK;
}

int bccb_batch_set_resident(bccb_batch_t b, int on) {
  if (!b || (on != 0 && on != 1 && on != 256 && on != 512 && on != 1024)) return BCCB_E_INVALID;
  if (on != 0 && !b->res_ok) return BCCB_E_UNSUPPORTED;
  if (on > 1) {
    // a given workgroup size: its LDS and the grid it keeps resident
    long lds = 0;
    std::vector<ResidentClass> table(b->res_ncls);
    BCCB_HIP(hipMemcpy(table.data(), b->d_rcls, table.size() * sizeof(ResidentClass), hipMemcpyDeviceToHost));
    for (const ResidentClass& r : table) lds = std::max(lds, resident_lds_bytes(r.N, r.ncs, on));
    const int nb = scene_fista_occupancy(on, static_cast<size_t>(lds), 0);
    if (nb < 1) return BCCB_E_UNSUPPORTED;
    int dev = 0, cus = 0;
    BCCB_HIP(hipGetDevice(&dev));
    BCCB_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    b->res_threads = on;
    b->res_lds = static_cast<size_t>(lds);
    b->res_blocks = std::max(1, std::min(b->n, nb * std::max(cus, 1)));
  }
  b->res_on = on != 0;
  return BCCB_OK;
}

int bccb_batch_resident_info(bccb_batch_t b, int* on, int* threads, int* blocks, int* lds_bytes) {
  if (!b) return BCCB_E_INVALID;
  if (on) *on = b->res_on ? 1 : (b->res_ok ? 0 : -1);
  if (threads) *threads = b->res_ok ? b->res_threads : 0;
  if (blocks) *blocks = b->res_ok ? b->res_blocks : 0;
  if (lds_bytes) *lds_bytes = b->res_ok ? static_cast<int>(b->res_lds) : 0;
  return BCCB_OK;
}

int bccb_batch_set_sparse_iterate(bccb_batch_t b, int on) {
  if (!b || (on != 0 && on != 1)) return BCCB_E_INVALID;
  for (BatchClass& c : b->cls) {
    const bool want = on == 1 && c.d_cnt != nullptr;
    while (want && !row_shape_ok(c.L1, c.cfg_row, true) && c.cfg_row.rpb > 1) c.cfg_row.rpb /= 2;
    c.sp_iter = want;
  }
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  b->graph_iters = -1;
  return BCCB_OK;
}

}  // extern "C"
