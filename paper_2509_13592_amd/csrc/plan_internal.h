// Internal layout of a bccb plan (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "bccb.h"
#include "kernels.h"
#include "resident_api.h"
#include "plan_math.h"

struct bccb_plan_s {
  int M1 = 0, M2 = 0, L1 = 0, L2 = 0, M = 0;
  long L = 0;
  double mu = 0.0;                 // 1 / max(Omega)
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<float> omega32;      // host copy of the FP32 eigenvalue grid [L2][L1]
  std::vector<uint8_t> mask;       // host copy of the array mask [M2][M1]

  float* d_omega = nullptr;        // [L2][L1] eigenvalues (eq. (21)), FP32
  int* d_sensor_of = nullptr;      // [M2][M1] index into y, or -1
  int2* d_sensors = nullptr;       // [M] (m1, m2) in increasing m1 + m2*M1
  float2* d_tw1 = nullptr;         // [L1] e^{-j 2 pi j / L1}
  float2* d_tw2 = nullptr;         // [L2]
  float2* d_xy = nullptr;          // [L] row-spectral iterate (in-place passes)
  float2* d_rhs = nullptr;         // [L] mu*b, w, or b
  float2* d_state = nullptr;       // [L] ADMM v / scratch
  float2* d_tmp = nullptr;         // [L] spectral scratch
  float2* d_coef = nullptr;        // [2] (1/L, -mu/L) and (0, 1/L)
  double* d_red = nullptr;         // reduction partials
  int* d_flag = nullptr;           // non-finite input flag
  double* h_red = nullptr;         // pinned host copy of the partials
  int* h_flag = nullptr;           // pinned host copy of the flag

  // sparse spectral support of Omega (the folded array elements): per column k1 the
  // bins sup[sup_ptr[k1] .. sup_ptr[k1+1]), and for each bin the snapshot entries
  // folding onto it, src[src_ptr[j] .. src_ptr[j+1]) = (sensor << 1) | sign bit
  int nsup = 0;
  bool has_support = false;
  std::vector<int> h_sup_ptr, h_src_ptr, h_src;
  std::vector<bccb::SupEntry> h_sup;
  int* d_sup_ptr = nullptr;
  bccb::SupEntry* d_sup = nullptr;
  int* d_src_ptr = nullptr;
  int* d_src = nullptr;
  float2* d_sup_rhs = nullptr;     // [nsup] per solve
  bccb::SupRhsDesc* d_sup_desc = nullptr;
  bccb::SupRhsDesc* h_sup_desc = nullptr;  // pinned
  int use_support = 1;

  // FISTA iterate kept per row as (index, value) slots while the row is sparse
  // (ROW_FISTA_SP): count [L2], slots [L2][L1/8]
  int sparse_iterate = 0;
  int* d_cnt = nullptr;
  unsigned short* d_sidx = nullptr;
  float2* d_sval = nullptr;

  // pruned iteration (sparse support): the spectral columns holding support bins,
  // padded to ncs (a multiple of 4) with -1; colslot[k1] = position of k1 or -1;
  // xyc [L2][ncs] the kept row spectra; c_t rotates over three SlotBufs
  std::vector<int> h_scol;
  int nscol = 0, ncs = 0;
  bool prune_ok = false;
  int use_prune = 1;
  int* d_scol = nullptr;
  int* d_colslot = nullptr;
  float2* d_xyc = nullptr;
  int* d_pcnt[3] = {nullptr, nullptr, nullptr};
  unsigned short* d_psidx[3] = {nullptr, nullptr, nullptr};
  float2* d_psval[3] = {nullptr, nullptr, nullptr};
  float2* d_pdense[3] = {nullptr, nullptr, nullptr};
  bccb::PassCfg cfg_rowp, cfg_colp;

  // single-scene cooperative solver (resident.h): groups > 0 turns it on for ISTA,
  // FISTA and ADMM when the spectral support is in use; FISTA momenta beta_t in
  // d_beta[t - 1] (capacity beta_cap); d_sync = abort and arrival words
  int resident_groups = 0;
  int resident_spread = 1;
  float* d_beta = nullptr;
  int beta_cap = 0;
  unsigned long long* d_sync = nullptr;
  unsigned long long res_solve = 0;   // cooperative solves enqueued so far (their tags)
  long long wall_ticks_per_s = 0;
  float2* d_rpart = nullptr;       // pruned form: [2][groups][nsup] per-group parts of DFT2 at the bins
  float2* d_psi = nullptr;         // pruned ADMM passes: [nsup] support part Psi of the scaled dual
  float2* d_vlast = nullptr;       // pruned ADMM passes: [nsup] the last column pass's V' per bin
  int resident_block = 256;        // threads per group of the pruned cooperative form (256 or 512)
  int res_pruned_spread = -1;      // spread and block the cached pruned-form check was made for
  int res_pruned_block = -1;
  bool res_pruned_ok = false;

  bccb::PassCfg cfg_row;           // launch shape of the row passes (N = L1)
  bccb::PassCfg cfg_col;           // launch shape of the column passes (N = L2)
  int use_graph = 1;

  // plans on a zero-padded embedding (bccb_plan_spaced): the caller's grid is A1 x A2 and
  // sits in the leading window of the L1 x L2 transform grid (L_i >= 2 A_i - 1, powers of
  // two); d_omega holds the eigenvalues of the circulant embedding of the Gram, and the row
  // pass keeps every element outside the window at zero
  bool emb = false;
  int A1 = 0, A2 = 0;
  long AL = 0;
  double gamma1 = 0.5, gamma2 = 0.5;
  bool emb_circulant = false;      // gamma = 1/2 on both axes: G is the A1 x A2 BCCB (ADMM available)
  std::vector<double> emb_omega;   // circulant: the A1 x A2 eigenvalue grid of G (eq. (21))
  float2* d_W1 = nullptr;          // [M1][A1] e^{-j 2 pi f_{1,l} m1}
  float2* d_W2 = nullptr;          // [M2][A2]
  float2* d_emb_u = nullptr;       // separable-product scratch, max(M2 A1, A2 M1)
  float2* d_emb_c = nullptr;       // [L] padded iterate (c^(t-1), or the ADMM z)
  float2* d_emb_c2 = nullptr;      // [L] padded ADMM c
  float* d_omega_rho = nullptr;    // [L] eigenvalues of the embedding of (G + rho I)^-1
  float2* d_emb_coef = nullptr;    // [2] multiplier coefficients of the ADMM passes
  float emb_rho = -1.f;            // rho d_omega_rho was built for

  // FP64 passes (solve_f64.cpp), allocated on the first FP64 call: eigenvalues, twiddles, grids
  double* d_omega64 = nullptr;
  double2* d_tw1_64 = nullptr;
  double2* d_tw2_64 = nullptr;
  double2* d_xy64 = nullptr;
  double2* d_rhs64 = nullptr;
  double2* d_state64 = nullptr;

  // peak extraction (bccb_extract_peaks): candidate keys [cand_batch][4096] and counts
  unsigned long long* d_cand = nullptr;
  int* d_ccount = nullptr;
  int cand_batch = 0;

  // one cached hipGraph of a solve's iteration loop, replayed while its key repeats
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  unsigned long long graph_key[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

#define BCCB_TRY(expr)              \
  do {                              \
    const int _rc = (expr);         \
    if (_rc != BCCB_OK) return _rc; \
  } while (0)
#define BCCB_HIP(expr)                              \
  do {                                              \
    if ((expr) != hipSuccess) return BCCB_E_DEVICE; \
  } while (0)

namespace bccb {

// kernel-launcher return code -> status
inline int kern(int rc) { return rc == 0 ? BCCB_OK : (rc == -2 ? BCCB_E_UNSUPPORTED : BCCB_E_DEVICE); }

bool elems_ok(int N, int E);
int adjoint_into(bccb_plan_s* p, const float2* y, float scale, float2* dst);
bool sparse_on(const bccb_plan_s* p);
int begin_call(bccb_plan_s* p);
int end_call(bccb_plan_s* p);
bool row_shape_ok(int L1, const PassCfg& c, bool sparse_iterate = false);
bool col_shape_ok(int L1, int L2, const PassCfg& c);
bool rowp_shape_ok(int L1, const PassCfg& c, int ncs);    // pruned row pass over ncs kept columns
bool colp_shape_ok(int ncs, int L2, const PassCfg& c);    // pruned column pass over ncs columns
bool pruned_on(const bccb_plan_s* p);
bool resident_on(const bccb_plan_s* p);
void default_config(bccb_plan_s* p);
void drop_graph(bccb_plan_s* p);
void plan_free(bccb_plan_s* p);
int row_pass_on(bccb_plan_s* p, const PassCfg& cfg, int mode, RowArgs a, hipStream_t s);
int col_pass_on(bccb_plan_s* p, const PassCfg& cfg, int mode, float2* xy, const float2* coef, float rho,
                float scale, hipStream_t s);
int row_pass(bccb_plan_s* p, int mode, RowArgs a);
int col_pass(bccb_plan_s* p, int mode, float2* xy, const float2* coef, float rho, float scale);

// Run `enqueue` (the iteration loop of a solve) on the plan's stream, through a
// cached hipGraph when enabled: the loop is captured on a private stream (the
// plan's stream may be the null stream, which cannot capture) and replayed
// while the key -- every argument the captured launches depend on -- repeats.
template <typename F>
int run_loop(bccb_plan_s* p, const unsigned long long (&key)[8], F&& enqueue) {
  if (!p->use_graph) return enqueue(p->stream);
  bool hit = p->graph_exec != nullptr;
  for (int i = 0; i < 8 && hit; ++i) hit = p->graph_key[i] == key[i];
  if (!hit) {
    drop_graph(p);
    if (!p->cap_stream && hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess) {
      p->cap_stream = nullptr;
      return BCCB_E_DEVICE;
    }
    if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return BCCB_E_DEVICE;
    const int rc = enqueue(p->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(p->cap_stream, &g);
    if (rc != BCCB_OK || ec != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return rc != BCCB_OK ? rc : BCCB_E_DEVICE;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return BCCB_E_DEVICE;
    p->graph_exec = ex;
    for (int i = 0; i < 8; ++i) p->graph_key[i] = key[i];
  }
  BCCB_HIP(hipGraphLaunch(p->graph_exec, p->stream));
  return BCCB_OK;
}

inline unsigned long long fbits(float f) {
  unsigned int u;
  std::memcpy(&u, &f, sizeof(u));
  return u;
}

// Time `reps` launches of `launch()` on stream s with hipEvents; ms per launch, or < 0 on error.
template <typename F>
float time_launches(hipStream_t s, int reps, F&& launch) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.f;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return -1.f; }
  float ms = -1.f;
  bool ok = launch() == 0;                                   // warm-up
  ok = ok && hipEventRecord(e0, s) == hipSuccess;
  for (int i = 0; i < reps && ok; ++i) ok = launch() == 0;
  ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
       hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ok ? ms / reps : -1.f;
}

}  // namespace bccb

namespace bccb {
// FP64 first column of the plan's Gram (eq. (17), property (iv) of Sec. III-A)
inline std::vector<cd> gram_first_column_plan(const bccb_plan_s* p) {
  return gram_first_column(p->mask.data(), p->M1, p->M2, p->L1, p->L2);
}
}  // namespace bccb
