// Host-side launch interface of the BCCB kernels (internal to libbccb).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace bccb {

// Row pass (transforms along l1, the contiguous axis of a [rows][L1] grid).
enum RowMode {
  ROW_FWD = 0,    // xy = DFT_rows(src)                (src == nullptr -> zeros)
  ROW_INV = 1,    // dst = scale * IDFT_rows(xy)
  ROW_ISTA = 2,   // u = IDFT_rows(xy); c = S_k(u + rhs); xy = DFT_rows(c)
  ROW_FISTA = 3,  // u = IDFT_rows(xy); c = S_k(u + rhs); z = c + beta (c - state); state = c; xy = DFT_rows(z)
  ROW_ADMM = 4,   // u = IDFT_rows(xy); c = rhs + u; z = S_k(c + v); v += c - z; xy = DFT_rows(z - v)
  ROW_FISTA_SP = 5,  // ROW_FISTA with c_{t-1} / c_t kept per row as (index, value) slots while the row
                     // has at most N/8 nonzeros (dense row in `state` otherwise; always dense at the last iteration)
  // Pruned forms for a sparse spectral support: the row spectra exchanged with the
  // column pass hold only the support columns, compact as [row][ncs] (spectral
  // column k1 at slot colslot[k1], -1 = not kept), and carry only the correction
  // -mu G z_t + mu b; the identity part z_t is rebuilt in the spatial domain.
  ROW_PRUNED_FWD = 6,  // xy[:, kept] = DFT_rows(src)[:, kept]   (src == nullptr -> zeros)
  ROW_PRUNED = 7,      // z = c1 + beta_prev (c1 - c2); u = z + IDFT_rows(xy); c = S_k(u) -> b0;
                       // xy[:, kept] = DFT_rows(c + beta (c - c1))[:, kept]
};

// An iterate stored per row as (index, value) slots while the row has at most
// N/8 nonzeros, as the dense row otherwise: cnt[row] <= N/8 -> slots
// sidx/sval[row * (N/8) + j], j < cnt; cnt[row] > N/8 -> dense[row * N + l].
struct SlotBuf {
  int* cnt = nullptr;
  unsigned short* sidx = nullptr;
  float2* sval = nullptr;
  float2* dense = nullptr;
};

struct RowArgs {
  float2* xy = nullptr;          // [nrows][N] row-spectral buffer, read and written in place
  const float2* src = nullptr;   // ROW_FWD input rows
  float2* dst = nullptr;         // ROW_INV output rows
  const float2* rhs = nullptr;   // mu*b (ISTA/FISTA) or w = (G + rho I)^-1 b (ADMM)
  float2* state = nullptr;       // c_{t-1} -> c_t (FISTA) or v (ADMM)
  float2* out_z = nullptr;       // ADMM: z at the last iteration
  float2* out_c = nullptr;       // ISTA: c at the last iteration; ADMM: c at the last iteration (nullable)
  const float2* tw = nullptr;    // [N] e^{-j 2 pi j / N}
  const float* kscale = nullptr; // per-scene multiplier of kappa (nullable = 1)
  int* flag = nullptr;           // set to 1 if a non-finite input is seen (ROW_FWD)
  int nrows = 0;                 // total rows over all scenes
  int rows_per_scene = 1;
  float kappa = 0.f, beta = 0.f, scale = 1.f;
  int last = 0;                  // last iteration: write the outputs, skip the forward DFT
  float rhs_scale = 1.f;         // ISTA/FISTA: u + rhs_scale * rhs
  const float* dscal = nullptr;  // device {kappa, rhs_scale} overriding the two scalars (nullable)
  float2* save_u = nullptr;      // FISTA: store u = IDFT_rows(xy) + rhs_scale*rhs (nullable)
  float2* save_c = nullptr;      // FISTA: store c_t (nullable)
  float2* out_prev = nullptr;    // FISTA: store c_{t-1} (the state before the update) (nullable)
  const int* scene_map = nullptr;// logical scene -> physical scene of the arenas (nullable = identity)
  int spread = 1;                // see PassCfg::spread
  // ROW_FISTA_SP storage: per physical row, cnt = number of nonzeros (> N/8: the row is dense in
  // `state`), slot j < cnt holds element sidx[row * (N/8) + j] with value sval[row * (N/8) + j]
  int* cnt = nullptr;
  unsigned short* sidx = nullptr;
  float2* sval = nullptr;
  // ROW_PRUNED*: kept-column map [scene][N] (scene stride colslot_stride), compact row length
  // ncs of xy, iterates c_{t-1} (b1), c_{t-2} (b2; cnt == nullptr -> zero) and c_t (b0);
  // at the last iteration c_t goes densely to out_c instead of b0
  const int* colslot = nullptr;
  long colslot_stride = 0;
  int ncs = 0;
  SlotBuf b0, b1, b2;
  float beta_prev = 0.f;
  float2* keep_c = nullptr;        // ROW_PRUNED, not last: also store c_t densely here (nullable)
  // ROW_ISTA / ROW_FISTA / ROW_ADMM over a zero-padded embedding: only the first act_cols
  // elements of the first act_rows rows of each scene are coefficients; the update there is
  // as above and every other element is held at zero (c = 0).  0 = the whole grid.
  int act_cols = 0, act_rows = 0;
  // ROW_PRUNED: dscal (nullable) overrides kappa with dscal[0]; at the last iteration out_prev
  // (nullable) receives c_{t-1} densely; out_prev is also honoured by ROW_FISTA
};

// Column pass (transforms along l2, stride L1).
enum ColMode {
  COL_FWD = 0,          // xy = DFT_cols(xy)
  COL_INV = 1,          // xy = scale * IDFT_cols(xy)
  COL_FILTER_AFFINE = 2,// xy = IDFT_cols((a + b*Omega) . DFT_cols(xy)), (a, b) = coef[scene]
  COL_FILTER_ADMM = 3,  // xy = IDFT_cols(scale/(Omega + rho) . DFT_cols(xy))
  COL_FILTER_CPLX = 4,  // xy = IDFT_cols(mulc . DFT_cols(xy))
  COL_MULINV_AFFINE = 5,// xy = IDFT_cols((a + b*Omega) . xy)
  COL_MULINV_ADMM = 6,  // xy = IDFT_cols(scale/(Omega + rho) . xy)
  // Sparse-support forms: Omega is nonzero only on a listed set of bins (the
  // folded array elements), and the right-hand side of the iteration lives on
  // the same bins in the spectral domain, so both are applied from a short
  // per-column list instead of dense grids.
  COL_SPARSE_AFFINE = 7,// xy = IDFT_cols(m . DFT_cols(xy) + r): m = a off the support, a + b Omega_j on it; r = rhs_j
  COL_SPARSE_ADMM = 8,  // m = scale/rho off the support, scale/(Omega_j + rho) on it; r = rhs_j/(Omega_j + rho)
  COL_PRUNED_AFFINE = 9,// kept columns only: m = 0 off the support, b Omega_j on it; r = rhs_j
  COL_PRUNED_CPLX = 10, // kept columns only, entries from `dil`: m = mulc[bin] - 1/L (complex),
                        // r = dscal[1] * inv_mu * rhs[orig] (0 for orig < 0)
  // ADMM over the kept columns with the scaled dual split as v = u + IDFT2(Psi),
  // Psi on the support bins (eqs. (13)-(15) rearranged; u and z stay spatial):
  // Y = DFT_cols(xy); V'_j = (rhs_j - rho Psi_j - Omega_j scale Y_j) / (Omega_j + rho)
  // (scale = 1/L); Psi_j += V'_j; vlast_j = V'_j; xy = IDFT_cols(Psi on the support, 0 off it)
  COL_PRUNED_ADMM = 11,
  COL_PRUNED_EXPAND = 12,  // kept columns only: xy = IDFT_cols(vlast on the support, 0 off it)
};

// One bin of a dilated support list: spectral row k2, and the entry of the
// plan's support list holding the same bin (its right-hand side), or -1.
struct DilEntry {
  int k2;
  int orig;
};

// One support bin of a column: spectral row k2 and its eigenvalue.
struct SupEntry {
  int k2;
  float omega;
};

struct ColArgs {
  float2* xy = nullptr;          // [nscenes][N][L1]
  const float* omega = nullptr;  // [N][L1] eigenvalues, scene stride omega_stride (0 = shared)
  long omega_stride = 0;
  const float2* mulc = nullptr;  // complex multiplier [N][L1], scene stride mulc_stride
  long mulc_stride = 0;
  const float2* coef = nullptr;  // per-scene (a, b) (device)
  const float2* tw = nullptr;    // [N]
  int L1 = 0;
  int nscenes = 1;
  float rho = 0.f, scale = 1.f;
  const int* scene_map = nullptr;// logical scene -> physical scene (nullable = identity)
  int spread = 1;                // see PassCfg::spread
  // sparse-support modes: entries of (scene s, column k1) are sup[sup_ptr[s*sup_ptr_stride + k1] ..
  // sup_ptr[s*sup_ptr_stride + k1 + 1]); their right-hand sides are sup_rhs[s*sup_rhs_stride + j]
  const int* sup_ptr = nullptr;
  long sup_ptr_stride = 0;
  const SupEntry* sup = nullptr;
  const float2* sup_rhs = nullptr;
  long sup_rhs_stride = 0;
  // compact column sets: ncols columns per scene at row stride ldx (0 = L1 for both);
  // column c of scene s is spectral column scol[s * scol_stride + c] (-1 = padding)
  int ncols = 0;
  int ldx = 0;
  const int* scol = nullptr;
  long scol_stride = 0;
  // COL_PRUNED_CPLX: dilated entries of column k1 are dil[sup_ptr[k1] .. sup_ptr[k1 + 1]);
  // the layer's multiplier grid is mulc (stride 0), dscal its {kappa, mu} pair
  const DilEntry* dil = nullptr;
  const float* dscal = nullptr;
  float inv_mu = 1.f;
  // COL_PRUNED_ADMM / COL_PRUNED_EXPAND: per support entry, indexed as sup_rhs
  float2* psi = nullptr;         // Psi_j, read and updated (ADMM)
  float2* vlast = nullptr;       // V'_j of the pass: written (ADMM), read (EXPAND)
};

// Spectral right-hand side on the support bins, per scene:
// rhs[rhs_off + j] = scale * sum over sources q of entry (entry_off + j) of sign_q * y[idx_q].
struct SupRhsDesc {
  const float2* y = nullptr;
  int entry_off = 0;
  int nentries = 0;
  long rhs_off = 0;
  float scale = 1.f;
  int pad = 0;
};
// src_ptr: [entries + 1] offsets into src; src[q] = (sensor index << 1) | (1 if (-1)^(m1+m2) = -1)
int launch_sup_rhs(const SupRhsDesc* desc, int nscenes, int max_entries, const int* src_ptr, const int* src,
                   float2* rhs, int* flag, hipStream_t s);

// LDS slots (float2) of one exchange area of an N-point transform: N plus one
// padding slot per 8 (bank spreading).
constexpr int fft_area(int N) { return N + N / 8; }

// LDS exchange areas of a transform of N points at E per thread: two (used in
// turn, one barrier per exchange) when it has three or more stages, else one.
constexpr int fft_areas(int N, int E) {
  int logn = 0, loge = 0;
  while ((1 << logn) < N) ++logn;
  while ((1 << loge) < E) ++loge;
  const int nst = logn / loge + (logn % loge ? 1 : 0);
  return nst >= 3 ? 2 : 1;
}

// LDS of the pruned row pass, in float2 units: two areas per row (slot
// expansions, then the transforms' exchange areas), N twiddles, the compact
// kept columns of each row, two occupancy masks of N bits per row and, for
// rows longer than a wavefront, T counts per row.
constexpr long rowp_lds_floats(int N, int E, int rpb, int ncs) {
  const int T = N / E;
  const int MW = (N + 31) / 32;
  return 2L * rpb * fft_area(N) + N + static_cast<long>(rpb) * ncs + (2L * rpb * MW + 1) / 2 +
         (T > 64 ? (static_cast<long>(rpb) * T + 1) / 2 : 0);
}

// Launch shape of the passes for one transform length: E elements per thread
// (T = N/E threads per transform), rows per block of the row pass, columns per
// block of the column pass.
struct PassCfg {
  int E = 16;
  int rpb = 1;
  int W = 1;
  int spread = 1;  // launch spread x the blocks; only every spread-th does work (1 = off)
};

// Returns 0, -1 (shape not launchable), -2 (size not compiled), -4 (HIP error).
int launch_row(int N, const PassCfg& cfg, int mode, const RowArgs& a, hipStream_t s);
int launch_col(int N, const PassCfg& cfg, int mode, const ColArgs& a, hipStream_t s);

#define BCCB_DECLARE_N(n)                                                                  \
  int row_launch_##n(int E, int mode, const RowArgs& a, int rpb, hipStream_t s);           \
  int col_launch_##n(int E, int mode, const ColArgs& a, int W, hipStream_t s);             \
  int lista_launch_##n(int which, const void* args, int E, int rpb_or_w, int groups, hipStream_t s);
BCCB_DECLARE_N(8)
BCCB_DECLARE_N(16)
BCCB_DECLARE_N(32)
BCCB_DECLARE_N(64)
BCCB_DECLARE_N(128)
BCCB_DECLARE_N(256)
BCCB_DECLARE_N(512)
BCCB_DECLARE_N(1024)
#undef BCCB_DECLARE_N

struct ListaBwdRowArgs {
  const float2* A_in = nullptr;    // row-spectral zbar_{j+1} (nullptr at j = K-1)
  float2* zbar_store = nullptr;    // spatial zbar_{j+1} written here when A_in is set
  const float2* zbar2 = nullptr;   // spatial zbar_{j+2} (nullable = 0)
  const float2* U = nullptr;       // saved u_j
  const float2* Cm1 = nullptr;     // saved c_{j-1} (nullable = 0)
  const float2* Cm2 = nullptr;     // saved c_{j-2} (nullable = 0)
  const float2* b = nullptr;       // D_s^H y per scene
  const float2* cout = nullptr;    // c_{K-1} (loss gradient at j = K-1)
  const float2* label = nullptr;   // c* (loss gradient at j = K-1)
  const double* norm_label = nullptr;  // per scene ||c*||^2
  const float* tau = nullptr;      // per scene
  const float* dscal = nullptr;    // layer j {theta_j mu_j, mu_j}
  float beta_j = 0.f, beta_j1 = 0.f, beta_jm1 = 0.f;
  float loss_scale = 0.f;          // 2 / batch
  float2* Aout = nullptr;          // DFT_rows(ubar_j)
  float2* Zout = nullptr;          // DFT_rows(z_j)
  double* part = nullptr;          // [rows][2] partial {dkappa, Re<ubar, b>}
  const float2* tw = nullptr;
  int nrows = 0, rows_per_scene = 1;
};

struct ListaBwdColArgs {
  float2* A = nullptr;             // [B][N][L1] in: DFT_rows(ubar), out: row-spectral zbar
  const float2* Z = nullptr;       // [B][N][L1] DFT_rows(z_j)
  const float2* mulc = nullptr;    // [N][L1] m_j / L
  float2* gm_part = nullptr;       // [groups][N][L1]
  const float2* tw = nullptr;
  int L1 = 0, nscenes = 0, groups = 1;
};

struct KktRowArgs {
  const float2* gc = nullptr;      // row-spectral G c rows; kept form: kept columns [rows][ncs] of
                                   // the row spectra of scale^-1 (b - G c)
  const float2* c = nullptr;
  const float2* b = nullptr;       // full form only
  const float* tau = nullptr;      // per physical scene
  double* part = nullptr;          // [physical rows] sum of e^2
  const int* scene_map = nullptr;
  const float2* tw = nullptr;
  int nrows = 0, rows_per_scene = 1;
  const int* colslot = nullptr;    // kept form: spectral column -> kept slot (-1 = none), [N]
  int ncs = 0;
  float scale = 1.f;               // kept form: b - G c = scale * IDFT_rows(kept spectra)
};

// Dense iteration-matrix product (the O(L^2) baseline).
struct DenseArgs {
  const float2* R = nullptr;     // [L][L] row-major, complex64
  const float2* x = nullptr;     // [L] input
  float2* out = nullptr;         // [L] product (mode 0) or next input (modes 1, 2)
  const float2* rhs = nullptr;   // mu*b (mode 1) or w = (G + rho I)^-1 b (mode 2)
  float2* state = nullptr;       // c_{t-1} (mode 1) or v (mode 2)
  float2* out_z = nullptr;       // mode 2: z (nullable)
  long L = 0;
  float kappa = 0.f, beta = 0.f, rho = 0.f;
};
int launch_dense_build(const float2* col, int L1, int L2, float2* R, hipStream_t s);
int launch_dense_gemv(int mode, const DenseArgs& a, hipStream_t s);

// Learned-FISTA backward and per-scene KKT passes: which = 0 backward row pass
// (ListaBwdRowArgs), 1 backward column pass (ListaBwdColArgs), 2 KKT row pass
// (KktRowArgs); E in {4, 8, 16}.
int lista_launch(int N, int which, const void* args, int E, int rpb_or_w, int groups, hipStream_t s);

// S[k2][k1] = scale * sum over kept elements folding onto (k1, k2) of (-1)^(m1+m2) y_m
int launch_scatter(const float2* y, const int* sensor_of, int M1, int M2, int L1, int L2,
                   float scale, float2* S, int* flag, hipStream_t s);

// Per-block partial sums (double) of 1/2|y_m - D_s c|^2 given spec = DFT2(c).
int launch_resid(const float2* spec, const float2* y, const int2* sensors, int M, int L1, int L2,
                 double* partial, int* nblocks, hipStream_t s);
// Per-block partials {sum e^2, max e, sum |c|, sum |b|^2} of the KKT residual.
int launch_kkt(const float2* c, const float2* b, const float2* gc, float tau, long L,
               double* partial, int* nblocks, hipStream_t s);
int launch_absmax(const float2* b, long L, double* partial, int* nblocks, hipStream_t s);
int launch_fill(float2* p, long n, hipStream_t s);   // zero fill (graph-safe, no memset node)
int launch_fill_int(int* p, long n, int value, hipStream_t s);
int launch_stream_copy(const void* src, void* dst, long n16, int variant, hipStream_t s);   // n16 16-byte vectors
// out = (1 + beta) a - beta b over n scenes of L points selected by map (nullable = identity)
int launch_momentum(float2* out, const float2* a, const float2* b, float beta, long L, int n, const int* map,
                    hipStream_t s);
int launch_copy(float2* dst, const float2* src, long n, hipStream_t s);

constexpr int kReduceBlocks = 512;

// Per-scene descriptor of a batched solve.
struct SceneDesc {
  const float2* y = nullptr;      // snapshot [M]
  const int* sensor_of = nullptr; // [M2][M1] index into y or -1
  float2* out = nullptr;          // output grid [L2][L1]
  int M1 = 0, M2 = 0;
  float scale = 1.f;              // multiplier of the scattered snapshot (mu for mu*b)
  int pad = 0;
};

// S[scene][k2][k1] = desc[scene].scale * (scatter of scene's snapshot), for n scenes of one size.
int launch_scatter_batch(const SceneDesc* desc, int n, int L1, int L2, float2* S, int* flag, hipStream_t s);
// desc[scene].out[i] = src[scene*L + i]
int launch_gather_batch(const SceneDesc* desc, int n, long L, const float2* src, hipStream_t s);

}  // namespace bccb
