/*
 * libbccb -- BCCB-structured LASSO solvers for single-snapshot 2D harmonic
 * recovery with sparse planar arrays, on AMD Instinct MI355X (gfx950).
 *
 * Problem (Sec. II): a planar array on the half-wavelength grid keeps M of its
 * M1 x M2 elements (mask, eq. (6)); the snapshot y_s = D_s c + n_s (eq. (7))
 * is explained by a coefficient grid c over the uniform harmonic grid
 * f_{i,l} = -1/2 + l/L_i (eq. (16)).  The LASSO (eq. (8), taken with the factor
 * 1/2 on the data term that its ISTA/FISTA/ADMM iterations imply) is solved by
 * ISTA (eq. (9)), FISTA (eqs. (10)-(12)) or ADMM (eqs. (13)-(15)).  Because the
 * Gram G = D_s^H D_s is block circulant with circulant blocks (eq. (17),
 * Sec. III-A), every G-product is computed as IDFT2(Omega . DFT2(c)) (eq. (23))
 * with the eigenvalues Omega of eq. (21).
 *
 * Layouts
 *   mask      host uint8 [M2][M1], mask[m2*M1 + m1] != 0 keeps element (m1, m2).
 *   y         device complex64 [M], the kept elements in increasing m1 + m2*M1
 *             (the row order of Psi, eq. (6)).
 *   grids     device complex64 [L2][L1] row-major: c[l1 + l2*L1] is the
 *             amplitude of harmonic (f_{1,l1}, f_{2,l2}) (eq. (4), index l1 + l2*L1).
 *   complex64 is interleaved (re, im) float pairs, i.e. bccb_c32.
 *
 * Ownership and ordering
 *   The caller owns every buffer it passes (device memory from any allocator).
 *   A plan owns its eigenvalues, twiddle tables and workspace and frees them
 *   in bccb_plan_destroy.  Work is enqueued on the plan's HIP stream
 *   (hipStream_t passed as void*, NULL = the null stream).  Solver and
 *   diagnostic calls return after the stream has drained (they read a status
 *   flag back), so their outputs are ready on return.  A plan is not thread
 *   safe and serves one stream at a time; distinct plans are independent.
 *
 * Errors
 *   Arguments are checked on the host before anything is enqueued; a negative
 *   code means nothing was written.  BCCB_E_NONFINITE means the results were
 *   computed from NaN/Inf input and must not be used.
 */
#ifndef BCCB_H
#define BCCB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bccb_plan_s* bccb_plan_t;
typedef struct { float re, im; } bccb_c32;
typedef struct { double re, im; } bccb_c64;

enum bccb_status {
  BCCB_OK = 0,
  BCCB_W_NOT_CONVERGED = 1, /* warning: results written, some scene missed its target     */
  BCCB_E_INVALID = -1,      /* bad argument (null pointer, size, tau < 0, rho <= 0, ...)  */
  BCCB_E_UNSUPPORTED = -2,  /* valid but not implemented (e.g. L_i not a power of two)    */
  BCCB_E_NOMEM = -3,        /* device allocation failed                                   */
  BCCB_E_DEVICE = -4,       /* a HIP call failed                                          */
  BCCB_E_NONFINITE = -5,    /* NaN or Inf in y or in the warm start                       */
  BCCB_E_SCRATCH = -6       /* grid larger than the allocation-free entry point's array   */
};

/* Human-readable name of a status code (static string). */
const char* bccb_status_string(int status);

/*
 * bccb_stream_copy -- copy `bytes` (a multiple of 16) from src to dst, both
 *   device pointers aligned to 16 bytes, with the library's streaming copy
 *   kernel (16-byte vector loads and stores), enqueued on `stream`.  variant
 *   (0..63) picks the kernel shape: bits 0-1 give 1, 2, 4 or 8 loads in flight
 *   per thread, bit 2 non-temporal hints, bits 3-5 256 << k workgroups.
 *   Not part of the method: it measures the device's achievable HBM
 *   bandwidth, the ceiling the passes are compared with.  BCCB_E_INVALID for
 *   null pointers, misalignment, a size that is not a multiple of 16 or a
 *   variant outside 0..63.
 */
int bccb_stream_copy(const void* src, void* dst, size_t bytes, int variant, void* stream);

/*
 * bccb_plan -- per-geometry setup (Sec. III-A, III-B).
 *   Builds the first column r of G (property (iv) of Sec. III-A, from the
 *   masked Kronecker sum of eq. (17)) and its eigenvalues Omega by eq. (21) in
 *   FP64 on the host, stores Omega as FP32 on the device, sets the step
 *   mu = 1/sigma_max(D_s)^2 = 1/max(Omega) (eq. (9)) and the DFT twiddles.
 *   mask: host [M2][M1], at least one nonzero.  1 <= M1, M2 <= 4096.
 *   L1, L2: powers of two in [8, 1024] (L1 != L2 allowed).  M_i > L_i
 *   (aliasing) is accepted: eq. (21) stays exact.
 *   stream: hipStream_t (may be NULL).  *out receives the plan.
 *   Returns BCCB_OK, BCCB_E_INVALID, BCCB_E_UNSUPPORTED, BCCB_E_NOMEM, BCCB_E_DEVICE.
 */
int bccb_plan(const uint8_t* mask, int M1, int M2, int L1, int L2, void* stream, bccb_plan_t* out);

/*
 * bccb_plan_spaced -- a plan for a uniform harmonic grid at element spacing
 *   (gamma1 lambda, gamma2 lambda) (Sec. II-A: the harmonics lie in
 *   [-gamma_i, gamma_i), sampled at f_{i,l} = -gamma_i + l 2 gamma_i / L_i,
 *   eq. (16)) and for grid lengths that are not powers of two.  On that grid
 *   the Gram D_s^H D_s is block Toeplitz with Toeplitz blocks (circulant only
 *   at gamma_i = 1/2, Sec. III-A): the plan embeds it in the leading
 *   L1 x L2 window of a P1 x P2 BCCB (P_i the smallest power of two
 *   >= max(8, 2 L_i - 1)) and computes every Gram product by eq. (23) on the
 *   padded grid, the iterate held at zero outside the window.  The step is
 *   mu = 1/sigma_max(D_s)^2 (eq. (9)): at gamma = 1/2 the largest eigenvalue
 *   L1 L2 x (most elements folding onto one bin) of eq. (21), otherwise the
 *   largest eigenvalue of D_s D_s^H found by Lanczos in FP64.
 *   mask: host [M2][M1] (as bccb_plan); L1, L2 in [2, 512], any integers;
 *   gamma1, gamma2 in (0, 1].  gamma1 = gamma2 = 1/2 with L_i powers of two
 *   in [8, 1024] returns an ordinary plan (bccb_plan).  With gamma != 1/2 at
 *   most 2048 kept elements (BCCB_E_UNSUPPORTED beyond).
 *   Grids passed to the calls below stay the caller's [L2][L1] grids.
 *   A plan made here serves bccb_plan_info (M and mu; omega_host must be
 *   NULL), bccb_adjoint, bccb_adjoint_maxabs, bccb_gram_apply,
 *   lasso_solve_ista, lasso_solve_fista, bccb_objective_kkt, bccb_kkt,
 *   bccb_extract_peaks, bccb_plan_get_config, bccb_plan_set_config and
 *   bccb_plan_autotune (the full row and column passes' shapes; sparse_iterate
 *   and resident_groups are refused) and, at gamma1 = gamma2 = 1/2 only,
 *   lasso_solve_admm ((G + rho I)^-1 is then the BCCB of spectrum
 *   1/(Omega + rho), Sec. III-A (ii), embedded the same way; the inverse of a
 *   Toeplitz Gram is not Toeplitz); every other call returns
 *   BCCB_E_UNSUPPORTED for it.  Memory: about 70 bytes per point of
 *   the P1 x P2 grid.
 */
int bccb_plan_spaced(const uint8_t* mask, int M1, int M2, int L1, int L2, double gamma1, double gamma2,
                     void* stream, bccb_plan_t* out);

/*
 * bccb_plan_embedding -- of a plan made by bccb_plan_spaced with a padded
 *   embedding: the transform grid P1 x P2 and (omega_host, nullable, host
 *   float [P2][P1]) the FP32 eigenvalues of the embedded Gram, Omega_e =
 *   DFT2 of the first column holding t(d1, d2) = G[(d1, d2), (0, 0)] (and
 *   t(-d) = conj t(d)) at (d1 mod P1, d2 mod P2), zero elsewhere.
 *   BCCB_E_UNSUPPORTED for an ordinary plan.
 */
int bccb_plan_embedding(bccb_plan_t plan, int* P1, int* P2, float* omega_host);

/* Free a plan and everything it owns (NULL is accepted). */
int bccb_plan_destroy(bccb_plan_t plan);

/* Rebind the plan to another hipStream_t. */
int bccb_set_stream(bccb_plan_t plan, void* stream);

/*
 * bccb_plan_info -- geometry facts of a plan.  Any output pointer may be NULL.
 *   M: number of kept elements; mu: step 1/max(Omega) in FP64;
 *   omega_host: host float [L2][L1] receiving the FP32 eigenvalue grid
 *   (Omega[k2][k1] is the eigenvalue of the mode e^{+j2pi(k1 l1/L1 + k2 l2/L2)}).
 */
int bccb_plan_info(bccb_plan_t plan, int* M, double* mu, float* omega_host);

/*
 * bccb_adjoint -- b = D_s^H y_s (the right-hand side of eqs. (9), (13)).
 *   Computed as the unnormalised 2D inverse DFT of y scattered onto the
 *   spectral grid with the (-1)^(m1+m2) factor that the grid offset -1/2 of
 *   eq. (16) puts on element (m1, m2).  y: device [M]; b: device [L2][L1].
 *   BCCB_E_NONFINITE if y holds NaN/Inf.
 */
int bccb_adjoint(bccb_plan_t plan, const bccb_c32* y, bccb_c32* b);

/* max_l |(D_s^H y)_l| in FP64 (for the regularisation weight tau = frac * max|A^H y|). */
int bccb_adjoint_maxabs(bccb_plan_t plan, const bccb_c32* y, double* maxabs);

/*
 * bccb_gram_apply -- gx = G x = IDFT2(Omega . DFT2(x)) (eq. (23)).
 *   x, gx: device [L2][L1]; may alias.
 */
int bccb_gram_apply(bccb_plan_t plan, const bccb_c32* x, bccb_c32* gx);

/*
 * lasso_solve_ista -- `iters` iterations of eq. (9):
 *   c <- S_{mu tau}(c - mu G c + mu D_s^H y), mu = 1/max(Omega).
 *   tau >= 0 (absolute weight of ||c||_1); iters >= 0; c0 device [L2][L1] or
 *   NULL for zeros; c_out device [L2][L1] (may alias c0).  iters = 0 copies c0
 *   (or zeros) to c_out.
 */
int lasso_solve_ista(bccb_plan_t plan, const bccb_c32* y, float tau, int iters,
                     const bccb_c32* c0, bccb_c32* c_out);

/*
 * lasso_solve_fista -- `iters` iterations of eqs. (10)-(12) with z^(1) = c^(0),
 *   alpha_1 = 1 (first momentum weight 0), momentum weights computed in FP64.
 *   Arguments as lasso_solve_ista.  Exactly `iters` Gram products.
 */
int lasso_solve_fista(bccb_plan_t plan, const bccb_c32* y, float tau, int iters,
                      const bccb_c32* c0, bccb_c32* c_out);

/*
 * lasso_solve_fista_noalloc -- for callers that cannot allocate device memory
 *   (tight serving loops, harnesses that forbid hipMalloc): the solve of
 *   lasso_solve_fista, same arguments and results, run through the plan's
 *   full row and column passes with every work buffer taken
 *   from one static device array of the library (6 MiB + 512 B per device,
 *   resolved on the first call with that device current and held until the
 *   process ends) instead of the plan's workspace.  The call allocates nothing
 *   (no hipMalloc / hipFree, no graph instantiation): it enqueues kernels and
 *   two small copies on the plan's stream and returns after draining it.
 *   Limit: L1 * L2 <= 2^18 (512 x 512); larger grids return BCCB_E_SCRATCH.
 *   The plan's device must be current (else BCCB_E_INVALID).  Every call on one
 *   GPU shares that GPU's array: calls that overlap on one device (several host
 *   threads, or streams in flight at once) race; calls issued one after another
 *   are safe.  Errors as lasso_solve_fista.
 */
int lasso_solve_fista_noalloc(bccb_plan_t plan, const bccb_c32* y, float tau, int iters,
                              const bccb_c32* c0, bccb_c32* c_out);

/*
 * lasso_solve_admm -- `iters` iterations of eqs. (13)-(15) from z = v = 0 with
 *   threshold tau/rho (scaled ADMM; equal to the printed rho*tau at rho = 1).
 *   (G + rho I)^-1 is the BCCB with spectrum 1/(Omega + rho) (closure under
 *   inversion, Sec. III-A (ii)), and (G + rho I)^-1 D_s^H y is precomputed.
 *   rho > 0.  z_out: device [L2][L1], the sparse iterate z^T; c_out: device
 *   [L2][L1] or NULL, the iterate c^T of eq. (13).
 */
int lasso_solve_admm(bccb_plan_t plan, const bccb_c32* y, float tau, float rho, int iters,
                     bccb_c32* z_out, bccb_c32* c_out);

/*
 * bccb_objective_kkt -- diagnostics of a coefficient grid c (device [L2][L1]).
 *   objective = 1/2 ||y - D_s c||^2 + tau ||c||_1 (eq. (8) with the factor 1/2),
 *   with D_s c read from DFT2(c) at the kept elements' bins.
 *   KKT: g = D_s^H y - G c, e_l = |g_l - tau c_l/|c_l|| (c_l != 0) or
 *   max(|g_l| - tau, 0) (c_l = 0); r_kkt = ||e||_2 / ||D_s^H y||_2,
 *   max_e_over_tau = max_l e_l / tau.  Sums in FP64 over FP32 terms.
 *   Any output pointer may be NULL.
 */
int bccb_objective_kkt(bccb_plan_t plan, const bccb_c32* y, float tau, const bccb_c32* c,
                       double* objective, double* r_kkt, double* max_e_over_tau);

/*
 * bccb_kkt -- the two monitors of a coefficient grid c under the names of the
 *   call list: *r_kkt = ||e||_2 / ||D_s^H y||_2 (the LASSO stationarity defect
 *   e of eq. (8) with the factor 1/2, as in bccb_objective_kkt) and *obj =
 *   1/2 ||y - D_s c||^2 + tau ||c||_1.  Same arguments, checks and arithmetic as
 *   bccb_objective_kkt; either output may be NULL.
 */
int bccb_kkt(bccb_plan_t plan, const bccb_c32* y, float tau, const bccb_c32* c, double* r_kkt, double* obj);

/*
 * bccb_plan_omega_device -- copy the plan's FP32 eigenvalue grid Omega (eq. (21),
 *   [L2][L1], the same values bccb_plan_info returns to the host) into the
 *   caller's device buffer omega_dev (L1*L2 floats), on the plan's stream;
 *   returns after the copy.  BCCB_E_INVALID for a null plan or buffer.
 */
int bccb_plan_omega_device(bccb_plan_t plan, float* omega_dev);

/*
 * Harmonics and directions of recovered coefficient grids (Sec. II-A: the support of c
 * marks the harmonic tuples (f_{1,l1}, f_{2,l2}) present; eq. (2) maps a tuple to a
 * direction, f1 = gamma1 cos(phi) sin(theta), f2 = gamma2 sin(phi) sin(theta)).
 */
typedef struct {
  int index;        /* grid index l1 + l2*L1 of the local maximum                        */
  float mag2;       /* |c|^2 there (FP32: re*re + im*im, each operation rounded)         */
  float f1, f2;     /* refined harmonic tuple (cycles per element)                        */
  float phi, theta; /* direction by eq. (2); theta = NaN outside the visible region       */
  bccb_c32 amp;     /* sum of the coefficients of the 3 x 3 neighbourhood                 */
} bccb_peak;

/*
 * bccb_extract_peaks -- for each of `batch` grids c (device [batch][L2][L1], the plan's
 *   grid; for a bccb_plan_spaced plan its L1 x L2), the strongest local maxima of |c|:
 *   grid points whose |c|^2 (FP32 as above) exceeds min_mag2 and beats all 8 neighbours
 *   (equal |c|^2: the smaller index ranks higher; the grid wraps when gamma1 = gamma2 =
 *   1/2, where f = -1/2 and f = 1/2 coincide), at most max_peaks (1..1024) by decreasing
 *   |c|^2 (ties: smaller index first).  Each is refined to the |c|-weighted mean of its
 *   3 x 3 neighbourhood's grid offsets, f_i = -gamma_i + (l_i + offset_i) 2 gamma_i / L_i
 *   (eq. (16); wrapped into [-1/2, 1/2) at half spacing), and mapped to (phi, theta) by
 *   inverting eq. (2): phi = atan2(f2/gamma2, f1/gamma1) in [-pi, pi), theta =
 *   asin(sqrt((f1/gamma1)^2 + (f2/gamma2)^2)), NaN when that exceeds 1.
 *   peaks: device [batch][max_peaks] (entries past counts[s] untouched); counts: device
 *   int [batch], the peaks written per grid, or -1 when more than 4096 local maxima exceed
 *   min_mag2 (nothing written for that grid: raise the threshold).  batch in 1..65535.
 *   Work buffers (32 KB per grid) are kept by the plan.  Returns after the stream drains.
 */
int bccb_extract_peaks(bccb_plan_t plan, const bccb_c32* c, int batch, int max_peaks, float min_mag2,
                       bccb_peak* peaks, int* counts);

/*
 * FP64 variants -- the same operations in complex128 on the device, for results at the
 * level of the paper's FP64 regular-vs-fast comparison (Table I, Sec. III-C): eigenvalues by
 * eq. (21) in FP64, radix-2 FFTs and updates in double precision, the full row and column
 * passes (no pruned or cooperative forms).  Plans from bccb_plan (power-of-two grids); the
 * FP64 buffers (56 bytes per grid point) are allocated on the first FP64 call.  Arguments,
 * layouts and errors as the FP32 calls, with complex128 device buffers (bccb_c64) and FP64
 * tau and rho; BCCB_E_UNSUPPORTED for a bccb_plan_spaced plan with a padded embedding.
 */
int bccb_adjoint_f64(bccb_plan_t plan, const bccb_c64* y, bccb_c64* b);
int bccb_gram_apply_f64(bccb_plan_t plan, const bccb_c64* x, bccb_c64* gx);
int lasso_solve_ista_f64(bccb_plan_t plan, const bccb_c64* y, double tau, int iters, const bccb_c64* c0,
                         bccb_c64* c_out);
int lasso_solve_fista_f64(bccb_plan_t plan, const bccb_c64* y, double tau, int iters, const bccb_c64* c0,
                          bccb_c64* c_out);
int lasso_solve_admm_f64(bccb_plan_t plan, const bccb_c64* y, double tau, double rho, int iters, bccb_c64* z_out,
                         bccb_c64* c_out);

/*
 * Batched solves -- many independent snapshots, each with its own plan (its
 * own array mask and grid size; plans may repeat), solved together.
 *
 * bccb_batch_create groups the scenes by grid size (L1, L2) into classes and
 * allocates, per class, contiguous device arenas for the iterates, the
 * right-hand sides and the eigenvalue grids (copied from the plans).  Each
 * solve then runs every class's column and row passes over all of its scenes
 * at once, with the whole iteration loop captured in one hipGraph (replayed
 * while `iters` repeats).  plans: host array of nscenes plan handles (they must
 * outlive the batch); stream: hipStream_t.  Memory: about 24 bytes per grid
 * point of every scene plus 4 for its eigenvalues.
 */
typedef struct bccb_batch_s* bccb_batch_t;

int bccb_batch_create(const bccb_plan_t* plans, int nscenes, void* stream, bccb_batch_t* out);
int bccb_batch_destroy(bccb_batch_t batch);

/* Number of size classes and, per class c < nclasses, its (L1, L2) and scene count. */
int bccb_batch_info(bccb_batch_t batch, int* nclasses, int* L1, int* L2, int* count);

/*
 * lasso_solve_batch_fista -- `iters` FISTA iterations (as lasso_solve_fista,
 *   from c^(0) = 0) on every scene of the batch.  y: host array of nscenes
 *   device pointers (complex64 [M_s]); tau: host array of nscenes weights
 *   (>= 0, finite); c_out: host array of nscenes device pointers
 *   (complex64 [L2_s][L1_s]).  BCCB_E_NONFINITE if any snapshot holds NaN/Inf.
 */
int lasso_solve_batch_fista(bccb_batch_t batch, const bccb_c32* const* y, const float* tau, int iters,
                            bccb_c32* const* c_out);

/*
 * bccb_batch_autotune -- per class, time the launchable row and column pass
 *   shapes over the whole class (`reps` launches each) and keep the fastest.
 */
int bccb_batch_autotune(bccb_batch_t batch, int reps);

/*
 * bccb_batch_class_config -- launch shape class `cls` (< nclasses of
 *   bccb_batch_info) runs with: cfg[0..5] = row-pass E, rows per block,
 *   column-pass E, columns per block, 1 if the class takes the pruned passes,
 *   and the columns its column pass transforms per scene.  cfg: host int[6].
 */
int bccb_batch_class_config(bccb_batch_t batch, int cls, int* cfg);

/*
 * bccb_batch_set_sparse_iterate -- 1 (the default for classes with L1 >= 8):
 *   keep every scene's FISTA iterate per row in (index, value) slots while the
 *   row is sparse, as bccb_config.sparse_iterate does for one plan; 0: dense
 *   iterates.  Same results either way (the stored values are exact).
 *   BCCB_E_INVALID for a null batch or a value other than 0 or 1.
 */
int bccb_batch_set_sparse_iterate(bccb_batch_t batch, int on);

/*
 * bccb_batch_set_support_columns -- 1 (the default): size classes whose every
 *   scene has a kept-column set (see bccb_config.support_columns) run the
 *   pruned passes; 0: the full passes (with sparse_iterate as set).  Results
 *   agree to FP32 rounding.  BCCB_E_INVALID for a null batch or a value other
 *   than 0 or 1.
 */
int bccb_batch_set_support_columns(bccb_batch_t batch, int on);

/*
 * bccb_batch_set_resident -- 1 (the default where the batch supports it): run
 *   the solve as one persistent launch in which each workgroup takes whole
 *   scenes from a queue (larger grids first) and runs every FISTA iteration of
 *   a scene (eqs. (10)-(12), the eq. (23) product in the support-column form)
 *   with its kept row spectra held in LDS; 0: the captured per-iteration pass
 *   graph.  Supported when every size class is square (L1 = L2 in 32, 64, 128,
 *   256), every scene has a kept-column set and a workgroup's state fits the
 *   device's LDS; the path is taken only while support columns are on.
 *   Results agree with the pass graph to FP32 rounding.  on = 256, 512 or 1024
 *   selects the persistent launch at that workgroup size (1 takes the size that
 *   keeps the most waves resident).  BCCB_E_UNSUPPORTED for a nonzero value on a
 *   batch without support (or a workgroup size whose LDS does not fit),
 *   BCCB_E_INVALID for a null batch or another value.
 */
int bccb_batch_set_resident(bccb_batch_t batch, int on);

/*
 * bccb_batch_resident_info -- *on = 1 if the persistent launch is selected, 0 if
 *   it is supported but off, -1 if the batch cannot take it; *threads, *blocks,
 *   *lds_bytes: its workgroup size, grid and dynamic LDS per workgroup (0 when
 *   unsupported).  Any output pointer may be null.
 */
int bccb_batch_resident_info(bccb_batch_t batch, int* on, int* threads, int* blocks, int* lds_bytes);

/*
 * Learned unrolled FISTA with a KKT-gated plain-FISTA fallback.
 *
 * Network (all scenes share one plan, i.e. one array mask and grid): layer k,
 * k = 0 .. layers-1, is one FISTA step (eqs. (10)-(12)) with its own step
 * mu_k = s_k / max(Omega), threshold kappa_k = theta_k mu_k tau (tau per scene)
 * and a BCCB spectrum corrected by a learned 5x5 complex circular convolution,
 * Omega'_k = Omega + Delta_k (*) Omega (still a BCCB: closure under linear
 * combination, Sec. III-A (i)):
 *   u_k = IDFT2((1 - mu_k Omega'_k) . DFT2(z_k)) + mu_k D_s^H y,
 *   c_k = S_{kappa_k}(u_k),  z_{k+1} = c_k + beta_k (c_k - c_{k-1}),
 * from z_0 = c_{-1} = 0, with the FISTA momentum weights beta_k.  Output c_{layers-1}.
 *
 * Parameters: device float [layers][52] = {s_k, theta_k, Re Delta_k[5][5],
 * Im Delta_k[5][5]} (row-major taps, tap (a, b), a, b in -2..2, shifts the
 * spectrum by a along k2 and b along k1).  s = theta = 1, Delta = 0 makes every
 * layer one plain FISTA iteration.
 * Snapshots: device complex64 [batch][M]; tau: host float [batch];
 * grids: device complex64 [batch][L2][L1].
 */
typedef struct bccb_lista_s* bccb_lista_t;
#define BCCB_LISTA_PER_LAYER 52

/* Workspace for up to max_batch scenes; train != 0 also keeps every layer's
 * activations (16 bytes per grid point per layer per scene) for lista_backward. */
int lista_create(bccb_plan_t plan, int layers, int max_batch, int train, bccb_lista_t* out);
int lista_destroy(bccb_lista_t net);

/* Forward pass; c_out (nullable) receives c_{layers-1}.  In training mode the
 * activations are kept for the next lista_backward. */
int lista_forward(bccb_lista_t net, const float* params, const bccb_c32* y, const float* tau, int batch,
                  bccb_c32* c_out);

/*
 * lista_backward -- gradient of loss = mean_s ||c_s - c*_s||^2 / ||c*_s||^2 over the
 *   batch of the last training-mode forward.  labels: device [batch][L2][L1];
 *   grad: device float [layers][52] (overwritten); *loss (nullable) the loss.
 *   The backward of the soft threshold and of each BCCB layer (adjoint spectrum
 *   conj(1 - mu_k Omega'_k)) runs in the same row/column passes as the forward.
 */
int lista_backward(bccb_lista_t net, const float* params, const bccb_c32* labels, float* grad, double* loss);

/* One Adam step on n device floats (bias-corrected, step >= 1).  lr_scale
 * (device float [n], nullable) multiplies the learning rate per parameter, e.g.
 * to move the 5x5 filter taps more slowly than the steps and thresholds. */
int lista_adam(float* params, const float* grad, float* m, float* v, int n, int step, float lr, float beta1,
               float beta2, float eps, const float* lr_scale, void* stream);

/*
 * lista_solve -- KKT-gated solve.  params != NULL: learned forward, then
 *   plain FISTA from the network output on the scenes whose KKT residual
 *   r = ||e||/||D_s^H y|| (as in bccb_objective_kkt) exceeds kkt_target,
 *   checked every check_every iterations; converged scenes drop out of the
 *   passes.  restart != 0: the fallback restarts the momentum (z = output,
 *   alpha = 1); restart == 0: it continues the unrolled FISTA (z from the last
 *   two layer outputs with the last layer's momentum weight, alpha resumed
 *   after the layers), so identity weights give exactly plain FISTA.  An output
 *   that is non-finite or farther from stationarity than zero is replaced by
 *   zero (and the momentum restarts).  params == NULL: plain FISTA from zero
 *   with the same checks.  Stops when every
 *   scene meets the target or after max_iters fallback iterations.
 *   c_out: device [batch][L2][L1]; iters_out (host int [batch], nullable):
 *   fallback iterations per scene; rkkt_out (host double [batch], nullable):
 *   final residuals.  Returns BCCB_W_NOT_CONVERGED (1) if some scene missed
 *   the target.
 */
int lista_solve(bccb_lista_t net, const float* params, const bccb_c32* y, const float* tau, int batch,
                double kkt_target, int check_every, int max_iters, int restart, bccb_c32* c_out, int* iters_out,
                double* rkkt_out);

/*
 * lista_autotune -- where the plan has a kept-column set (see
 *   bccb_config.support_columns), time the launchable shapes of the fallback
 *   FISTA's pruned passes over the context's whole batch capacity, `reps`
 *   launches each, with the iterate in the sparse form most iterations see,
 *   and keep the fastest; otherwise nothing changes.  The pruned learned
 *   layers (same kernels over the dilated column set) then take the tuned
 *   element counts, with rows / columns per block reduced where their column
 *   set needs it.  Timing only: results agree to FP32 rounding.  The context's
 *   buffers hold nothing a later call reads.
 */
int lista_autotune(bccb_lista_t net, int reps);

/*
 * lista_set_resident -- 1 (the default where the context supports it): the
 *   gated solve runs each check interval of the fallback FISTA over the active
 *   scenes as one launch of the persistent whole-solve kernel (see
 *   bccb_batch_set_resident), the iterate, its kept spectra and the rows'
 *   counts carried between the intervals in the context's buffers, and the
 *   interval's KKT residuals formed by the same launch; 0: the pruned passes
 *   per iteration, checked by separate kernels.  Supported for square grids of 32..256 points
 *   with a kept-column set whose workgroup state fits the device's LDS.
 *   Results agree to FP32 rounding.  For callers comparing the two forms.
 *   BCCB_E_UNSUPPORTED for 1 on a context without support, BCCB_E_INVALID for a
 *   null context or a value other than 0 or 1.
 */
int lista_set_resident(bccb_lista_t net, int on);

/*
 * Dense "regular" baseline (Sec. II-B and the runtime comparison of Sec. III-C):
 * the explicit L x L complex64 iteration matrix, multiplied by the iterate
 * every iteration -- O(L^2) bytes and flops per iteration against the
 * O(L log L) of the BCCB passes.  kind 0: I - mu G (ISTA, FISTA); kind 1:
 * (G + rho I)^-1 (ADMM).  The matrix is built on the device from its first
 * column (property (iv) of Sec. III-A; the column computed in FP64 on the host)
 * and needs 8 L^2 bytes (34.4 GB at L = 256^2).  BCCB_E_NOMEM if it does not fit.
 */
typedef struct bccb_dense_s* bccb_dense_t;

int bccb_dense_create(bccb_plan_t plan, int kind, float rho, bccb_dense_t* out);
int bccb_dense_destroy(bccb_dense_t dense);
/* y = R x (x, y device [L2][L1], must not alias) */
int bccb_dense_apply(bccb_dense_t dense, const bccb_c32* x, bccb_c32* y);
/* `iters` iterations of solver 0 = ISTA, 1 = FISTA (kind 0 matrix) or 2 = ADMM
 * (kind 1 matrix; rho fixed at creation), same arithmetic as the BCCB solvers
 * with every Gram product taken through the dense matrix. */
int lasso_solve_dense(bccb_dense_t dense, int solver, const bccb_c32* y, float tau, int iters, bccb_c32* out);

/*
 * Launch configuration of a plan's passes.  A length-L transform runs as a
 * Stockham FFT over L/E threads holding E elements each; small E spreads one
 * row or column over more threads (lower latency for a single scene), large
 * E packs it into fewer threads (fewer LDS exchanges, better for batches).
 *   row_elems, col_elems: E in {4, 8, 16, 32}, E <= L1 (rows) / L2 (columns);
 *   row_rows_per_block: rows per workgroup, (L1/row_elems)*rows <= 256;
 *   col_cols_per_block: columns per workgroup, divides L1, (L2/col_elems)*cols <= 256;
 *   use_graph: 1 = capture each solve's iteration loop in a hipGraph (replayed
 *   while the solve arguments repeat), 0 = launch every pass directly.
 *   spectral_support: 1 = when Omega is sparse (the L1 L2 x fold-count grid of a
 *   mask, nonzero on at most L/4 bins), apply the multiplier and the right-hand
 *   side D_s^H y (whose 2D DFT is the scattered snapshot, nonzero on the same
 *   bins) from a per-column list inside the column pass, so the row pass reads
 *   no right-hand-side grid; 0 = dense Omega grid and a b grid.
 *   row_spread, col_spread: 1, 2, 4 or 8 -- launch that many times the blocks
 *   of a pass and let only every n-th work; on a GPU that deals consecutive
 *   blocks to its dies round-robin this keeps a single scene's working set in
 *   one die's L2 between passes.  Timing only.
 *   sparse_iterate: 1 = FISTA keeps c^(t) (eq. (11)) per row as up to L1/8
 *   (column index, value) pairs while the row has that few nonzeros -- after
 *   the soft threshold (eq. (9)) most rows do -- and as the dense row
 *   otherwise, so the row pass moves a few bytes per row instead of 16 B per
 *   grid point for c^(t-1) and c^(t); the values are stored exactly, so the
 *   iterates are those of the dense form.  Needs L1 >= 8.  0 = dense c^(t).
 *   support_columns: 1 = with spectral_support in effect, ISTA and FISTA split
 *   (I - mu G) z + mu b into z plus IDFT2 of a spectrum that lives on the
 *   support bins (Omega and DFT2(b) vanish elsewhere, eq. (21)): the column pass
 *   transforms only the spectral columns holding support bins, the row pass
 *   exchanges only those columns with it and rebuilds z in the spatial domain
 *   from c^(t-1), c^(t-2) (kept per row as above).  ADMM takes the same passes
 *   with its scaled dual split as v_t = (z_{t-1} - z_t) + IDFT2(Psi_t), Psi on
 *   the support bins and updated by the column pass (eqs. (13)-(15) rearranged
 *   so that x is never formed by cancelling the large support part of v), and
 *   one more pair of passes forms x^(T) when it is asked for.  Taken when those
 *   columns are at most L1/2 (after padding to a multiple of 4) and L1 >= 8;
 *   otherwise the full passes run.  0 = always the full passes.
 *   prow_elems, prow_rows_per_block: the pruned row pass's shape (as the row
 *   pass; rows * (2 L1 + ...) must fit the 64 KB of LDS a workgroup can hold);
 *   pcol_elems, pcol_cols_per_block: the pruned column pass's shape (columns
 *   per block must divide the padded kept-column count).  Ignored (and
 *   returned as set internally) when the plan has no such column set.
 *   resident_groups: 0 = the passes above; G > 0 = ISTA, FISTA and ADMM run as
 *   one cooperative launch of G workgroups (256 threads each) that stay resident
 *   for the whole solve: workgroup g owns L2/G grid rows and L1/G columns, keeps
 *   the iterate state of its rows and the spectral multiplier of its columns in
 *   registers, and meets the others at a grid barrier between the column and
 *   the row phase of every iteration (the same arithmetic as the passes at
 *   E = 4).  Needs the spectral support (a mask smaller than the grid), L1 and
 *   L2 in {32, ..., 512}, G <= 256 dividing both, L1 L2 / (1024 G) in 1..4
 *   (workgroups of 256 threads) or L1 L2 / G = 512 (128 threads), and all
 *   G x resident_spread workgroups co-resident; a barrier that waits longer
 *   than one second abandons the solve and it returns BCCB_E_DEVICE.
 *   With support_columns in effect as well, ISTA, FISTA and ADMM run the
 *   pruned cooperative form when it fits: each group publishes its own rows'
 *   parts of DFT2 of the iterate (ADMM: of z - v) at the support bins (Omega's
 *   nonzeros, eq. (21); (Omega + rho)^-1 differs from 1 / rho only there),
 *   and after one grid barrier per iteration every group adds all parts and
 *   builds its rows' correction from them, so only nsup values per group
 *   cross between groups; it has 4 resident_block / L1 rows per group of
 *   resident_block threads (L2 L1 / (4 resident_block) groups, the value of
 *   resident_groups then only switching it on) and needs
 *   its rows' twiddles at the support bins, the row transform areas and the
 *   support tables in 64 KB of LDS.
 *   resident_spread: 1, 2, 4 or 8 -- as row_spread, for the cooperative launch.
 *   resident_block: 256 or 512 (0 = 256) -- threads per group of the pruned
 *   cooperative form.
 * The configuration changes timing only; results agree to FP32 rounding.
 */
typedef struct {
  int row_elems;
  int row_rows_per_block;
  int col_elems;
  int col_cols_per_block;
  int use_graph;
  int spectral_support;
  int row_spread;
  int col_spread;
  int sparse_iterate;
  int support_columns;
  int prow_elems;
  int prow_rows_per_block;
  int pcol_elems;
  int pcol_cols_per_block;
  int resident_groups;
  int resident_spread;
  int resident_block;
} bccb_config;

/* Current configuration of a plan (a heuristic until set or tuned). */
int bccb_plan_get_config(bccb_plan_t plan, bccb_config* cfg);

/*
 * bccb_plan_support_columns -- *ncols (nullable): number of spectral columns k1
 *   holding support bins of Omega (Sec. III-A, eq. (21)); *pruned (nullable):
 *   1 if ISTA / FISTA solves on this plan take the pruned passes under the
 *   current configuration (support_columns and spectral_support set, the
 *   columns few enough), 2 if they take the pruned form of the cooperative
 *   solver (resident_groups set as well, and that form launchable), else 0.
 */
int bccb_plan_support_columns(bccb_plan_t plan, int* ncols, int* pruned);

/* Set a configuration; BCCB_E_INVALID if a pass shape cannot be launched. */
int bccb_plan_set_config(bccb_plan_t plan, const bccb_config* cfg);

/*
 * bccb_plan_autotune -- time every launchable (E, rows per block) of the FISTA
 *   row pass and every (E, columns per block) of the column pass on the plan's
 *   workspace (`reps` launches each, hipEvents), keep the fastest, and return
 *   it in *chosen (nullable).  Where the plan has a kept-column set (see
 *   support_columns) the pruned passes are tuned too, and support_columns is
 *   set to whichever pair is faster per iteration (when spectral_support is on).
 *   With the spectral support on, the chosen passes and every launchable
 *   cooperative shape (resident_groups, resident_spread) are then timed as the
 *   iterations of a 200-iteration FISTA solve (reps / 10 solves each, at least
 *   one; the passes replayed from their captured graph when use_graph is set)
 *   and the fastest is kept (resident_groups = 0 for the passes).
 *   use_graph is left as it was.
 */
int bccb_plan_autotune(bccb_plan_t plan, int reps, bccb_config* chosen);

/*
 * bccb_profile_passes -- measured duration of one solver iteration's passes.
 *   Launches `reps` column passes, then `reps` row passes, of `solver`
 *   (0 = ISTA, 1 = FISTA, 2 = ADMM) back to back on the plan's stream over the
 *   plan's own workspace (whatever it holds; outputs are discarded), each
 *   group bracketed by hipEvents, and returns the average milliseconds per
 *   launch.  reps >= 1.  Used for the live roofline figures of the benchmark.
 */
int bccb_profile_passes(bccb_plan_t plan, int solver, int reps, double* col_ms, double* row_ms);

/*
 * bccb_profile_resident -- measured duration of one cooperative solve (see
 *   resident_groups) of `iters` iterations of `solver` (0 = ISTA, 1 = FISTA,
 *   2 = ADMM): `reps` launches back to back on the plan's stream over the plan's
 *   own workspace (whatever it holds; outputs are discarded), bracketed by
 *   hipEvents; *ms = average milliseconds per launch, including the small
 *   kernel that clears the barrier counter before each.  BCCB_E_UNSUPPORTED if
 *   the plan's solves do not take the cooperative solver.
 */
int bccb_profile_resident(bccb_plan_t plan, int solver, int iters, int reps, double* ms);

#ifdef __cplusplus
}
#endif

#endif /* BCCB_H */
