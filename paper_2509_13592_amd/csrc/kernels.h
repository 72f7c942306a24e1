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
};

// Launch shape of the passes for one transform length: E elements per thread
// (T = N/E threads per transform), rows per block of the row pass, columns per
// block of the column pass.
struct PassCfg {
  int E = 16;
  int rpb = 1;
  int W = 1;
};

// Returns 0, -1 (shape not launchable), -2 (size not compiled), -4 (HIP error).
int launch_row(int N, const PassCfg& cfg, int mode, const RowArgs& a, hipStream_t s);
int launch_col(int N, const PassCfg& cfg, int mode, const ColArgs& a, hipStream_t s);

#define BCCB_DECLARE_N(n)                                                                  \
  int row_launch_##n(int E, int mode, const RowArgs& a, int rpb, hipStream_t s);           \
  int col_launch_##n(int E, int mode, const ColArgs& a, int W, hipStream_t s);
BCCB_DECLARE_N(8)
BCCB_DECLARE_N(16)
BCCB_DECLARE_N(32)
BCCB_DECLARE_N(64)
BCCB_DECLARE_N(128)
BCCB_DECLARE_N(256)
BCCB_DECLARE_N(512)
BCCB_DECLARE_N(1024)
#undef BCCB_DECLARE_N

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
