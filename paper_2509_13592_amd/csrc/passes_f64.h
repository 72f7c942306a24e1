// Launch interface of the FP64 passes (passes_f64.hip; internal to libbccb).  Returns 0, -1
// (size not supported) or -4 (HIP error).
#pragma once

#include <hip/hip_runtime.h>

namespace bccb {

enum RowMode64 {
  ROW64_FWD = 0,    // xy = DFT_rows(src)              (src == nullptr -> zeros)
  ROW64_INV = 1,    // dst = scale * IDFT_rows(xy)
  ROW64_ISTA = 2,   // c = S_k(IDFT_rows(xy) + rhs); xy = DFT_rows(c)
  ROW64_FISTA = 3,  // c = S_k(IDFT_rows(xy) + rhs); z = c + beta (c - state); state = c; xy = DFT_rows(z)
  ROW64_ADMM = 4,   // c = rhs + IDFT_rows(xy); z = S_k(c + v); v += c - z; xy = DFT_rows(z - v)
};

enum ColMode64 {
  COL64_AFFINE = 0,  // xy = IDFT_cols((ca + cb Omega) . DFT_cols(xy))
  COL64_ADMM = 1,    // xy = IDFT_cols(scale / (Omega + rho) . DFT_cols(xy))
  COL64_INV = 2,     // xy = IDFT_cols(xy)
};

struct RowArgs64 {
  int mode = ROW64_FWD;
  double2* xy = nullptr;
  const double2* src = nullptr;
  double2* dst = nullptr;
  const double2* rhs = nullptr;
  double2* state = nullptr;
  double2* out_c = nullptr;
  double2* out_z = nullptr;
  const double2* tw = nullptr;   // [N] e^{-j 2 pi j / N}
  int* flag = nullptr;
  int nrows = 0, rows_per_scene = 1;
  double kappa = 0.0, beta = 0.0, scale = 1.0;
  int last = 0;
  int act_cols = 0, act_rows = 0;   // coefficient window (0 = the whole grid)
};

struct ColArgs64 {
  int mode = COL64_AFFINE;
  double2* xy = nullptr;
  const double* omega = nullptr;   // [N][L1]
  const double2* tw = nullptr;
  int L1 = 0;
  double ca = 0.0, cb = 0.0, scale = 1.0, rho = 0.0;
};

int launch_row64(int N, const RowArgs64& a, hipStream_t s);
int launch_col64(int N, const ColArgs64& a, hipStream_t s);
int launch_scatter64(const double2* y, const int* sensor_of, int M1, int M2, int L1, int L2, double scale,
                     double2* S, int* flag, hipStream_t s);
int launch_fill64(double2* p, long n, hipStream_t s);
// xy[i] /= omega[i] + rho, i < n
int launch_spectral_div64(double2* xy, const double* omega, double rho, long n, hipStream_t s);
int launch_copy64(double2* d, const double2* src, long n, hipStream_t s);

}  // namespace bccb
