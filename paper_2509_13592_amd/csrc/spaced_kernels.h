// Launchers of the zero-padded-embedding kernels (spaced_kernels.hip).  Return 0, -1 (shape
// not launchable) or -4 (HIP error).
#pragma once

#include <hip/hip_runtime.h>

namespace bccb {

// out (out_cols x out_rows window, row stride ld) = scale * D_s^H y on the A1 x A2 grid,
// zero elsewhere in the window: U[m2][l1] = scale sum_{m1} conj(W1[m1][l1]) y(m1, m2), then
// out[l2][l1] = sum_{m2} conj(W2[m2][l2]) U[m2][l1] (eq. (4) factored).  U: M2 * A1 scratch.
int launch_sep_adjoint(const float2* y, const int* sensor_of, const float2* W1, const float2* W2, int M1, int M2,
                       int A1, int A2, float scale, float2* U, int out_cols, int out_rows, int ld, float2* out,
                       int* flag, hipStream_t s);

// Per-block partial sums (double) of 1/2 |y_m - (D_s c)_m|^2 with D_s c = (W2 C W1^T) at the
// kept elements (c: A2 rows of A1, row stride ldc).  T: A2 * M1 scratch.
int launch_sep_resid(const float2* c, int ldc, const float2* W1, const float2* W2, const int2* sensors,
                     const float2* y, int M, int M1, int A1, int A2, float2* T, double* partial, int* nblocks,
                     int* flag, hipStream_t s);

// dst [P2][P1] = src [A2][A1] zero-padded (src == nullptr: zeros); dst [A2][A1] = window of src [..][P1]
int launch_pad(const float2* src, int A1, int A2, int P1, int P2, float2* dst, hipStream_t s);
int launch_crop(const float2* src, int A1, int A2, int P1, float2* dst, hipStream_t s);

}  // namespace bccb
