// Internal layout of a bccb plan (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "bccb.h"

struct bccb_plan_s {
  int M1 = 0, M2 = 0, L1 = 0, L2 = 0, M = 0;
  long L = 0;
  double mu = 0.0;                 // 1 / max(Omega)
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<float> omega32;      // host copy of the FP32 eigenvalue grid [L2][L1]

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
};
