// Host-side launch interface of the single-scene cooperative solver
// (resident.h; internal to libbccb).
#pragma once

#include "kernels.h"

namespace bccb {

// One cooperative launch runs a whole ISTA, FISTA or ADMM solve of one scene:
// G workgroups own L2/G rows and L1/G columns each and meet at grid barriers
// between the column and the row phase of every iteration.
enum ResidentMode {
  RES_ISTA = 0,
  RES_FISTA = 1,
  RES_ADMM = 2,
  // pruned forms: each group's part of the spectrum at the support bins is all
  // that crosses between groups, and every group adds up all the parts, so an
  // iteration needs one grid barrier
  RES_PRUNED_ISTA = 3,
  RES_PRUNED_FISTA = 4,
  RES_PRUNED_ADMM = 5,
};

constexpr int kResidentMaxChunks = 4;   // 1024-point chunks per workgroup and phase (256 threads)
constexpr int kResidentMaxGroups = 256;
constexpr int kResidentArriveOffset = 16;   // 64-bit sync words: [0] abort, then one arrival word per group
constexpr int kResidentArriveStride = 16;   // (64-bit words) one 128-byte line per arrival word
constexpr int kResidentSyncWords = kResidentArriveOffset + kResidentMaxGroups * kResidentArriveStride;

struct ResidentArgs {
  float2* xy = nullptr;             // [L2][L1] row spectra exchanged between the phases
                                    // (pruned forms: [2][groups][nsup] per-group parts)
  const float2* init = nullptr;     // ISTA/FISTA warm start c^(0) (nullable = 0)
  float2* out_c = nullptr;          // ISTA/FISTA c^(T); ADMM c^(T) (nullable)
  float2* out_z = nullptr;          // ADMM z^(T)
  const float2* tw1 = nullptr;      // [L1] e^{-j 2 pi j / L1}
  const float2* tw2 = nullptr;      // [L2]
  const float* beta = nullptr;      // FISTA: momentum of iteration t at beta[t - 1]
  const float2* coef = nullptr;     // ISTA/FISTA: (a, b) of the multiplier a + b Omega (device)
  const int* sup_ptr = nullptr;     // support bins of column k1: sup[sup_ptr[k1] .. sup_ptr[k1 + 1])
  const SupEntry* sup = nullptr;
  const float2* sup_rhs = nullptr;  // right-hand side on the support bins
  float kappa = 0.f, rho = 0.f, scale = 1.f;
  int iters = 0;
  int groups = 1;                   // G: workgroups that work
  int spread = 1;                   // launch spread x G workgroups, every spread-th works (see PassCfg)
  // [kResidentSyncWords] 64-bit words: the abort word (the tag of a solve being abandoned)
  // and the arrival words (tag | barrier number); they are never reset: tags grow from
  // solve to solve, so what earlier solves left is always below what this one waits for
  unsigned long long* sync = nullptr;
  unsigned long long tag = 0;       // this solve's id in the high 32 bits
  int* flag = nullptr;              // |= 1: non-finite warm start; |= 2: a barrier wait timed out
  long long timeout_ticks = 0;      // wall-clock ticks one barrier wait may take
  // pruned forms: xy holds [G][nsup] per-group parts of DFT2 of the iterate at the support
  // bins; scol[s] = spectral column of slot s (-1 = padding), colslot[k1] = slot of
  // column k1 (-1 = not kept); nsup = entries of sup
  const int* scol = nullptr;
  const int* colslot = nullptr;
  int ncs = 0;
  int nsup = 0;
};

// Returns 0, -1 (shape or arguments not launchable, or not co-resident), -2 (size
// not compiled), -4 (HIP error).  check_only: validate the shape and residency only.
int launch_resident(int L1, int L2, int mode, const ResidentArgs& a, int check_only, hipStream_t s);

int resident_launch_32(int L2, int mode, const ResidentArgs& a, int check_only, hipStream_t s);
int resident_launch_64(int L2, int mode, const ResidentArgs& a, int check_only, hipStream_t s);
int resident_launch_128(int L2, int mode, const ResidentArgs& a, int check_only, hipStream_t s);
int resident_launch_256(int L2, int mode, const ResidentArgs& a, int check_only, hipStream_t s);
int resident_launch_512(int L2, int mode, const ResidentArgs& a, int check_only, hipStream_t s);

}  // namespace bccb
