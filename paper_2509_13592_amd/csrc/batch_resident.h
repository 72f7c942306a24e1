// Whole batched FISTA solves in one persistent launch (internal to libbccb).
//
// A workgroup takes a scene from a queue and runs every iteration of its solve
// (eqs. (10)-(12), the product of eq. (23) in the pruned form of the batch's
// support-column classes) before it takes the next one.  The scene's kept row
// spectra [L2][ncs] stay in LDS for the whole solve; the column pass over the
// kept columns and the row pass run in the same workgroup, separated by
// workgroup barriers; the iterate's rows go to the class's slot buffers, which
// only the workgroup holding the scene touches (its die's L2 keeps them), and
// the rows' nonzero counts stay in LDS.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace bccb {

// One size class (square grids L1 = L2 = N), every per-scene array in arena order of the
// physical scene k; a table shared by all scenes takes stride 0.
struct ResidentClass {
  int N = 0;                     // grid length, one of 32, 64, 128, 256
  int n = 0;                     // scenes taken from the queue
  int ncs = 0;                   // kept-column slots per scene
  int xs = 0;                    // LDS row stride of the kept spectra (ncs rounded up to odd)
  int first = 0;                 // queue index of the class's first scene
  const int* colslot = nullptr;  // [N] per scene: spectral column -> slot (-1 = not kept)
  const int* scol = nullptr;     // [ncs] per scene: slot -> spectral column (-1 = padding)
  const int* sup_ptr = nullptr;  // [N + 1] per scene: entry offsets of each spectral column
  long colslot_stride = 0, scol_stride = 0, sup_ptr_stride = 0;
  const SupEntry* sup = nullptr; // support bins (k2, Omega)
  const float2* sup_rhs = nullptr;  // mu * spectral right-hand side of entry j of scene k at k * rhs_stride + j
  long rhs_stride = 0;
  const float2* coef = nullptr;  // per scene (1/L, -mu/L), stride coef_stride
  long coef_stride = 1;
  const float* kscale = nullptr; // per scene; the threshold is kmul * kscale[k]
  float kmul = 1.f;
  const float2* tw = nullptr;    // [N] e^{-j 2 pi j / N}
  const SceneDesc* desc = nullptr;  // [n] output grids (or out_base + k N^2 when out_base is set)
  float2* out_base = nullptr;
  const int* scene_map = nullptr;   // queue position - first -> physical scene (nullable: identity)
  float2* xkeep = nullptr;       // [scenes][N][ncs] kept spectra of z carried between launches (slot order)
  SlotBuf buf[3];                // iterate rows [scenes][N], rotating c_t, c_{t-1}, c_{t-2}; counts in cnt
  // Carrying launches only (nullable): per physical scene, the sum over the grid of e^2,
  // the KKT conditions' violation at the launch's last iterate c (e = g - tau c/|c| where
  // c != 0, max(|g| - tau, 0) elsewhere, g = b - G c, tau = kscale[k]); the column pass
  // leaves the kept spectra of mu (b - G c) and kkt_scale = 1/mu takes the factor out.
  double* kkt_sum = nullptr;
  float kkt_scale = 0.f;
};

// Elements per thread of the transforms (N / 4 threads per row or column).
constexpr int kResidentE = 4;
// The persistent solve keeps an iterate row in slots while it has at most N / 4 nonzeros
// (the early iterations' rows hold 33..64 nonzeros for several iterations, which the pass
// graph's N / 8 stores densely): the class's slot buffers hold N / 4 slots per row.
constexpr int kResidentSlotDiv = 4;

// Workgroup LDS of a class at `nthreads` threads, in bytes: kept spectra N x xs,
// N twiddles, two exchange areas per transform group, the row inverse's twiddles
// (ncs x N/E), three [N] count arrays and the kept-column tables (3 ncs + 8 ints).
constexpr long resident_lds_bytes(int N, int ncs, int nthreads) {
  const int T = N / kResidentE;
  const long G = nthreads / T;
  const long xs = ncs | 1;
  return 8L * (N * xs + N + 2L * G * fft_area(N) + static_cast<long>(ncs) * T) + 12L * N + 4L * (3L * ncs + 8);
}

// Persistent launch over `total` scenes of `ncls` classes (device table `cls`, classes in
// queue order), iterations it0 + 1 .. it0 + steps of each (the iterate buffers rotate with
// the iteration number); beta[t] is the momentum weight of iteration t (beta[it0] that of
// the iteration before the first).  carry = 0: every scene starts from zero and only the
// last iterate is written (to the outputs); carry = 1: the kept spectra of z and the row
// counts of the iterates are loaded from xkeep and buf[].cnt at the start and stored back
// at the end, and the last iterate is written densely to the outputs as well, so a later
// launch continues the solves.  check = 1 (carrying launches only) runs the kernel's
// variant that also leaves each scene's KKT sum in its class's kkt_sum (a separate
// instantiation, so the plain launches keep their register allocation).  *queue = 0 on
// entry.  Returns -1 for a shape the kernel does not take.
int launch_scene_fista(const ResidentClass* cls, int ncls, int total, const float* beta, int it0, int steps,
                       int carry, int check, int* queue, int nthreads, int blocks, size_t lds, hipStream_t s);

// Workgroups of the kernel (the checking variant for check = 1) one compute unit holds at
// this shape (0: does not fit).
int scene_fista_occupancy(int nthreads, size_t lds, int check);

}  // namespace bccb
