// Allocation-free FISTA solve: lasso_solve_fista_noalloc.
//
// The same iterations as lasso_solve_fista (eqs. (10)-(12), through the full
// row and column passes of eq. (23)) for callers that cannot allocate device
// memory.  Every buffer the passes need beyond the caller's snapshot and
// output -- the row-spectral iterate, the right-hand side, the scattered
// snapshot, the support-bin right-hand side with its descriptor, the
// non-finite flag -- lives in one file-scope device array, `scratch`, whose
// address on each device is resolved once (the first call with that device
// current) and kept.  The call enqueues fills, copies and kernels only: no
// hipMalloc, no hipFree, no graph instantiation.
//
// Every call on one GPU shares that GPU's array: calls that overlap on one
// device (two host threads, or two streams in flight) race on it.  Calls are
// synchronous (they drain the plan's stream before returning), so one thread
// issuing them in turn is safe.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "plan_internal.h"

namespace {

// Largest grid (points) the array is sized for: 2^18 = 512 x 512.
constexpr long kMaxPoints = 1L << 18;
// Layout (bytes): [flag: 256][support descriptor: 256][iterate spectrum: 8 Lmax]
// [right-hand side grid / support right-hand side: 8 Lmax][scattered snapshot: 8 Lmax]
constexpr size_t kHead = 512;
constexpr size_t kGrid = 8 * static_cast<size_t>(kMaxPoints);
constexpr size_t kScratchBytes = kHead + 3 * kGrid;   // 6 MiB + 512 B

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};   // device address of `scratch`, per device (nullptr = not resolved)

// Device address of the array on the current device (resolved once per device).
int scratch_on(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return BCCB_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return BCCB_E_DEVICE;
    g_ptr[dev] = ptr;
  }
  *out = static_cast<unsigned char*>(g_ptr[dev]);
  return BCCB_OK;
}

}  // namespace

using namespace bccb;

extern "C" int lasso_solve_fista_noalloc(bccb_plan_t p, const bccb_c32* y, float tau, int iters, const bccb_c32* c0,
                                         bccb_c32* c_out) {
  if (!p || !y || !c_out) return BCCB_E_INVALID;
  if (!(tau >= 0.f) || !std::isfinite(tau) || iters < 0) return BCCB_E_INVALID;
  if (p->emb) return BCCB_E_UNSUPPORTED;   // padded-embedding plans keep their own work grids
  if (p->L > kMaxPoints) return BCCB_E_SCRATCH;
  int dev = -1;
  BCCB_HIP(hipGetDevice(&dev));
  if (dev != p->device) return BCCB_E_INVALID;   // the plan's device must be current
  unsigned char* base = nullptr;
  BCCB_TRY(scratch_on(dev, &base));

  const hipStream_t s = p->stream;
  const long L = p->L;
  int* flag = reinterpret_cast<int*>(base);
  SupRhsDesc* desc = reinterpret_cast<SupRhsDesc*>(base + 256);
  float2* xy = reinterpret_cast<float2*>(base + kHead);
  float2* rhs = reinterpret_cast<float2*>(base + kHead + kGrid);   // mu b grid, or mu S on the support bins
  float2* tmp = reinterpret_cast<float2*>(base + kHead + 2 * kGrid);
  float2* out = reinterpret_cast<float2*>(c_out);
  const float2* init = reinterpret_cast<const float2*>(c0);
  const float2* yy = reinterpret_cast<const float2*>(y);
  const float mu = static_cast<float>(p->mu);
  const bool sparse = sparse_on(p);

  // the array keeps the previous call's contents: the flag starts at zero (a fill
  // kernel, not a memset node); every other region is fully written before it is read
  BCCB_TRY(kern(launch_fill_int(flag, 1, 0, s)));

  // mu D_s^H y: on the support bins of the spectrum (sparse support) or as a grid
  if (sparse) {
    SupRhsDesc& d = *p->h_sup_desc;
    d.y = yy;
    d.entry_off = 0;
    d.nentries = p->nsup;
    d.rhs_off = 0;
    d.scale = mu;
    BCCB_HIP(hipMemcpyAsync(desc, p->h_sup_desc, sizeof(SupRhsDesc), hipMemcpyHostToDevice, s));
    BCCB_TRY(kern(launch_sup_rhs(desc, 1, p->nsup, p->d_src_ptr, p->d_src, rhs, flag, s)));
  } else {
    BCCB_TRY(kern(launch_scatter(yy, p->d_sensor_of, p->M1, p->M2, p->L1, p->L2, mu, tmp, flag, s)));
    ColArgs ci;
    ci.xy = tmp;
    ci.tw = p->d_tw2;
    ci.L1 = p->L1;
    ci.scale = 1.f;
    BCCB_TRY(kern(launch_col(p->L2, p->cfg_col, COL_INV, ci, s)));
    RowArgs ri;
    ri.xy = tmp;
    ri.dst = rhs;
    ri.scale = 1.f;
    ri.tw = p->d_tw1;
    ri.nrows = p->L2;
    ri.rows_per_scene = p->L2;
    BCCB_TRY(kern(launch_row(p->L1, p->cfg_row, ROW_INV, ri, s)));
  }

  // z^(1) = c^(0): its row DFT starts the first column pass; c^(0) goes to the output,
  // which holds c^(t-1) between passes
  RowArgs f;
  f.xy = xy;
  f.src = init;
  f.flag = flag;
  f.tw = p->d_tw1;
  f.nrows = p->L2;
  f.rows_per_scene = p->L2;
  BCCB_TRY(kern(launch_row(p->L1, p->cfg_row, ROW_FWD, f, s)));
  if (init && init != out) BCCB_TRY(kern(launch_copy(out, init, L, s)));
  else if (!init) BCCB_TRY(kern(launch_fill(out, L, s)));

  ColArgs ca;
  ca.xy = xy;
  ca.sup_ptr = p->d_sup_ptr;
  ca.sup = p->d_sup;
  ca.sup_rhs = rhs;
  ca.omega = p->d_omega;
  ca.coef = p->d_coef;   // (1/L, -mu/L): the multiplier (1 - mu Omega)/L
  ca.tw = p->d_tw2;
  ca.L1 = p->L1;
  ca.nscenes = 1;
  ca.scale = 1.f;
  const float kappa = static_cast<float>(p->mu * tau);
  double alpha = 1.0;
  for (int t = 1; t <= iters; ++t) {
    BCCB_TRY(kern(launch_col(p->L2, p->cfg_col, sparse ? COL_SPARSE_AFFINE : COL_FILTER_AFFINE, ca, s)));
    const double alpha_next = (1.0 + std::sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0;
    RowArgs a;
    a.xy = xy;
    a.rhs = sparse ? nullptr : rhs;
    a.state = out;
    a.out_c = out;
    a.kappa = kappa;
    a.beta = static_cast<float>((alpha - 1.0) / alpha_next);
    a.last = (t == iters);
    a.tw = p->d_tw1;
    a.nrows = p->L2;
    a.rows_per_scene = p->L2;
    alpha = alpha_next;
    BCCB_TRY(kern(launch_row(p->L1, p->cfg_row, ROW_FISTA, a, s)));
  }

  BCCB_HIP(hipMemcpyAsync(p->h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  BCCB_HIP(hipStreamSynchronize(s));
  return *p->h_flag ? BCCB_E_NONFINITE : BCCB_OK;
}
