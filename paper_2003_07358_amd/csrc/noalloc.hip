// fhs_facet_prox_step_noalloc: the facet step with the library's own static
// device scratch in place of a caller-attached workspace, for callers that
// cannot allocate device memory (code under graph capture, tight serving
// loops, harnesses that forbid allocation).
//
// The scratch is one file-scope __device__ array of kScratchBytes; every GPU
// the library runs on holds its own copy until the process ends.  Host code
// never uses the array's name as an address: its device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and kept.
// Calls on one GPU share the array (it keeps the previous call's contents;
// the step writes every workspace word it reads before reading it, so
// nothing needs clearing), so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "fhs_internal.h"

namespace fhs {

namespace {

constexpr int64_t kScratchBytes = int64_t(32) << 20;  // 32 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// thread-local workspace override of the compute sequences (null: the plan's)
thread_local void *tl_ws = nullptr;

// Device address of this device's scratch, looked up on first use.
int scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(FHS_EHIP, "fhs_facet_prox_step_noalloc: no current HIP device");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FHS_EHIP, std::string("fhs_facet_prox_step_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FHS_OK;
}

struct WorkspaceScope {
  void *prev;
  explicit WorkspaceScope(void *ws) : prev(tl_ws) { tl_ws = ws; }
  ~WorkspaceScope() { tl_ws = prev; }
};

}  // namespace

void *ws_base(const fhs_plan *p) { return tl_ws ? tl_ws : p->ws; }

}  // namespace fhs

using namespace fhs;

extern "C" {

int64_t fhs_noalloc_scratch_bytes(void) { return kScratchBytes; }

int fhs_facet_prox_step_noalloc(const fhs_plan *p, const float *xcheck, float *pdual, float *w, const float *theta,
                                const double *theta_bar, const double *mu, const double *mu_bar, double zeta,
                                double kappa, float *grad, void *stream) {
  if (!p) return fail(FHS_EINVAL, "null plan");
  if (!xcheck || !pdual || !w || !theta || !theta_bar || !mu || !mu_bar || !grad)
    return fail(FHS_EINVAL, "fhs_facet_prox_step_noalloc: null array");
  if (!(zeta > 0) || !(kappa > 0)) return fail(FHS_EINVAL, "zeta and kappa must be positive");
  if (p->ws_bytes > kScratchBytes)
    return fail(FHS_EUNSUPPORTED, "fhs_facet_prox_step_noalloc: the plan needs " + std::to_string(p->ws_bytes) +
                                      " bytes of workspace, more than the " + std::to_string(kScratchBytes) +
                                      "-byte static scratch (use fhs_facet_prox_step with a workspace)");
  void *ptr = nullptr;
  if (int rc = scratch_address(&ptr)) return rc;
  WorkspaceScope scope(ptr);
  return facet_prox_step(p, xcheck, pdual, w, theta, theta_bar, mu, mu_bar, zeta, kappa, grad, stream, nullptr);
}

}  // extern "C"
