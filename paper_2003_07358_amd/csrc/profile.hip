// Optional per-kernel timing with HIP events (diagnostics entry points).
// Events are created up front by fhs_plan_profile; compute calls only record
// them on the launch stream around the selected kernel.
#include <hip/hip_runtime.h>

#include "fhs_internal.h"

namespace fhs {

void prof_begin(const fhs_plan *p, int kid, void *stream) {
  if (p->prof_kernel != kid) return;
  const int n = static_cast<int>(p->prof_events.size()) / 2;
  if (p->prof_next >= n) return;
  (void)hipEventRecord(static_cast<hipEvent_t>(p->prof_events[2 * p->prof_next]), static_cast<hipStream_t>(stream));
}

void prof_end(const fhs_plan *p, int kid, void *stream) {
  if (p->prof_kernel != kid) return;
  const int n = static_cast<int>(p->prof_events.size()) / 2;
  if (p->prof_next >= n) return;
  (void)hipEventRecord(static_cast<hipEvent_t>(p->prof_events[2 * p->prof_next + 1]), static_cast<hipStream_t>(stream));
  ++p->prof_next;
}

void prof_release(fhs_plan *p) {
  for (void *e : p->prof_events) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
  p->prof_events.clear();
  p->prof_next = 0;
  p->prof_kernel = -1;
}

}  // namespace fhs

using namespace fhs;

extern "C" {

int fhs_plan_profile(fhs_plan *p, int32_t kernel_id, int32_t max_launches) {
  if (!p) return fail(FHS_EINVAL, "fhs_plan_profile: null plan");
  if (kernel_id < -1 || kernel_id >= FHS_K_COUNT) return fail(FHS_EINVAL, "unknown kernel id");
  prof_release(p);
  if (kernel_id < 0) return FHS_OK;
  if (max_launches < 1 || max_launches > 65536) return fail(FHS_EINVAL, "max_launches must be in 1..65536");
  for (int i = 0; i < 2 * max_launches; ++i) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
      prof_release(p);
      return fail(FHS_EHIP, "hipEventCreate failed");
    }
    p->prof_events.push_back(e);
  }
  p->prof_kernel = kernel_id;
  return FHS_OK;
}

int fhs_plan_profile_read(fhs_plan *p, double *total_ms, int64_t *launches) {
  if (!p || !total_ms || !launches) return fail(FHS_EINVAL, "fhs_plan_profile_read: null argument");
  double tot = 0.0;
  for (int i = 0; i < p->prof_next; ++i) {
    hipEvent_t a = static_cast<hipEvent_t>(p->prof_events[2 * i]);
    hipEvent_t b = static_cast<hipEvent_t>(p->prof_events[2 * i + 1]);
    if (hipEventSynchronize(b) != hipSuccess) return fail(FHS_EHIP, "hipEventSynchronize failed");
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return fail(FHS_EHIP, "hipEventElapsedTime failed");
    tot += ms;
  }
  *total_ms = tot;
  *launches = p->prof_next;
  p->prof_next = 0;
  return FHS_OK;
}

}  // extern "C"
