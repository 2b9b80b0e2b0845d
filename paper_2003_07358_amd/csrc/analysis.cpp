// Dispatch of the SARA analysis launch on its mode (one translation unit of
// kernels per mode, see analysis_impl.h).
#include "fhs_internal.h"

namespace fhs {

int launch_analysis(const AnaArgs &a, int nthreads, bool first, void *stream) {
  if (a.nbase_wg <= 0 && !(first && a.b[kBases].strips > 0)) return FHS_OK;
  const size_t lds = static_cast<size_t>(a.lds_words) * sizeof(float);
  switch (a.mode) {
    case 0: return launch_analysis_m0(a, nthreads, first, lds, stream);
    case 1: return a.f32 ? launch_analysis_m1f(a, nthreads, first, lds, stream)
                         : launch_analysis_m1(a, nthreads, first, lds, stream);
    case 2: return launch_analysis_m2(a, nthreads, first, lds, stream);
    case 3: return launch_analysis_m3(a, nthreads, first, lds, stream);
    default: return fail(FHS_EINVAL, "analysis: unknown mode");
  }
}

}  // namespace fhs
