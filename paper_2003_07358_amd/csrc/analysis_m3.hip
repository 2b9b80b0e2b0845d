// SARA analysis kernels of mode 3 (see analysis_impl.h): the l21 dual update
// restricted to the coefficient rows of selected facets.
#include "analysis_impl.h"

namespace fhs {
int launch_analysis_m3(const AnaArgs &a, int nthreads, bool first, size_t lds, void *stream) {
  return a.f32 ? ana::launch_mode<3, float>(a, nthreads, first, lds, stream)
               : ana::launch_mode<3, double>(a, nthreads, first, lds, stream);
}
}  // namespace fhs
