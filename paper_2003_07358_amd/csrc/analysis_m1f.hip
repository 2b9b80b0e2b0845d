// SARA analysis kernels of mode 1 with FP32 accumulation: the mixed-precision
// form of the l21 dual update (see analysis_impl.h).
#include "analysis_impl.h"

namespace fhs {
int launch_analysis_m1f(const AnaArgs &a, int nthreads, bool first, size_t lds, void *stream) {
  return ana::launch_mode<1, float>(a, nthreads, first, lds, stream);
}
}  // namespace fhs
