// SARA analysis kernels of mode 0 (see analysis_impl.h).
#include "analysis_impl.h"

namespace fhs {
int launch_analysis_m0(const AnaArgs &a, int nthreads, bool first, size_t lds, void *stream) {
  return ana::launch_mode<0>(a, nthreads, first, lds, stream);
}
}  // namespace fhs
