// Explicit kernel instantiations of the f64 conduction solver for one group
// of line lengths (split over translation units to compile in parallel).
#include "hm_conduct_kernels.hpp"

namespace hm {

#define HM_GROUP_SIZES(X) X(105) X(125) X(135) X(147) X(175) X(189) X(225) X(243)
#define X(N) make_cond_kernels<double, N>(),
static const CondKernels kTable[] = {HM_GROUP_SIZES(X)};
#undef X

const CondKernels* cond_kernels_f64_g1(int n) {
  for (const CondKernels& k : kTable)
    if (k.n == n) return &k;
  return nullptr;
}

}  // namespace hm
