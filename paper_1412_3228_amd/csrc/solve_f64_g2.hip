// Explicit kernel instantiations of the f64 solver for one group of line
// lengths (split over translation units to compile in parallel).
#include "hm_solve_kernels.hpp"

namespace hm {

#define HM_GROUP_SIZES(X) X(105) X(125) X(135) X(147)
#define X(N) make_axis_kernels<double, N>(),
static const AxisKernels kTable[] = {HM_GROUP_SIZES(X)};
#undef X

const AxisKernels* axis_kernels_f64_g2(int n) {
  for (const AxisKernels& k : kTable)
    if (k.n == n) return &k;
  return nullptr;
}

}  // namespace hm
