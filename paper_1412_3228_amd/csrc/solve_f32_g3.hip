// Explicit kernel instantiations of the f32 solver for one group of line
// lengths (split over translation units to compile in parallel).
#include "hm_solve_kernels.hpp"

namespace hm {

#define HM_GROUP_SIZES(X) X(175) X(189) X(225) X(243)
#define X(N) make_axis_kernels<float, N>(),
static const AxisKernels kTable[] = {HM_GROUP_SIZES(X)};
#undef X

const AxisKernels* axis_kernels_f32_g3(int n) {
  for (const AxisKernels& k : kTable)
    if (k.n == n) return &k;
  return nullptr;
}

}  // namespace hm
