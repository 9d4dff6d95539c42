// Explicit kernel instantiations of the f32 solver for one group of line
// lengths (split over translation units to compile in parallel).
#include "hm_solve_kernels.hpp"

namespace hm {

#define HM_GROUP_SIZES(X) X(1) X(3) X(5) X(7) X(9) X(15) X(21) X(25) X(27) X(35)
#define X(N) make_axis_kernels<float, N>(),
static const AxisKernels kTable[] = {HM_GROUP_SIZES(X)};
#undef X

const AxisKernels* axis_kernels_f32_g0(int n) {
  for (const AxisKernels& k : kTable)
    if (k.n == n) return &k;
  return nullptr;
}

}  // namespace hm
