// Explicit kernel instantiations of the f32 solver for the line lengths
// with a factor 11 or 13 (one schedule per sweep).
#include "hm_solve_kernels.hpp"

namespace hm {

#define HM_GROUP_SIZES(X) X(11) X(13) X(33) X(39) X(55) X(65) X(77) X(91) X(99) X(117) X(121)
#define X(N) make_axis_kernels_basic<float, N>(),
static const AxisKernels kTable[] = {HM_GROUP_SIZES(X)};
#undef X

const AxisKernels* axis_kernels_f32_g4(int n) {
  for (const AxisKernels& k : kTable)
    if (k.n == n) return &k;
  return nullptr;
}

}  // namespace hm
