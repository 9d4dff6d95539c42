// Explicit kernel instantiations of the f64 conduction solver for one group
// of line lengths (split over translation units to compile in parallel).
#include "hm_conduct_kernels.hpp"

namespace hm {

#define HM_GROUP_SIZES(X) X(1) X(3) X(5) X(7) X(9) X(15) X(21) X(25) X(27) X(35) X(45) X(49) X(63) X(75) X(81)
#define X(N) make_cond_kernels<double, N>(),
static const CondKernels kTable[] = {HM_GROUP_SIZES(X)};
#undef X

const CondKernels* cond_kernels_f64_g0(int n) {
  for (const CondKernels& k : kTable)
    if (k.n == n) return &k;
  return nullptr;
}

}  // namespace hm
