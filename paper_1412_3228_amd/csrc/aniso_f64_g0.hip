// Explicit x-sweep instantiations with general (anisotropic) material rows,
// f64, for one group of line lengths.
#include "hm_aniso_kernels.hpp"

namespace hm {

#define HM_GROUP_SIZES(X) X(3) X(5) X(7) X(9) X(15) X(21) X(25) X(27) X(35) X(45) X(49) X(63) X(75) X(81)
#define X(N) make_aniso_kernels<double, N>(),
static const AnisoKernels kTable[] = {HM_GROUP_SIZES(X)};
#undef X

const AnisoKernels* aniso_kernels_f64_g0(int n) {
  for (const AnisoKernels& k : kTable)
    if (k.n == n) return &k;
  return nullptr;
}

}  // namespace hm
