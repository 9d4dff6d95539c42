// Explicit x-sweep instantiations with general (anisotropic) material rows,
// f64, for one group of line lengths.
#include "hm_aniso_kernels.hpp"

namespace hm {

#define HM_GROUP_SIZES(X) X(105) X(125) X(135) X(147) X(175) X(189) X(225) X(243)
#define X(N) make_aniso_kernels<double, N>(),
static const AnisoKernels kTable[] = {HM_GROUP_SIZES(X)};
#undef X

const AnisoKernels* aniso_kernels_f64_g1(int n) {
  for (const AnisoKernels& k : kTable)
    if (k.n == n) return &k;
  return nullptr;
}

}  // namespace hm
