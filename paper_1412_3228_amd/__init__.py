"""MI355X (gfx950) filtered-property Lippmann-Schwinger solver.

Method: L. Gelebart, F. Ouaki, "Filtering material properties to improve
FFT-based methods for numerical homogenization" (arXiv:1412.3228).  The
compute path is the HIP library libhm.so (C ABI in include/hm.h); this
package is its thin Python binding.
"""
from .api import (  # noqa: F401
    EffectiveTensor,
    HmSolveError,
    device_ok,
    hm_conduct_solve,
    hm_effective_conductivity,
    hm_effective_tensor,
    hm_effective_tensor_aniso,
    hm_effective_tensor_batch,
    hm_effective_tensor_phases,
    hm_filter,
    hm_filter_noalloc,
    hm_filter_phases,
    hm_flux_field,
    hm_fourier_series,
    hm_solve,
    hm_solve_aniso,
    hm_solve_adjoint,
    hm_solve_phases,
    hm_stiffness_component,
    hm_stress_field,
    last_history,
    last_timing,
    release_plans,
    schedule_count,
)
from ._lib import EXPORTS, HmError, LIB_PATH, load  # noqa: F401
