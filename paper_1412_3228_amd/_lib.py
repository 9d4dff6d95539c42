"""ctypes declarations of the C ABI in include/hm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhm.so")

HM_OK = 0
HM_NOT_CONVERGED = 1
HM_STALLED = 2
HM_DIVERGED = 3
HM_E_ARG = -1
HM_E_SIZE = -2
HM_E_NOMEM = -3
HM_E_DEVICE = -4
HM_E_DATA = -5

RULES = {"none": 0, "voigt": 1, "reuss": 2, "laminate": 3}
PRECS = {"fp64": 0, "mixed": 1}
# sphere capacity of hm_filter_noalloc (HM_FILTER_NOALLOC_MAX_SPHERES in include/hm.h)
HM_FILTER_NOALLOC_MAX_SPHERES = 3072
METHODS = {"fixed_point": 0, "cg": 1}

# Every symbol include/hm.h declares.
EXPORTS = ("hm_filter", "hm_filter_noalloc", "hm_solve", "hm_effective_tensor", "hm_effective_tensor_batch", "hm_solve_adjoint",
           "hm_conduct_solve", "hm_effective_conductivity", "hm_fourier_series", "hm_stiffness_component",
           "hm_filter_phases", "hm_solve_phases", "hm_effective_tensor_phases", "hm_solve_aniso",
           "hm_effective_tensor_aniso", "hm_stress_field", "hm_flux_field", "hm_last_error", "hm_last_timing",
           "hm_last_history", "hm_schedule_count", "hm_release_plans",
           "hm_device_ok")


class HmGrid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3)]


class HmIso(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_double), ("mu", ctypes.c_double)]


class HmSphere(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double * 3), ("r", ctypes.c_double)]


class HmSolveOpts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("c0_alpha", ctypes.c_double), ("check_every", ctypes.c_int),
                ("stall_window", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("profile", ctypes.c_int), ("autotune", ctypes.c_int), ("schedule", ctypes.c_int),
                ("method", ctypes.c_int)]


class HmTiming(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("n_load", ctypes.c_int), ("ms", ctypes.c_double * 5),
                ("x_lines", ctypes.c_int), ("y_width", ctypes.c_int), ("z_width", ctypes.c_int),
                ("z_threads", ctypes.c_int), ("z_groups", ctypes.c_int),
                ("kernel", (ctypes.c_char * 64) * 5), ("active_loads", ctypes.c_double)]


class HmProblem(ctypes.Structure):
    _fields_ = [("grid", HmGrid), ("phases", HmIso * 2), ("rule", ctypes.c_int), ("d_frac", ctypes.c_void_p),
                ("d_incl", ctypes.c_void_p), ("spheres", ctypes.POINTER(HmSphere)), ("n_spheres", ctypes.c_int)]


class HmReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("err", ctypes.c_double),
                ("err0", ctypes.c_double), ("seconds", ctypes.c_double)]


_P = ctypes.POINTER
_vp = ctypes.c_void_p
_dp = _P(ctypes.c_double)
_lib = None


class HmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("hm error %d: %s" % (code, msg))
        self.code = code


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libhm.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libhm.so is not built (%s); run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    lib.hm_filter.argtypes = [_P(HmGrid), _P(HmSphere), ctypes.c_int, ctypes.c_double, ctypes.c_int,
                              ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp]
    lib.hm_filter_noalloc.argtypes = lib.hm_filter.argtypes
    lib.hm_solve.argtypes = [_P(HmGrid), _P(HmIso), ctypes.c_int, _vp, _vp, _P(HmSphere), ctypes.c_int,
                             _dp, ctypes.c_int, _P(HmSolveOpts), _vp, _dp, _P(HmReport), _vp]
    lib.hm_effective_tensor.argtypes = [_P(HmGrid), _P(HmIso), ctypes.c_int, _vp, _vp, _P(HmSphere),
                                        ctypes.c_int, _P(HmSolveOpts), _dp, _vp, _P(HmReport), _vp]
    lib.hm_effective_tensor_batch.argtypes = [_P(HmProblem), ctypes.c_int, _P(HmSolveOpts), _dp, _P(HmReport),
                                              _vp]
    lib.hm_solve_adjoint.argtypes = [_P(HmGrid), _P(HmIso), ctypes.c_int, _vp, _vp, _P(HmSphere),
                                     ctypes.c_int, ctypes.c_int, _dp, _vp, ctypes.c_int, _dp, _vp, _vp]
    lib.hm_conduct_solve.argtypes = [_P(HmGrid), _dp, ctypes.c_int, _vp, _vp, _P(HmSphere), ctypes.c_int,
                                     _dp, ctypes.c_int, _P(HmSolveOpts), _vp, _dp, _P(HmReport), _vp]
    lib.hm_effective_conductivity.argtypes = [_P(HmGrid), _dp, ctypes.c_int, _vp, _vp, _P(HmSphere),
                                              ctypes.c_int, _P(HmSolveOpts), _dp, _vp, _P(HmReport), _vp]
    lib.hm_fourier_series.argtypes = [_P(HmGrid), _P(ctypes.c_int), ctypes.c_int, _vp, _vp, _vp]
    lib.hm_flux_field.argtypes = [_P(HmGrid), _dp, ctypes.c_int, _vp, _vp, _P(HmSphere), ctypes.c_int, ctypes.c_int,
                                  _vp, ctypes.c_int, _vp, _vp]
    lib.hm_stress_field.argtypes = [_P(HmGrid), _P(HmIso), ctypes.c_int, _vp, _vp, _P(HmSphere), ctypes.c_int,
                                    ctypes.c_int, _vp, ctypes.c_int, _vp, _vp]
    lib.hm_solve_aniso.argtypes = [_P(HmGrid), _dp, ctypes.c_int, _vp, _vp, _P(HmSphere), ctypes.c_int, _dp,
                                   ctypes.c_int, _P(HmSolveOpts), _vp, _dp, _P(HmReport), _vp]
    lib.hm_effective_tensor_aniso.argtypes = [_P(HmGrid), _dp, ctypes.c_int, _vp, _vp, _P(HmSphere), ctypes.c_int,
                                              _P(HmSolveOpts), _dp, _vp, _P(HmReport), _vp]
    lib.hm_filter_phases.argtypes = [_P(HmGrid), _P(HmSphere), _P(ctypes.c_int), ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]
    lib.hm_solve_phases.argtypes = [_P(HmGrid), _P(HmIso), ctypes.c_int, ctypes.c_int, _vp, _dp, ctypes.c_int,
                                    _P(HmSolveOpts), _vp, _dp, _P(HmReport), _vp]
    lib.hm_effective_tensor_phases.argtypes = [_P(HmGrid), _P(HmIso), ctypes.c_int, ctypes.c_int, _vp,
                                               _P(HmSolveOpts), _dp, _vp, _P(HmReport), _vp]
    lib.hm_stiffness_component.argtypes = [_P(HmGrid), _P(HmIso), ctypes.c_int, _vp, _vp, _P(HmSphere),
                                           ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp]
    for f in ("hm_filter", "hm_filter_noalloc", "hm_solve", "hm_effective_tensor", "hm_effective_tensor_batch", "hm_solve_adjoint",
              "hm_conduct_solve", "hm_effective_conductivity", "hm_fourier_series", "hm_stiffness_component",
              "hm_filter_phases", "hm_solve_phases", "hm_effective_tensor_phases", "hm_solve_aniso",
              "hm_effective_tensor_aniso", "hm_stress_field", "hm_flux_field", "hm_device_ok"):
        getattr(lib, f).restype = ctypes.c_int
    lib.hm_schedule_count.argtypes = [_P(HmGrid), ctypes.c_int, _P(ctypes.c_int), _P(ctypes.c_int),
                                      _P(ctypes.c_int)]
    lib.hm_schedule_count.restype = ctypes.c_int
    lib.hm_last_timing.argtypes = [_P(HmTiming)]
    lib.hm_last_timing.restype = ctypes.c_int
    lib.hm_last_history.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp]
    lib.hm_last_history.restype = ctypes.c_int
    lib.hm_last_error.argtypes = []
    lib.hm_last_error.restype = ctypes.c_char_p
    lib.hm_release_plans.argtypes = []
    lib.hm_release_plans.restype = None
    lib.hm_device_ok.argtypes = []
    _lib = lib
    return lib


def check(rc: int, allow_warnings: bool = True) -> int:
    """Raises HmError on a negative code; returns warnings (>0) unchanged."""
    if rc < 0 or (rc > 0 and not allow_warnings):
        msg = load().hm_last_error().decode()
        raise HmError(rc, msg)
    return rc
