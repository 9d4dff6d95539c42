"""Python binding of the C ABI (include/hm.h) on torch device tensors.

Only argument marshalling lives here: every step of the filter, the solve
and the gradient runs in the HIP library.  PyTorch provides device memory
and the current stream.  Importing works without a GPU; calling needs the
built library and a gfx950 device, and fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import math
import warnings
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L

_DT = {"fp64": torch.float64, "mixed": torch.float32}


def _lib():
    lib = L.load()
    return lib


def _device(device) -> torch.device:
    d = torch.device(device)
    if d.type != "cuda":
        raise ValueError("the HIP library needs a cuda (HIP) device, got %s" % d)
    return d


def _grid(n: Sequence[int], dim: int) -> L.HmGrid:
    g = L.HmGrid()
    g.dim = int(dim)
    for i in range(3):
        g.n[i] = int(n[i])
    return g


def _spheres(spheres) -> tuple:
    sph = np.asarray(spheres, dtype=np.float64).reshape(-1, 4)
    arr = (L.HmSphere * max(1, sph.shape[0]))()
    for k in range(sph.shape[0]):
        arr[k].c[0], arr[k].c[1], arr[k].c[2] = (float(v) for v in sph[k, :3])
        arr[k].r = float(sph[k, 3])
    return arr, int(sph.shape[0])


def _phases(phases) -> ctypes.Array:
    arr = (L.HmIso * 2)()
    for p in range(2):
        arr[p].lam = float(phases[p][0])
        arr[p].mu = float(phases[p][1])
    return arr


def _stream(dev: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _opts(prec, tol, max_iter, c0_alpha, check_every, stall_window, use_graph, profile=False,
          autotune=True, schedule=None, method="fixed_point") -> L.HmSolveOpts:
    o = L.HmSolveOpts()
    o.prec = L.PRECS[prec]
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.c0_alpha = float(c0_alpha)
    o.check_every = int(check_every)
    o.stall_window = int(stall_window)
    o.use_graph = 1 if use_graph else 0
    o.profile = 1 if profile else 0
    o.autotune = 1 if (autotune and schedule is None) else 0
    o.schedule = -1 if schedule is None else int(schedule[0]) | int(schedule[1]) << 4 | int(schedule[2]) << 8
    o.method = L.METHODS[method]
    return o


def _reports(rep, k):
    return [{"iters": rep[i].iters, "status": rep[i].status, "err": rep[i].err,
             "err0": rep[i].err0, "seconds": rep[i].seconds} for i in range(k)]


def _check_field(t: torch.Tensor, N: int, dtype, dev, name: str):
    if t is None:
        return
    if t.device != dev or t.dtype != dtype or t.numel() != N or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s tensor of %d entries on %s" % (name, dtype, N, dev))


def hm_filter(n, dim, spheres, radius_vox: float, subsamples: int, rule: str, prec: str = "fp64",
              device="cuda:0"):
    """Per-voxel counts, fractions and normal-sphere ids (see hm_filter in include/hm.h)."""
    dev = _device(device)
    N = int(n[0] * n[1] * n[2])
    count = torch.empty(N, dtype=torch.int32, device=dev)
    frac = torch.empty(N, dtype=_DT[prec], device=dev)
    incl = torch.empty(N, dtype=torch.int32, device=dev)
    g = _grid(n, dim)
    sph, ns = _spheres(spheres)
    rc = _lib().hm_filter(ctypes.byref(g), sph, ns, float(radius_vox), int(subsamples), L.RULES[rule],
                          L.PRECS[prec], _ptr(count), _ptr(frac), _ptr(incl), _stream(dev))
    L.check(rc)
    return count, frac, incl


def hm_filter_noalloc(n, dim, spheres, radius_vox: float, subsamples: int, rule: str, prec: str = "fp64",
                      count=None, frac=None, incl=None, device="cuda:0"):
    """hm_filter into caller-owned outputs with no allocation inside the
    library (see hm_filter_noalloc in include/hm.h); outputs are allocated
    here only when not given."""
    dev = _device(device)
    N = int(n[0] * n[1] * n[2])
    count = torch.empty(N, dtype=torch.int32, device=dev) if count is None else count
    frac = torch.empty(N, dtype=_DT[prec], device=dev) if frac is None else frac
    incl = torch.empty(N, dtype=torch.int32, device=dev) if incl is None else incl
    _check_field(count, N, torch.int32, dev, "count")
    _check_field(frac, N, _DT[prec], dev, "frac")
    _check_field(incl, N, torch.int32, dev, "incl")
    g = _grid(n, dim)
    sph, ns = _spheres(spheres)
    rc = _lib().hm_filter_noalloc(ctypes.byref(g), sph, ns, float(radius_vox), int(subsamples), L.RULES[rule],
                                  L.PRECS[prec], _ptr(count), _ptr(frac), _ptr(incl), _stream(dev))
    L.check(rc)
    return count, frac, incl


def hm_solve(n, dim, phases, rule: str, frac: torch.Tensor, incl: Optional[torch.Tensor], spheres, E,
             prec: str = "fp64", tol: float = 1e-4, max_iter: int = 10000, c0_alpha: float = 1.0,
             check_every: int = 1, stall_window: int = 0, use_graph: bool = False, want_eps: bool = False,
             profile: bool = False, autotune: bool = True, method: str = "fixed_point", schedule=None):
    """Solve for the rows of E (n_load x 6 tensor components); method "fixed_point" or "cg";
    schedule = (x, y, z) variant indices pins the tile schedules (no autotuning)."""
    dev = frac.device
    N = int(n[0] * n[1] * n[2])
    _check_field(frac, N, _DT[prec], dev, "frac")
    _check_field(incl, N, torch.int32, dev, "incl")
    Ea = np.ascontiguousarray(np.asarray(E, dtype=np.float64).reshape(-1, 6))
    nl = Ea.shape[0]
    sig = np.zeros((nl, 6))
    rep = (L.HmReport * nl)()
    eps = torch.empty((nl, 6, N), dtype=_DT[prec], device=dev) if want_eps else None
    g = _grid(n, dim)
    sph, ns = _spheres(spheres)
    o = _opts(prec, tol, max_iter, c0_alpha, check_every, stall_window, use_graph, profile, autotune, schedule,
              method)
    rc = _lib().hm_solve(ctypes.byref(g), _phases(phases), L.RULES[rule], _ptr(frac), _ptr(incl), sph, ns,
                         Ea.ctypes.data_as(L._dp), nl, ctypes.byref(o), _ptr(eps),
                         sig.ctypes.data_as(L._dp), rep, _stream(dev))
    L.check(rc)
    return {"status": rc, "sig_mean": sig, "reports": _reports(rep, nl), "eps": eps}


def hm_effective_tensor(n, dim, phases, rule: str, frac: torch.Tensor, incl: Optional[torch.Tensor], spheres,
                        prec: str = "fp64", tol: float = 1e-4, max_iter: int = 10000, c0_alpha: float = 1.0,
                        check_every: int = 1, stall_window: int = 0, use_graph: bool = False,
                        want_eps: bool = False, profile: bool = False, autotune: bool = True,
                        schedule=None, method: str = "fixed_point"):
    """Effective Mandel tensor from the unit-strain solves (6 in 3D, 3 in 2D)."""
    dev = frac.device
    N = int(n[0] * n[1] * n[2])
    _check_field(frac, N, _DT[prec], dev, "frac")
    _check_field(incl, N, torch.int32, dev, "incl")
    k = 3 if dim == 2 else 6
    C = np.zeros((k, k))
    rep = (L.HmReport * k)()
    eps = torch.empty((k, 6, N), dtype=_DT[prec], device=dev) if want_eps else None
    g = _grid(n, dim)
    sph, ns = _spheres(spheres)
    o = _opts(prec, tol, max_iter, c0_alpha, check_every, stall_window, use_graph, profile, autotune, schedule,
              method)
    rc = _lib().hm_effective_tensor(ctypes.byref(g), _phases(phases), L.RULES[rule], _ptr(frac), _ptr(incl),
                                    sph, ns, ctypes.byref(o), C.ctypes.data_as(L._dp), _ptr(eps), rep,
                                    _stream(dev))
    L.check(rc)
    return {"status": rc, "C": C, "reports": _reports(rep, k), "eps": eps}


def _conductivities(k) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(k, dtype=np.float64).reshape(2))
    return a


def hm_conduct_solve(n, dim, k, rule: str, frac: torch.Tensor, incl: Optional[torch.Tensor], spheres, G,
                     prec: str = "fp64", tol: float = 1e-4, max_iter: int = 10000, c0_alpha: float = 1.0,
                     check_every: int = 1, stall_window: int = 0, use_graph: bool = False,
                     want_grad: bool = False, profile: bool = False):
    """Conduction solve for the rows of G (n_load x 3 mean-gradient components); k = (matrix, inclusion)."""
    dev = frac.device
    N = int(n[0] * n[1] * n[2])
    _check_field(frac, N, _DT[prec], dev, "frac")
    _check_field(incl, N, torch.int32, dev, "incl")
    Ga = np.ascontiguousarray(np.asarray(G, dtype=np.float64).reshape(-1, 3))
    nl = Ga.shape[0]
    q = np.zeros((nl, 3))
    rep = (L.HmReport * nl)()
    grad = torch.empty((nl, 3, N), dtype=_DT[prec], device=dev) if want_grad else None
    g = _grid(n, dim)
    sph, ns = _spheres(spheres)
    kk = _conductivities(k)
    o = _opts(prec, tol, max_iter, c0_alpha, check_every, stall_window, use_graph, profile, False, None)
    rc = _lib().hm_conduct_solve(ctypes.byref(g), kk.ctypes.data_as(L._dp), L.RULES[rule], _ptr(frac), _ptr(incl),
                                 sph, ns, Ga.ctypes.data_as(L._dp), nl, ctypes.byref(o), _ptr(grad),
                                 q.ctypes.data_as(L._dp), rep, _stream(dev))
    L.check(rc)
    return {"status": rc, "flux_mean": q, "reports": _reports(rep, nl), "grad": grad}


def hm_effective_conductivity(n, dim, k, rule: str, frac: torch.Tensor, incl: Optional[torch.Tensor], spheres,
                              prec: str = "fp64", tol: float = 1e-4, max_iter: int = 10000, c0_alpha: float = 1.0,
                              check_every: int = 1, stall_window: int = 0, use_graph: bool = False,
                              want_grad: bool = False, profile: bool = False):
    """Effective conductivity tensor (dim x dim) from the unit-gradient solves."""
    dev = frac.device
    N = int(n[0] * n[1] * n[2])
    _check_field(frac, N, _DT[prec], dev, "frac")
    _check_field(incl, N, torch.int32, dev, "incl")
    nd = 2 if dim == 2 else 3
    K = np.zeros((nd, nd))
    rep = (L.HmReport * nd)()
    grad = torch.empty((nd, 3, N), dtype=_DT[prec], device=dev) if want_grad else None
    g = _grid(n, dim)
    sph, ns = _spheres(spheres)
    kk = _conductivities(k)
    o = _opts(prec, tol, max_iter, c0_alpha, check_every, stall_window, use_graph, profile, False, None)
    rc = _lib().hm_effective_conductivity(ctypes.byref(g), kk.ctypes.data_as(L._dp), L.RULES[rule], _ptr(frac),
                                          _ptr(incl), sph, ns, ctypes.byref(o), K.ctypes.data_as(L._dp),
                                          _ptr(grad), rep, _stream(dev))
    L.check(rc)
    return {"status": rc, "K": K, "reports": _reports(rep, nd), "grad": grad}


def _phase_array(phases) -> ctypes.Array:
    arr = (L.HmIso * len(phases))()
    for p, ph in enumerate(phases):
        arr[p].lam = float(ph[0])
        arr[p].mu = float(ph[1])
    return arr


def hm_filter_phases(n, dim, spheres, labels, n_phases: int, radius_vox: float, subsamples: int, rule: str,
                     prec: str = "fp64", device="cuda:0"):
    """Per-phase counts and fractions, each (n_phases - 1, N)."""
    dev = _device(device)
    N = int(n[0] * n[1] * n[2])
    count = torch.empty((n_phases - 1, N), dtype=torch.int32, device=dev)
    frac = torch.empty((n_phases - 1, N), dtype=_DT[prec], device=dev)
    g = _grid(n, dim)
    sph, ns = _spheres(spheres)
    lab = (ctypes.c_int * max(1, ns))(*(int(v) for v in np.asarray(labels).reshape(-1)))
    rc = _lib().hm_filter_phases(ctypes.byref(g), sph, lab, ns, int(n_phases), float(radius_vox), int(subsamples),
                                 L.RULES[rule], L.PRECS[prec], _ptr(count), _ptr(frac), _stream(dev))
    L.check(rc)
    return count, frac


def hm_solve_phases(n, dim, phases, rule: str, frac: torch.Tensor, E, prec: str = "fp64", tol: float = 1e-4,
                    max_iter: int = 10000, c0_alpha: float = 1.0, check_every: int = 1, stall_window: int = 0,
                    use_graph: bool = False, want_eps: bool = False, method: str = "fixed_point",
                    autotune: bool = True):
    """hm_solve for a cell of len(phases) phases; frac is (len(phases) - 1, N)."""
    dev = frac.device
    N = int(n[0] * n[1] * n[2])
    _check_field(frac, N * (len(phases) - 1), _DT[prec], dev, "frac")
    Ea = np.ascontiguousarray(np.asarray(E, dtype=np.float64).reshape(-1, 6))
    nl = Ea.shape[0]
    sig = np.zeros((nl, 6))
    rep = (L.HmReport * nl)()
    eps = torch.empty((nl, 6, N), dtype=_DT[prec], device=dev) if want_eps else None
    g = _grid(n, dim)
    o = _opts(prec, tol, max_iter, c0_alpha, check_every, stall_window, use_graph, False, autotune, None, method)
    rc = _lib().hm_solve_phases(ctypes.byref(g), _phase_array(phases), len(phases), L.RULES[rule], _ptr(frac),
                                Ea.ctypes.data_as(L._dp), nl, ctypes.byref(o), _ptr(eps),
                                sig.ctypes.data_as(L._dp), rep, _stream(dev))
    L.check(rc)
    return {"status": rc, "sig_mean": sig, "reports": _reports(rep, nl), "eps": eps}


def hm_effective_tensor_phases(n, dim, phases, rule: str, frac: torch.Tensor, prec: str = "fp64",
                               tol: float = 1e-4, max_iter: int = 10000, c0_alpha: float = 1.0,
                               check_every: int = 1, stall_window: int = 0, use_graph: bool = False,
                               method: str = "fixed_point", profile: bool = False, autotune: bool = True):
    """Effective Mandel tensor of a cell of len(phases) phases."""
    dev = frac.device
    N = int(n[0] * n[1] * n[2])
    _check_field(frac, N * (len(phases) - 1), _DT[prec], dev, "frac")
    k = 3 if dim == 2 else 6
    C = np.zeros((k, k))
    rep = (L.HmReport * k)()
    g = _grid(n, dim)
    o = _opts(prec, tol, max_iter, c0_alpha, check_every, stall_window, use_graph, profile, autotune, None, method)
    rc = _lib().hm_effective_tensor_phases(ctypes.byref(g), _phase_array(phases), len(phases), L.RULES[rule],
                                           _ptr(frac), ctypes.byref(o), C.ctypes.data_as(L._dp), None, rep,
                                           _stream(dev))
    L.check(rc)
    return {"status": rc, "C": C, "reports": _reports(rep, k)}


def _mandel_pair(C_phases) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(C_phases, dtype=np.float64).reshape(2, 6, 6))
    return a


def hm_solve_aniso(n, dim, C_phases, rule: str, frac: torch.Tensor, incl: Optional[torch.Tensor], spheres, E,
                   prec: str = "fp64", tol: float = 1e-4, max_iter: int = 10000, c0_alpha: float = 1.0,
                   check_every: int = 1, stall_window: int = 0, use_graph: bool = False, want_eps: bool = False,
                   method: str = "fixed_point", autotune: bool = True):
    """hm_solve for two anisotropic phases given as Mandel matrices (2, 6, 6)."""
    dev = frac.device
    N = int(n[0] * n[1] * n[2])
    _check_field(frac, N, _DT[prec], dev, "frac")
    _check_field(incl, N, torch.int32, dev, "incl")
    Cp = _mandel_pair(C_phases)
    Ea = np.ascontiguousarray(np.asarray(E, dtype=np.float64).reshape(-1, 6))
    nl = Ea.shape[0]
    sig = np.zeros((nl, 6))
    rep = (L.HmReport * nl)()
    eps = torch.empty((nl, 6, N), dtype=_DT[prec], device=dev) if want_eps else None
    g = _grid(n, dim)
    sph, ns = _spheres(spheres)
    o = _opts(prec, tol, max_iter, c0_alpha, check_every, stall_window, use_graph, False, autotune, None, method)
    rc = _lib().hm_solve_aniso(ctypes.byref(g), Cp.ctypes.data_as(L._dp), L.RULES[rule], _ptr(frac), _ptr(incl),
                               sph, ns, Ea.ctypes.data_as(L._dp), nl, ctypes.byref(o), _ptr(eps),
                               sig.ctypes.data_as(L._dp), rep, _stream(dev))
    L.check(rc)
    return {"status": rc, "sig_mean": sig, "reports": _reports(rep, nl), "eps": eps}


def hm_effective_tensor_aniso(n, dim, C_phases, rule: str, frac: torch.Tensor, incl: Optional[torch.Tensor],
                              spheres, prec: str = "fp64", tol: float = 1e-4, max_iter: int = 10000,
                              c0_alpha: float = 1.0, check_every: int = 1, stall_window: int = 0,
                              use_graph: bool = False, method: str = "fixed_point", profile: bool = False,
                              autotune: bool = True):
    """Effective Mandel tensor for two anisotropic phases."""
    dev = frac.device
    N = int(n[0] * n[1] * n[2])
    _check_field(frac, N, _DT[prec], dev, "frac")
    _check_field(incl, N, torch.int32, dev, "incl")
    Cp = _mandel_pair(C_phases)
    k = 3 if dim == 2 else 6
    C = np.zeros((k, k))
    rep = (L.HmReport * k)()
    g = _grid(n, dim)
    sph, ns = _spheres(spheres)
    o = _opts(prec, tol, max_iter, c0_alpha, check_every, stall_window, use_graph, profile, autotune, None, method)
    rc = _lib().hm_effective_tensor_aniso(ctypes.byref(g), Cp.ctypes.data_as(L._dp), L.RULES[rule], _ptr(frac),
                                          _ptr(incl), sph, ns, ctypes.byref(o), C.ctypes.data_as(L._dp), None, rep,
                                          _stream(dev))
    L.check(rc)
    return {"status": rc, "C": C, "reports": _reports(rep, k)}


def hm_stress_field(n, dim, phases, rule: str, frac: torch.Tensor, incl: Optional[torch.Tensor], spheres,
                    eps: torch.Tensor, prec: str = "fp64"):
    """Local stress c~ : eps for strain fields eps (n_load, 6, N); returns the same shape."""
    dev = frac.device
    N = int(n[0] * n[1] * n[2])
    _check_field(frac, N, _DT[prec], dev, "frac")
    _check_field(incl, N, torch.int32, dev, "incl")
    nl = eps.numel() // (6 * N)
    _check_field(eps, 6 * N * nl, _DT[prec], dev, "eps")
    sig = torch.empty((nl, 6, N), dtype=_DT[prec], device=dev)
    g = _grid(n, dim)
    sph, ns = _spheres(spheres)
    rc = _lib().hm_stress_field(ctypes.byref(g), _phases(phases), L.RULES[rule], _ptr(frac), _ptr(incl), sph, ns,
                                L.PRECS[prec], _ptr(eps), nl, _ptr(sig), _stream(dev))
    L.check(rc)
    return sig


def hm_flux_field(n, dim, k, rule: str, frac: torch.Tensor, incl: Optional[torch.Tensor], spheres,
                  grad: torch.Tensor, prec: str = "fp64"):
    """Local flux k~ g for gradient fields grad (n_load, 3, N); returns the same shape."""
    dev = frac.device
    N = int(n[0] * n[1] * n[2])
    _check_field(frac, N, _DT[prec], dev, "frac")
    _check_field(incl, N, torch.int32, dev, "incl")
    nl = grad.numel() // (3 * N)
    _check_field(grad, 3 * N * nl, _DT[prec], dev, "grad")
    q = torch.empty((nl, 3, N), dtype=_DT[prec], device=dev)
    g = _grid(n, dim)
    sph, ns = _spheres(spheres)
    kk = _conductivities(k)
    rc = _lib().hm_flux_field(ctypes.byref(g), kk.ctypes.data_as(L._dp), L.RULES[rule], _ptr(frac), _ptr(incl), sph,
                              ns, L.PRECS[prec], _ptr(grad), nl, _ptr(q), _stream(dev))
    L.check(rc)
    return q


def hm_fourier_series(n, dim, field: torch.Tensor, m, prec: str = "fp64"):
    """Truncated Fourier series of a grid field on the voxel centres of an m grid, (m_z, m_y, m_x)."""
    dev = field.device
    N = int(n[0] * n[1] * n[2])
    _check_field(field, N, _DT[prec], dev, "field")
    mm = (ctypes.c_int * 3)(*(int(v) for v in m))
    out = torch.empty((int(m[2]), int(m[1]), int(m[0])), dtype=_DT[prec], device=dev)
    g = _grid(n, dim)
    rc = _lib().hm_fourier_series(ctypes.byref(g), mm, L.PRECS[prec], _ptr(field), _ptr(out), _stream(dev))
    L.check(rc)
    return out


def hm_stiffness_component(n, dim, phases, rule: str, frac: torch.Tensor, incl: Optional[torch.Tensor], spheres,
                           I: int, J: int, prec: str = "fp64"):
    """Mandel entry (I, J) of the filtered stiffness at every voxel (N reals)."""
    dev = frac.device
    N = int(n[0] * n[1] * n[2])
    _check_field(frac, N, _DT[prec], dev, "frac")
    _check_field(incl, N, torch.int32, dev, "incl")
    out = torch.empty(N, dtype=_DT[prec], device=dev)
    g = _grid(n, dim)
    sph, ns = _spheres(spheres)
    rc = _lib().hm_stiffness_component(ctypes.byref(g), _phases(phases), L.RULES[rule], _ptr(frac), _ptr(incl),
                                       sph, ns, L.PRECS[prec], int(I), int(J), _ptr(out), _stream(dev))
    L.check(rc)
    return out


def hm_effective_tensor_batch(problems, prec: str = "fp64", tol: float = 1e-4, max_iter: int = 10000,
                              c0_alpha: float = 1.0, check_every: int = 16, stall_window: int = 0,
                              use_graph: bool = True, autotune: bool = True):
    """Effective tensors of many cells (dicts with n, dim, phases, rule, frac, incl, spheres) in one batch."""
    if not problems:
        raise ValueError("no problems")
    dev = problems[0]["frac"].device
    arr = (L.HmProblem * len(problems))()
    keep = []
    ks = []
    for i, pr in enumerate(problems):
        n = pr["n"]
        N = int(n[0] * n[1] * n[2])
        _check_field(pr["frac"], N, _DT[prec], dev, "frac")
        _check_field(pr.get("incl"), N, torch.int32, dev, "incl")
        arr[i].grid = _grid(n, pr["dim"])
        ph = _phases(pr["phases"])
        arr[i].phases[0] = ph[0]
        arr[i].phases[1] = ph[1]
        arr[i].rule = L.RULES[pr["rule"]]
        arr[i].d_frac = pr["frac"].data_ptr()
        arr[i].d_incl = 0 if pr.get("incl") is None else pr["incl"].data_ptr()
        sph, ns = _spheres(pr["spheres"])
        keep.append(sph)
        arr[i].spheres = ctypes.cast(sph, ctypes.POINTER(L.HmSphere))
        arr[i].n_spheres = ns
        ks.append(3 if pr["dim"] == 2 else 6)
    C = np.zeros(sum(k * k for k in ks))
    rep = (L.HmReport * sum(ks))()
    o = _opts(prec, tol, max_iter, c0_alpha, check_every, stall_window, use_graph, False, autotune)
    rc = _lib().hm_effective_tensor_batch(arr, len(problems), ctypes.byref(o), C.ctypes.data_as(L._dp), rep,
                                          _stream(dev))
    L.check(rc)
    out = []
    co = ro = 0
    allrep = _reports(rep, sum(ks))
    for k in ks:
        out.append({"C": C[co:co + k * k].reshape(k, k).copy(), "reports": allrep[ro:ro + k]})
        co += k * k
        ro += k
    return {"status": rc, "results": out}


def hm_solve_adjoint(n, dim, phases, rule: str, frac: torch.Tensor, incl: Optional[torch.Tensor], spheres,
                     dLdC, eps: torch.Tensor, prec: str = "fp64", want_dfrac: bool = True):
    """dL/d(lambda_0, mu_0, lambda_1, mu_1) and dL/dfrac from the unit-strain fields."""
    dev = frac.device
    N = int(n[0] * n[1] * n[2])
    k = 3 if dim == 2 else 6
    _check_field(frac, N, _DT[prec], dev, "frac")
    _check_field(incl, N, torch.int32, dev, "incl")
    if eps.device != dev or eps.dtype != _DT[prec] or eps.numel() != k * 6 * N or not eps.is_contiguous():
        raise ValueError("eps must hold the %d unit-strain fields (%d x 6 x %d)" % (k, k, N))
    G = np.ascontiguousarray(np.asarray(dLdC, dtype=np.float64).reshape(k, k))
    dph = np.zeros(4)
    dfr = torch.empty(N, dtype=_DT[prec], device=dev) if want_dfrac else None
    g = _grid(n, dim)
    sph, ns = _spheres(spheres)
    rc = _lib().hm_solve_adjoint(ctypes.byref(g), _phases(phases), L.RULES[rule], _ptr(frac), _ptr(incl), sph,
                                 ns, L.PRECS[prec], G.ctypes.data_as(L._dp), _ptr(eps), k,
                                 dph.ctypes.data_as(L._dp), _ptr(dfr), _stream(dev))
    L.check(rc)
    return dph, dfr


def last_timing():
    """Per-kernel average milliseconds of this thread's last profiled solve."""
    t = L.HmTiming()
    L.check(_lib().hm_last_timing(ctypes.byref(t)))
    names = ("xsweep", "ysweep_fwd", "zsweep", "ysweep_inv", "finalize")
    return {"iterations": t.iterations, "n_load": t.n_load, "active_loads": t.active_loads,
            "ms": {n: t.ms[i] for i, n in enumerate(names)},
            "schedule": {"x_lines": t.x_lines, "y_width": t.y_width, "z_width": t.z_width,
                         "z_threads": t.z_threads, "z_groups": t.z_groups},
            "kernels": {n: t.kernel[i].value.decode() for i, n in enumerate(names)}}


def last_history(n_load: int, cap: int):
    """Errors (n_load x cap) and mean stresses (n_load x cap x 6) of every
    iterate of this thread's last single-cell solve; NaN past each load
    case's reported iterate."""
    err = np.zeros((n_load, cap))
    sig = np.zeros((n_load, cap, 6))
    L.check(_lib().hm_last_history(int(n_load), int(cap), err.ctypes.data_as(L._dp), sig.ctypes.data_as(L._dp)))
    return err, sig


def schedule_count(n, dim, prec="fp64"):
    """Numbers of compiled schedule variants of the x, y and z sweeps."""
    g = _grid(n, dim)
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    L.check(_lib().hm_schedule_count(ctypes.byref(g), L.PRECS[prec], ctypes.byref(a), ctypes.byref(b),
                                     ctypes.byref(c)))
    return a.value, b.value, c.value


class HmSolveError(RuntimeError):
    """A solve whose stop status makes a derived quantity invalid."""


def release_plans():
    _lib().hm_release_plans()


def device_ok() -> bool:
    return bool(_lib().hm_device_ok())


class EffectiveTensor(torch.autograd.Function):
    """C_eff(lame, frac) with a backward pass through hm_solve_adjoint.

    forward(lame, frac, cell) where lame = (lambda_0, mu_0, lambda_1, mu_1)
    (CPU float64 tensor), frac the per-voxel fraction field (device tensor
    of the solve precision) and cell a dict with keys n, dim, rule, incl,
    spheres, prec, tol, max_iter and optionally checkpoint.  The unit-strain
    fields are kept for the backward pass unless cell["checkpoint"] is
    true, in which case they are recomputed there (less memory, one more
    batched solve).

    The gradient uses the variational (Hill) identity, which holds at the
    discrete equilibrium only, so the solve's stop matters: a load case that
    diverged or hit max_iter raises HmSolveError; a stalled one (the mixed
    path's stop at its single-precision floor, with cell["stall_window"])
    gives a gradient accurate to that floor and emits a warning.  The final
    equilibrium errors and statuses of the forward solve are written to
    cell["reports"] so callers can bound the gradient error.
    """

    @staticmethod
    def _solve(cell, ph, frac, want_eps):
        out = hm_effective_tensor(cell["n"], cell["dim"], ph, cell["rule"], frac.detach(), cell.get("incl"),
                                  cell["spheres"], prec=cell.get("prec", "fp64"), tol=cell.get("tol", 1e-4),
                                  max_iter=cell.get("max_iter", 10000), check_every=cell.get("check_every", 8),
                                  stall_window=cell.get("stall_window", 0), want_eps=want_eps)
        cell["reports"] = out["reports"]
        bad = [r for r in out["reports"] if r["status"] in (1, 3)]
        if bad:
            raise HmSolveError("the effective-tensor solve did not converge (statuses %s, errors %s): its "
                               "gradient would not satisfy the equilibrium the adjoint identity needs"
                               % ([r["status"] for r in out["reports"]], [r["err"] for r in out["reports"]]))
        if any(r["status"] == 2 for r in out["reports"]):
            warnings.warn("effective-tensor solve stalled at equilibrium errors %s: the gradient is accurate to "
                          "that floor only" % ["%.2e" % r["err"] for r in out["reports"]], RuntimeWarning)
        return out

    @staticmethod
    def forward(ctx, lame, frac, cell):
        ph = ((float(lame[0]), float(lame[1])), (float(lame[2]), float(lame[3])))
        keep = not cell.get("checkpoint", False)
        out = EffectiveTensor._solve(cell, ph, frac, keep)
        ctx.cell = cell
        ctx.ph = ph
        ctx.eps = out["eps"]
        ctx.save_for_backward(frac)
        ctx.reports = out["reports"]
        return torch.from_numpy(out["C"].copy())

    @staticmethod
    def backward(ctx, gC):
        (frac,) = ctx.saved_tensors
        cell = ctx.cell
        eps = ctx.eps
        if eps is None:
            eps = EffectiveTensor._solve(cell, ctx.ph, frac, True)["eps"]
        dph, dfr = hm_solve_adjoint(cell["n"], cell["dim"], ctx.ph, cell["rule"], frac.detach(), cell.get("incl"),
                                    cell["spheres"], gC.detach().cpu().numpy(), eps,
                                    prec=cell.get("prec", "fp64"))
        ctx.eps = None
        return torch.from_numpy(dph), dfr, None
