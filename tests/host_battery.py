"""Argument checks of the C ABI that run on the host before any device call.

Each case calls one entry point with one bad argument and expects its error
code and a word of its message.  The cases whose arguments are all valid
reach the first device call; with no usable GPU they must fail there with
HM_E_DEVICE or HM_E_NOMEM (never a crash).  Stand-in device pointers are
never dereferenced on the host, and the battery refuses to run where a GPU
is usable, so that no kernel is ever launched on them.

Used in-process by tests/test_host_logic.py and, under AddressSanitizer and
UndefinedBehaviorSanitizer, by tests/test_host_sanitized.py (run as a script:
``python host_battery.py LIB_PATH``).
"""
from __future__ import annotations

import ctypes
import importlib.util
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def load_decls():
    """The ctypes declarations module, loaded without importing the package
    (whose __init__ pulls in torch)."""
    path = os.path.join(ROOT, "paper_1412_3228_amd", "_lib.py")
    spec = importlib.util.spec_from_file_location("hm_lib_decls", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _cases(L, lib):
    FAKE = ctypes.c_void_p(0x10000)   # stand-in device pointer (never dereferenced on the host)
    FAKE_I = ctypes.c_void_p(0x20000)
    NONE = None
    DEV = (L.HM_E_DEVICE, L.HM_E_NOMEM)

    def grid(n=(15, 15, 15), dim=3):
        g = L.HmGrid()
        g.dim = dim
        for i in range(3):
            g.n[i] = n[i]
        return ctypes.byref(g)

    def spheres(rows):
        arr = (L.HmSphere * max(1, len(rows)))()
        for k, (x, y, z, r) in enumerate(rows):
            arr[k].c[0], arr[k].c[1], arr[k].c[2], arr[k].r = x, y, z, r
        return arr

    def iso(p0=(1.0, 1.0), p1=(10.0, 10.0)):
        a = (L.HmIso * 2)()
        a[0].lam, a[0].mu = p0
        a[1].lam, a[1].mu = p1
        return a

    def opts(**kw):
        o = L.HmSolveOpts()
        o.prec, o.tol, o.max_iter, o.c0_alpha, o.check_every = 0, 1e-4, 100, 1.0, 1
        o.stall_window, o.use_graph, o.profile, o.autotune, o.schedule, o.method = 0, 0, 0, 1, -1, 0
        for k, v in kw.items():
            setattr(o, k, v)
        return ctypes.byref(o)

    def dbl(vals):
        return (ctypes.c_double * len(vals))(*vals)

    sph1 = spheres([(7.0, 7.0, 7.0, 3.0)])
    E6 = dbl([1, 0, 0, 0, 0, 0])
    sig = dbl([0] * 6 * 8)
    C36 = dbl([0] * 36)
    eye = [1.0 if i % 7 == 0 else 0.0 for i in range(36)]
    cm_ok = dbl(eye + [2 * v for v in eye])
    cm_bad = dbl(eye + [-v for v in eye])
    i3 = (ctypes.c_int * 3)
    out3 = [ctypes.c_int(0) for _ in range(3)]

    def filt(g=None, sph=sph1, ns=1, r=1.0, S=8, rule=3, prec=0, cnt=FAKE, frac=FAKE, incl=FAKE_I):
        return lambda: lib.hm_filter(g if g is not None else grid(), sph, ns, r, S, rule, prec, cnt, frac, incl,
                                     NONE)

    def solve(g=None, ph=None, rule=3, frac=FAKE, incl=FAKE_I, sph=sph1, ns=1, E=E6, nl=1, o=None):
        return lambda: lib.hm_solve(g if g is not None else grid(), ph if ph is not None else iso(), rule, frac, incl,
                                    sph, ns, E, nl, o if o is not None else opts(), NONE, sig, NONE, NONE)

    big = spheres([(0.5 + (k % 15), 0.5 + (k // 15) % 15, 0.5 + (k // 225) % 15, 0.4) for k in range(5000)])
    two = spheres([(5.0, 5.0, 5.0, 2.0), (8.0, 5.0, 5.0, 2.0)])
    lab_mixed = (ctypes.c_int * 2)(1, 2)
    lab_bad = (ctypes.c_int * 2)(1, 3)

    c = []
    # grids
    c += [("grid NULL", lambda: lib.hm_filter(None, sph1, 1, 1.0, 8, 3, 0, FAKE, FAKE, FAKE_I, NONE),
           (L.HM_E_ARG,), "NULL"),
          ("dim 4", filt(g=grid(dim=4)), (L.HM_E_ARG,), "dim"),
          ("n not positive", filt(g=grid((15, -3, 15))), (L.HM_E_ARG,), "positive"),
          ("even length", filt(g=grid((16, 15, 15))), (L.HM_E_SIZE,), "odd"),
          ("prime 17", filt(g=grid((17, 15, 15))), (L.HM_E_SIZE,), "no compiled transform"),
          ("length 245", filt(g=grid((15, 15, 245))), (L.HM_E_SIZE,), "no compiled transform"),
          ("2D with depth", filt(g=grid((15, 15, 3), dim=2)), (L.HM_E_ARG,), "n[2] == 1"),
          ("3D too thin", filt(g=grid((15, 1, 15))), (L.HM_E_SIZE,), "at least 3")]
    # spheres and filter settings
    c += [("n_spheres < 0", filt(ns=-1), (L.HM_E_ARG,), "n_spheres"),
          ("spheres NULL", filt(sph=None, ns=2), (L.HM_E_ARG,), "NULL"),
          ("radius 0", filt(sph=spheres([(7, 7, 7, 0.0)])), (L.HM_E_ARG,), "radius"),
          ("radius NaN", filt(sph=spheres([(7, 7, 7, math.nan)])), (L.HM_E_ARG,), "radius"),
          ("centre outside", filt(sph=spheres([(15.0, 7, 7, 2.0)])), (L.HM_E_ARG,), "outside"),
          ("unknown rule", filt(rule=9), (L.HM_E_ARG,), "rule"),
          ("unknown precision", filt(prec=4), (L.HM_E_ARG,), "precision"),
          ("odd subsamples", filt(S=7), (L.HM_E_ARG,), "even"),
          ("subsamples 34", filt(S=34), (L.HM_E_ARG,), "even"),
          ("filter radius 0", filt(r=0.0), (L.HM_E_ARG,), "radius_vox"),
          ("filter radius too wide", filt(r=9.0), (L.HM_E_ARG,), "radius_vox"),
          ("count NULL", filt(cnt=None), (L.HM_E_ARG,), "NULL"),
          ("noalloc over capacity",
           lambda: lib.hm_filter_noalloc(grid(), big, L.HM_FILTER_NOALLOC_MAX_SPHERES + 1, 1.0, 8, 3, 0, FAKE, FAKE,
                                         FAKE_I, NONE), (L.HM_E_SIZE,), "at most"),
          ("phases filter n_phases 1",
           lambda: lib.hm_filter_phases(grid(), two, lab_mixed, 2, 1, 1.0, 8, 1, 0, FAKE, FAKE, NONE),
           (L.HM_E_ARG,), "n_phases"),
          ("phases filter labels NULL",
           lambda: lib.hm_filter_phases(grid(), two, None, 2, 3, 1.0, 8, 1, 0, FAKE, FAKE, NONE),
           (L.HM_E_ARG,), "labels"),
          ("phases filter label range",
           lambda: lib.hm_filter_phases(grid(), two, lab_bad, 2, 3, 1.0, 8, 1, 0, FAKE, FAKE, NONE),
           (L.HM_E_ARG,), "label"),
          ("phases filter overlap",
           lambda: lib.hm_filter_phases(grid(), two, lab_mixed, 2, 3, 1.0, 8, 1, 0, FAKE, FAKE, NONE),
           (L.HM_E_ARG,), "overlap")]
    # valid filters: the host tables are built, then the device call fails
    c += [("filter valid", filt(), DEV, None),
          ("filter 5000 spheres", filt(sph=big, ns=5000, r=0.5), DEV, None),
          ("filter point rule", filt(rule=0), DEV, None)]
    # solver options, phases and problems
    c += [("opts NULL", solve(o=ctypes.POINTER(L.HmSolveOpts)()), (L.HM_E_ARG,), "opts"),
          ("opts precision", solve(o=opts(prec=3)), (L.HM_E_ARG,), "precision"),
          ("tol negative", solve(o=opts(tol=-1.0)), (L.HM_E_ARG,), "tol"),
          ("tol NaN", solve(o=opts(tol=math.nan)), (L.HM_E_ARG,), "tol"),
          ("max_iter negative", solve(o=opts(max_iter=-1)), (L.HM_E_ARG,), "max_iter"),
          ("c0_alpha 0", solve(o=opts(c0_alpha=0.0)), (L.HM_E_ARG,), "c0_alpha"),
          ("check_every 0", solve(o=opts(check_every=0)), (L.HM_E_ARG,), "check_every"),
          ("stall_window negative", solve(o=opts(stall_window=-2)), (L.HM_E_ARG,), "stall_window"),
          ("unknown method", solve(o=opts(method=7)), (L.HM_E_ARG,), "method"),
          ("CG profiled", solve(o=opts(method=1, profile=1)), (L.HM_E_ARG,), "profiling"),
          ("mu 0", solve(ph=iso(p1=(1.0, 0.0))), (L.HM_E_ARG,), "mu > 0"),
          ("3 lambda + 2 mu <= 0", solve(ph=iso(p0=(-1.0, 1.0))), (L.HM_E_ARG,), "lambda"),
          ("phases NULL", solve(ph=ctypes.POINTER(L.HmIso)()), (L.HM_E_ARG,), "phases"),
          ("frac NULL", solve(frac=None), (L.HM_E_ARG,), "d_frac"),
          ("laminate without incl", solve(incl=None), (L.HM_E_ARG,), "d_incl"),
          ("solve unknown rule", solve(rule=5), (L.HM_E_ARG,), "rule"),
          ("n_load 0", solve(nl=0), (L.HM_E_ARG,), "n_load"),
          ("n_load 5000", solve(nl=5000), (L.HM_E_ARG,), "n_load"),
          ("E NaN", solve(E=dbl([1, 0, math.nan, 0, 0, 0])), (L.HM_E_ARG,), "non-finite"),
          ("E NULL", solve(E=ctypes.POINTER(ctypes.c_double)()), (L.HM_E_ARG,), "NULL"),
          ("solve valid", solve(), DEV, None),
          ("solve valid 8 loads", solve(E=dbl([1, 0, 0, 0, 0, 0] * 8), nl=8), DEV, None),
          ("effective tensor valid",
           lambda: lib.hm_effective_tensor(grid(), iso(), 1, FAKE, NONE, sph1, 1, opts(), C36, NONE, NONE, NONE),
           DEV, None),
          ("effective tensor C NULL",
           lambda: lib.hm_effective_tensor(grid(), iso(), 1, FAKE, NONE, sph1, 1, opts(), None, NONE, NONE, NONE),
           (L.HM_E_ARG,), "C_mandel")]
    # multi-phase and anisotropic cells
    ph3 = (L.HmIso * 3)()
    for p, (lam, mu) in enumerate([(1.0, 1.0), (5.0, 5.0), (20.0, 20.0)]):
        ph3[p].lam, ph3[p].mu = lam, mu
    c += [("n_phases 9",
           lambda: lib.hm_effective_tensor_phases(grid(), ph3, 9, 1, FAKE, opts(), C36, NONE, NONE, NONE),
           (L.HM_E_ARG,), "n_phases"),
          ("2-layer with 3 phases",
           lambda: lib.hm_effective_tensor_phases(grid(), ph3, 3, 3, FAKE, opts(), C36, NONE, NONE, NONE),
           (L.HM_E_ARG,), "two phases"),
          ("phases solve valid",
           lambda: lib.hm_solve_phases(grid(), ph3, 3, 1, FAKE, E6, 1, opts(), NONE, sig, NONE, NONE), DEV, None),
          ("aniso not SPD",
           lambda: lib.hm_effective_tensor_aniso(grid(), cm_bad, 3, FAKE, FAKE_I, sph1, 1, opts(), C36, NONE, NONE,
                                                 NONE), (L.HM_E_ARG,), "positive definite"),
          ("aniso NULL",
           lambda: lib.hm_solve_aniso(grid(), None, 3, FAKE, FAKE_I, sph1, 1, E6, 1, opts(), NONE, sig, NONE, NONE),
           (L.HM_E_ARG,), "C_phases"),
          ("aniso valid",
           lambda: lib.hm_effective_tensor_aniso(grid(), cm_ok, 3, FAKE, FAKE_I, sph1, 1, opts(), C36, NONE, NONE,
                                                 NONE), DEV, None)]
    # conduction
    k_ok, k_bad = dbl([1.0, 10.0]), dbl([1.0, -2.0])
    G3 = dbl([1.0, 0.0, 0.0])
    flux = dbl([0] * 3)
    K9 = dbl([0] * 9)
    c += [("conductivity negative",
           lambda: lib.hm_conduct_solve(grid(), k_bad, 1, FAKE, NONE, sph1, 1, G3, 1, opts(), NONE, flux, NONE,
                                        NONE), (L.HM_E_ARG,), "conductivity"),
          ("conduction CG",
           lambda: lib.hm_conduct_solve(grid(), k_ok, 1, FAKE, NONE, sph1, 1, G3, 1, opts(method=1), NONE, flux,
                                        NONE, NONE), (L.HM_E_ARG,), "fixed-point"),
          ("conduction G NaN",
           lambda: lib.hm_conduct_solve(grid(), k_ok, 1, FAKE, NONE, sph1, 1, dbl([math.inf, 0, 0]), 1, opts(),
                                        NONE, flux, NONE, NONE), (L.HM_E_ARG,), "non-finite"),
          ("conductivity valid",
           lambda: lib.hm_effective_conductivity(grid(), k_ok, 3, FAKE, FAKE_I, sph1, 1, opts(), K9, NONE, NONE,
                                                 NONE), DEV, None)]
    # batches
    P = (L.HmProblem * 3)()
    for q in range(3):
        P[q].grid.dim = 3
        for i in range(3):
            P[q].grid.n[i] = (15, 21, 15)[q] if i == 0 else 15
        P[q].phases[0].lam, P[q].phases[0].mu = 1.0, 1.0
        P[q].phases[1].lam, P[q].phases[1].mu = 10.0, 10.0
        P[q].rule = 1
        P[q].d_frac = FAKE
        P[q].d_incl = None
        P[q].spheres = ctypes.cast(sph1, ctypes.POINTER(L.HmSphere))
        P[q].n_spheres = 1
    Cb = dbl([0] * 36 * 3)
    Pbad = (L.HmProblem * 3)()
    ctypes.memmove(Pbad, P, ctypes.sizeof(P))
    Pbad[2].phases[1].mu = -1.0
    c += [("batch NULL", lambda: lib.hm_effective_tensor_batch(None, 3, opts(), Cb, NONE, NONE), (L.HM_E_ARG,),
           "no problems"),
          ("batch profiled", lambda: lib.hm_effective_tensor_batch(P, 3, opts(profile=1), Cb, NONE, NONE),
           (L.HM_E_ARG,), "profiling"),
          ("batch bad problem", lambda: lib.hm_effective_tensor_batch(Pbad, 3, opts(), Cb, NONE, NONE),
           (L.HM_E_ARG,), "problem 2"),
          ("batch valid", lambda: lib.hm_effective_tensor_batch(P, 3, opts(), Cb, NONE, NONE), DEV, None)]
    # series, voxel fields, adjoint
    dLdC = dbl([0.0] * 36)
    dph = dbl([0.0] * 4)
    c += [("series m 0", lambda: lib.hm_fourier_series(grid(), i3(45, 0, 45), 0, FAKE, FAKE, NONE), (L.HM_E_SIZE,),
           "m[1]"),
          ("series even n", lambda: lib.hm_fourier_series(grid((14, 15, 15)), i3(45, 45, 45), 0, FAKE, FAKE, NONE),
           (L.HM_E_SIZE,), "odd"),
          ("series too large",
           lambda: lib.hm_fourier_series(grid(), i3(4096, 4096, 4096), 0, FAKE, FAKE, NONE), (L.HM_E_SIZE,),
           "too large"),
          ("series valid", lambda: lib.hm_fourier_series(grid(), i3(45, 45, 45), 0, FAKE, FAKE, NONE), DEV, None),
          ("stiffness index", lambda: lib.hm_stiffness_component(grid(), iso(), 1, FAKE, NONE, sph1, 1, 0, 6, 0,
                                                                  FAKE, NONE), (L.HM_E_ARG,), "Mandel"),
          ("stress eps NULL", lambda: lib.hm_stress_field(grid(), iso(), 1, FAKE, NONE, sph1, 1, 0, None, 6, FAKE,
                                                          NONE), (L.HM_E_ARG,), "d_eps"),
          ("flux n_load 0", lambda: lib.hm_flux_field(grid(), k_ok, 1, FAKE, NONE, sph1, 1, 0, FAKE, 0, FAKE, NONE),
           (L.HM_E_ARG,), "n_load"),
          ("stiffness valid", lambda: lib.hm_stiffness_component(grid(), iso(), 1, FAKE, NONE, sph1, 1, 0, 0, 0,
                                                                  FAKE, NONE), DEV, None),
          ("adjoint n_load", lambda: lib.hm_solve_adjoint(grid(), iso(), 1, FAKE, NONE, sph1, 1, 0, dLdC, FAKE, 5,
                                                          dph, FAKE, NONE), (L.HM_E_ARG,), "n_load"),
          ("adjoint dLdC NaN",
           lambda: lib.hm_solve_adjoint(grid(), iso(), 1, FAKE, NONE, sph1, 1, 0, dbl([math.nan] * 36), FAKE, 6, dph,
                                        FAKE, NONE), (L.HM_E_ARG,), "non-finite"),
          ("adjoint valid", lambda: lib.hm_solve_adjoint(grid(), iso(), 1, FAKE, NONE, sph1, 1, 0, dLdC, FAKE, 6, dph,
                                                         FAKE, NONE), DEV, None)]
    # queries
    tim = L.HmTiming()
    err = dbl([0.0] * 4)
    c += [("schedule count", lambda: lib.hm_schedule_count(grid((125, 125, 125)), 1, *[ctypes.byref(v) for v in out3]),
           (L.HM_OK,), None),
          ("schedule count NULL", lambda: lib.hm_schedule_count(grid(), 0, None, None, None), (L.HM_E_ARG,), "NULL"),
          ("timing NULL", lambda: lib.hm_last_timing(None), (L.HM_E_ARG,), "NULL"),
          ("timing before any solve", lambda: lib.hm_last_timing(ctypes.byref(tim)), (L.HM_E_ARG,), "profiled"),
          ("history before any solve", lambda: lib.hm_last_history(1, 4, err, None), (L.HM_E_ARG,), "solve")]
    return c, out3


def run(lib_path=None):
    """Runs every case; returns (number of cases, list of failures)."""
    L = load_decls()
    lib = L.load(lib_path or L.LIB_PATH)
    if lib.hm_device_ok():
        raise RuntimeError("a usable GPU is present: the battery's stand-in device pointers must not reach it")
    cases, out3 = _cases(L, lib)
    bad = []
    for name, fn, codes, word in cases:
        rc = fn()
        msg = lib.hm_last_error().decode()
        if rc not in codes:
            bad.append("%s: rc %d not in %s (%s)" % (name, rc, codes, msg))
        elif word is not None and word not in msg:
            bad.append("%s: message %r lacks %r" % (name, msg, word))
    if min(v.value for v in out3) < 1:
        bad.append("schedule count: %s" % [v.value for v in out3])
    lib.hm_release_plans()
    return len(cases), bad


if __name__ == "__main__":
    n, bad = run(sys.argv[1] if len(sys.argv) > 1 else None)
    for b in bad:
        print("FAIL", b)
    print("host battery: %d cases, %d failures" % (n, len(bad)), flush=True)
    sys.exit(1 if bad else 0)
