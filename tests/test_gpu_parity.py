"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances: filter counts and fractions bit-exact (integer counts, one IEEE
division); FP64 solve outputs within 1e-10 relative (max-norm over the
compared array); mixed-precision effective tensors within 1e-5.  Solves are
compared at equal iteration counts (tol = 0, fixed max_iter) unless stated.
"""
import math

import numpy as np
import pytest
import torch

from gpu_helpers import log, oracle_fields_to_comps, oracle_solve, rel
from oracle import filter as ofilter, gradient as ogradient, solver as osolver
from workloads import fig1_disk_case, lame, random_fraction_case, rsa_spheres, small_sphere_case, workload_c1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    import paper_1412_3228_amd as hm_mod
    assert torch.cuda.is_available(), "GPU tests need a device"
    assert hm_mod.device_ok(), "device is not gfx950"
    return hm_mod


DEV = "cuda:0"


def _gpu_filter(hm, w, prec="fp64"):
    c, f, i = hm.hm_filter(w.n, w.dim, w.spheres, w.radius_vox, w.subsamples, w.rule, prec, DEV)
    return c.cpu().numpy(), f.cpu().numpy(), i.cpu().numpy(), f, i


def _multi_sphere_case(n=45, k=6, seed=11, rule="laminate", radius=1.0, S=8):
    rng = np.random.Generator(np.random.PCG64(seed))
    r = (3 * 0.25 * n ** 3 / (4 * math.pi * k)) ** (1 / 3)
    sph = rsa_spheres(rng, (n, n, n), [r] * k, gap=1.0)
    w = small_sphere_case(n=(n, n, n), rule=rule, radius_vox=radius, subsamples=S)
    return w.with_(spheres=sph, name="multi-%d" % n)


@pytest.mark.parametrize("case", ["3d-r1-S4", "3d-r0.55-S8-shift", "2d-c1-r1-S16", "2d-c1-none", "multi-45",
                                  "3d-wide-sphere", "3d-crowded"])
def test_filter_bit_exact(hm, case):
    log("filter case %s" % case)
    if case == "3d-r1-S4":
        w = small_sphere_case(n=(15, 15, 15), radius_vox=1.0, subsamples=4)
    elif case == "3d-r0.55-S8-shift":
        w = small_sphere_case(n=(21, 15, 9), fraction=0.1, radius_vox=0.55, subsamples=8,
                              offset=(0.3125, -0.25, 0.125))
    elif case == "2d-c1-r1-S16":
        w = workload_c1("laminate")
    elif case == "2d-c1-none":
        w = workload_c1("none")
    elif case == "3d-wide-sphere":
        # the filter ball of surface voxels straddles half a period from the
        # centre: stencil points take other periodic images
        w = small_sphere_case(n=(9, 15, 9), radius_vox=1.0, subsamples=4, offset=(0.2, -0.1, 0.3))
        w = w.with_(spheres=np.array([[4.7, 7.4, 4.8, 4.3]]))
    elif case == "3d-crowded":
        # more spheres near a voxel than the candidate list holds
        rng = np.random.Generator(np.random.PCG64(5))
        c = 3.0 + rng.random((14, 3)) * 3.0
        sph = np.concatenate([c, 0.45 + 0.3 * rng.random((14, 1))], axis=1)
        w = small_sphere_case(n=(9, 9, 9), radius_vox=2.5, subsamples=4).with_(spheres=sph)
    else:
        w = _multi_sphere_case()
    cnt, frac, incl, _, _ = _gpu_filter(hm, w)
    ref = ofilter.filter_field(w)
    assert np.array_equal(cnt, ref["count"])
    assert np.array_equal(frac, ref["frac"])
    assert np.array_equal(incl, ref["incl"])
    cnt32, frac32, _, _, _ = _gpu_filter(hm, w, "mixed")
    ref32 = ofilter.filter_field(w, "f32")
    assert np.array_equal(frac32, ref32["frac"])


@pytest.mark.parametrize("rule", ["none", "voigt", "reuss", "laminate"])
def test_solve_fixed_iterations_2d(hm, rule):
    w = workload_c1(rule)
    log("2d solve %s" % rule)
    _, frac_np, incl_np, frac, incl = _gpu_filter(hm, w)
    ref_f = ofilter.filter_field(w)
    for k in (0, 1, 7):
        out = hm.hm_solve(w.n, w.dim, w.phases, rule, frac, incl, w.spheres, w.loads, prec="fp64",
                          tol=0.0, max_iter=k, want_eps=True)
        r = oracle_solve(w, ref_f["frac"], ref_f["incl"], w.loads, 0.0, k)[0]
        assert out["reports"][0]["iters"] == r["iters"] == k
        assert out["reports"][0]["status"] == 1
        sig_ref = np.array([r["sig_mean"][i, j] for (i, j) in [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]])
        assert rel(out["sig_mean"][0], sig_ref) < 1e-10
        assert abs(out["reports"][0]["err"] - r["err"]) <= 1e-10 * r["err"] + 1e-13
        e_gpu = out["eps"][0].cpu().numpy()
        assert rel(e_gpu, oracle_fields_to_comps(r["eps"])) < 1e-10


def test_solve_fixed_iterations_3d_anisotropic_grid(hm):
    w = small_sphere_case(n=(15, 9, 21), fraction=0.15, contrast=20.0, rule="laminate",
                          radius_vox=1.0, subsamples=4, offset=(0.25, 0.5, -0.75))
    log("3d anisotropic grid solve")
    _, _, _, frac, incl = _gpu_filter(hm, w)
    ref_f = ofilter.filter_field(w)
    E = np.array([[0.01, -0.004, 0.002, 0.001, -0.003, 0.005], [0.0, 0.0, 0.0, 0.0, 0.0, 0.01]])
    out = hm.hm_solve(w.n, w.dim, w.phases, w.rule, frac, incl, w.spheres, E, prec="fp64", tol=0.0,
                      max_iter=6, want_eps=True)
    refs = oracle_solve(w, ref_f["frac"], ref_f["incl"], E, 0.0, 6)
    for l, r in enumerate(refs):
        sig_ref = np.array([r["sig_mean"][i, j] for (i, j) in [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]])
        assert rel(out["sig_mean"][l], sig_ref) < 1e-10
        assert abs(out["reports"][l]["err"] - r["err"]) <= 1e-10 * r["err"] + 1e-13
        assert rel(out["eps"][l].cpu().numpy(), oracle_fields_to_comps(r["eps"])) < 1e-10


@pytest.mark.parametrize("rule", ["reuss", "laminate"])
def test_mostly_fractional_field_grows_the_stiffness_table(hm, rule):
    # Half of the 45^3 voxels fractional: more rows than the stiffness table
    # of a fresh plan holds, so it grows and is rebuilt; then a sphere cell
    # with few fractional voxels reuses the grown table on the same plan.
    n = (45, 45, 45)
    w = small_sphere_case(n=n, fraction=0.2, contrast=8.0, rule=rule, radius_vox=1.0, subsamples=4)
    f = random_fraction_case(23, n).reshape(-1)
    incl = np.where((f > 0) & (f < 1), 0, -1).astype(np.int32)
    E = np.array([[0.01, -0.004, 0.002, 0.001, -0.003, 0.005], [0.0, 0.0, 0.0, 0.0, 0.0, 0.01]])
    hm.release_plans()
    log("stiffness table growth %s: %d fractional voxels" % (rule, int(np.sum(incl == 0))))
    cases = [(f, incl)]
    _, f2, i2, _, _ = _gpu_filter(hm, w)
    cases.append((f2, i2))
    for fr, ic in cases:
        out = hm.hm_solve(w.n, w.dim, w.phases, rule, torch.tensor(fr, device=DEV), torch.tensor(ic, device=DEV),
                          w.spheres, E, prec="fp64", tol=0.0, max_iter=3, want_eps=True)
        refs = oracle_solve(w, fr, ic, E, 0.0, 3)
        for l, r in enumerate(refs):
            sig_ref = np.array([r["sig_mean"][i, j] for (i, j) in [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]])
            assert rel(out["sig_mean"][l], sig_ref) < 1e-10
            assert abs(out["reports"][l]["err"] - r["err"]) <= 1e-10 * r["err"] + 1e-13
            assert rel(out["eps"][l].cpu().numpy(), oracle_fields_to_comps(r["eps"])) < 1e-10


def test_effective_tensor_converged_fp64(hm):
    w = small_sphere_case(n=(15, 15, 15), fraction=0.2, contrast=10.0, rule="laminate",
                          radius_vox=1.0, subsamples=4)
    log("effective tensor fp64")
    _, _, _, frac, incl = _gpu_filter(hm, w)
    out = hm.hm_effective_tensor(w.n, w.dim, w.phases, w.rule, frac, incl, w.spheres, prec="fp64",
                                 tol=1e-10, max_iter=2000, check_every=4)
    fld = osolver.build_field(w)
    C, reps = osolver.effective_tensor(fld, osolver.reference_medium(w.phases), 1e-10, 2000, 3)
    assert [r["iters"] for r in out["reports"]] == [r["iters"] for r in reps]
    assert rel(out["C"], C) < 1e-10
    assert all(r["status"] == 0 for r in out["reports"])


def test_effective_tensor_c1_tol(hm):
    w = workload_c1("none")
    log("c1 tol 1e-8")
    _, _, _, frac, incl = _gpu_filter(hm, w)
    out = hm.hm_solve(w.n, w.dim, w.phases, w.rule, frac, incl, w.spheres, w.loads, prec="fp64",
                      tol=w.tol, max_iter=5000, check_every=16)
    ref_f = ofilter.filter_field(w)
    r = oracle_solve(w, ref_f["frac"], ref_f["incl"], w.loads, w.tol, 5000)[0]
    assert out["reports"][0]["iters"] == r["iters"]
    assert out["reports"][0]["status"] == 0
    assert abs(out["sig_mean"][0][5] - r["sig_mean"][0, 1]) < 1e-10 * abs(r["sig_mean"][0, 1])


def test_mixed_precision_effective_tensor(hm):
    w = small_sphere_case(n=(27, 27, 27), fraction=0.25, contrast=20.0, rule="laminate",
                          radius_vox=1.0, subsamples=4)
    log("mixed effective tensor")
    _, _, _, frac32, incl = _gpu_filter(hm, w, "mixed")
    out = hm.hm_effective_tensor(w.n, w.dim, w.phases, w.rule, frac32, incl, w.spheres, prec="mixed",
                                 tol=1e-4, max_iter=3000, check_every=8, stall_window=20)
    fld = osolver.build_field(w)
    C, _ = osolver.effective_tensor(fld, osolver.reference_medium(w.phases), 1e-9, 3000, 3)
    log("mixed C rel err %.3e, iters %s" % (rel(out["C"], C), [r["iters"] for r in out["reports"]]))
    assert rel(out["C"], C) < 1e-5


def test_graph_replay_matches_eager(hm):
    w = small_sphere_case(n=(21, 21, 21), fraction=0.2, contrast=10.0, rule="voigt",
                          radius_vox=1.0, subsamples=4)
    log("graph vs eager")
    _, _, _, frac, incl = _gpu_filter(hm, w)
    a = hm.hm_effective_tensor(w.n, w.dim, w.phases, w.rule, frac, incl, w.spheres, prec="fp64",
                               tol=1e-6, max_iter=500, check_every=5, use_graph=False)
    for rep in range(3):
        b = hm.hm_effective_tensor(w.n, w.dim, w.phases, w.rule, frac, incl, w.spheres, prec="fp64",
                                   tol=1e-6, max_iter=500, check_every=5, use_graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(a["C"], b["C"])
        assert [r["iters"] for r in a["reports"]] == [r["iters"] for r in b["reports"]]


def test_status_codes(hm):
    w = small_sphere_case(n=(9, 9, 9), fraction=0.2, contrast=10.0, rule="voigt",
                          radius_vox=1.0, subsamples=4)
    log("status codes")
    _, _, _, frac, incl = _gpu_filter(hm, w)
    E = np.array([[0.01, 0, 0, 0, 0, 0]])
    bad = hm.hm_solve(w.n, w.dim, w.phases, "voigt", frac, incl, w.spheres, E, tol=1e-6, max_iter=2000,
                      c0_alpha=0.5, check_every=10)
    assert bad["status"] == 3 and bad["reports"][0]["status"] == 3
    few = hm.hm_solve(w.n, w.dim, w.phases, "voigt", frac, incl, w.spheres, E, tol=1e-12, max_iter=3)
    assert few["status"] == 1 and few["reports"][0]["iters"] == 3
    from paper_1412_3228_amd import HmError
    with pytest.raises(HmError) as ei:
        hm.hm_solve(w.n, w.dim, w.phases, "none", frac, incl, w.spheres, E, tol=1e-6, max_iter=5)
    assert ei.value.code == -5


def test_high_contrast_mean_stress_swing_is_not_divergence(hm):
    # contrast 1e3, shear load: e_i spikes far above e_0 while the residual
    # falls; GPU and oracle both run to convergence in the same iterations
    w = fig1_disk_case(7, 1e3, "none")
    log("mean stress swing")
    _, _, _, frac, incl = _gpu_filter(hm, w)
    ref_f = ofilter.filter_field(w)
    E = np.array([[0.0, 0.0, 0.0, 0.0, 0.0, 0.01]])
    out = hm.hm_solve(w.n, w.dim, w.phases, "none", frac, incl, w.spheres, E, prec="fp64", tol=1e-4,
                      max_iter=5000, check_every=1)
    r = oracle_solve(w, ref_f["frac"], ref_f["incl"], E, 1e-4, 5000)[0]
    assert r["status"] == 0 and max(r["errs"]) > 1e3 * r["errs"][0]
    assert out["reports"][0]["status"] == 0
    assert out["reports"][0]["iters"] == r["iters"]
    sig_ref = np.array([r["sig_mean"][i, j] for (i, j) in [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]])
    assert rel(out["sig_mean"][0], sig_ref) < 1e-10


def test_adjoint_matches_oracle_gradient(hm):
    w = small_sphere_case(n=(9, 9, 9), fraction=0.2, contrast=5.0, rule="laminate",
                          radius_vox=1.0, subsamples=4)
    log("adjoint")
    _, _, _, frac, incl = _gpu_filter(hm, w)
    out = hm.hm_effective_tensor(w.n, w.dim, w.phases, w.rule, frac, incl, w.spheres, prec="fp64",
                                 tol=1e-12, max_iter=3000, check_every=8, want_eps=True)
    G = np.random.default_rng(3).standard_normal((6, 6))
    dph, dfr = hm.hm_solve_adjoint(w.n, w.dim, w.phases, w.rule, frac, incl, w.spheres, G, out["eps"])
    flt = ofilter.filter_field(w)
    vox = ofilter.all_voxels(w.n)
    nrm = ofilter.interface_normals(w.n, 3, w.spheres, flt["incl"], vox)
    fld = osolver.StiffnessField(w.n, 3, w.phases, "laminate", flt["frac"], nrm)
    C, reps = osolver.effective_tensor(fld, osolver.reference_medium(w.phases), 1e-12, 3000, 3, keep_fields=True)
    rph, rfr = ogradient.hill_gradient(fld, [r["eps"] for r in reps], G, w.phases, nrm)
    assert rel(dph, rph) < 1e-9
    assert rel(dfr.cpu().numpy(), rfr) < 1e-9


def test_profiled_solve_matches_and_reports_timing(hm):
    w = small_sphere_case(n=(21, 21, 21), fraction=0.2, contrast=10.0, rule="laminate",
                          radius_vox=1.0, subsamples=4)
    log("profiled solve")
    _, _, _, frac, incl = _gpu_filter(hm, w)
    a = hm.hm_effective_tensor(w.n, w.dim, w.phases, w.rule, frac, incl, w.spheres, prec="fp64",
                               tol=1e-6, max_iter=500, check_every=7)
    b = hm.hm_effective_tensor(w.n, w.dim, w.phases, w.rule, frac, incl, w.spheres, prec="fp64",
                               tol=1e-6, max_iter=500, check_every=7, profile=True)
    assert np.array_equal(a["C"], b["C"])
    t = hm.last_timing()
    # events around the kernels of iterations 1, 5, 9, ... up to the last one evaluated
    its = [r["iters"] for r in b["reports"]]
    sampled = list(range(1, max(its) + 1, 4))
    assert len(sampled) >= 2
    assert t["iterations"] == len(sampled)
    assert t["active_loads"] == pytest.approx(np.mean([sum(n >= i for n in its) for i in sampled]), rel=1e-12)
    assert all(t["ms"][k] > 0 for k in ("xsweep", "ysweep_fwd", "zsweep", "ysweep_inv"))
    assert t["ms"]["finalize"] == 0.0  # the inverse y-sweep ends the iteration
    # instance names as profilers print them: sweep<double,21,...>
    for k in ("xsweep", "ysweep_fwd", "zsweep", "ysweep_inv"):
        assert t["kernels"][k].startswith(k.split("_")[0]) and "<double,21," in t["kernels"][k]
    assert t["kernels"]["ysweep_fwd"].endswith(",-1>") and t["kernels"]["ysweep_inv"].endswith(",1>")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n", [(45, 45, 45), (27, 21, 25), (63, 15, 35)])
def test_every_compiled_schedule_matches_oracle(hm, prec, n):
    """Each tile-schedule variant the autotuner may pick gives the oracle's iterate."""
    w = small_sphere_case(n=n, fraction=0.2, contrast=20.0, rule="laminate", radius_vox=1.0, subsamples=4,
                          offset=(0.5, -0.25, 0.125))
    nx, ny, nz = hm.schedule_count(w.n, 3, prec)
    log("schedules %s %s: %d x %d x %d" % (prec, n, nx, ny, nz))
    _, _, _, frac, incl = _gpu_filter(hm, w, prec)
    ref_f = ofilter.filter_field(w)
    k = 3
    refs = oracle_solve(w, ref_f["frac"], ref_f["incl"], w.loads[[0, 5]], 0.0, k)
    tol = 1e-10 if prec == "fp64" else 2e-5
    combos = [(x, 0, 0) for x in range(nx)] + [(0, y, 0) for y in range(ny)] + [(0, 0, z) for z in range(nz)]
    for sch in combos:
        out = hm.hm_effective_tensor(w.n, 3, w.phases, w.rule, frac, incl, w.spheres, prec=prec, tol=0.0,
                                     max_iter=k, schedule=sch, want_eps=True)
        for col, r in zip((0, 5), refs):
            e = out["eps"][col].cpu().numpy().astype(np.float64)
            err = rel(e, oracle_fields_to_comps(r["eps"]))
            assert err < tol, (sch, col, err)


def test_history_matches_oracle_iterates(hm):
    """hm_last_history: e_i and <sigma_i> of every iterate against the oracle's."""
    w = small_sphere_case(n=(15, 9, 21), fraction=0.15, contrast=20.0, rule="laminate",
                          radius_vox=1.0, subsamples=4, offset=(0.25, 0.5, -0.75))
    log("iterate history")
    _, _, _, frac, incl = _gpu_filter(hm, w)
    ref_f = ofilter.filter_field(w)
    E = np.array([[0.01, -0.004, 0.002, 0.001, -0.003, 0.005], [0.0, 0.0, 0.0, 0.0, 0.0, 0.01]])
    K = 5
    hm.hm_solve(w.n, w.dim, w.phases, w.rule, frac, incl, w.spheres, E, prec="fp64", tol=0.0, max_iter=K,
                check_every=2, use_graph=True)
    err, sig = hm.last_history(2, K + 3)
    assert np.all(np.isnan(err[:, K + 1:])) and np.all(np.isnan(sig[:, K + 1:]))
    for k in range(K + 1):
        refs = oracle_solve(w, ref_f["frac"], ref_f["incl"], E, 0.0, k)
        for l, r in enumerate(refs):
            s_ref = np.array([r["sig_mean"][i, j] for (i, j) in [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]])
            assert rel(sig[l, k], s_ref) < 1e-10
            assert abs(err[l, k] - r["err"]) <= 1e-10 * r["err"] + 1e-13
    from paper_1412_3228_amd import HmError
    with pytest.raises(HmError):
        hm.last_history(3, 4)
