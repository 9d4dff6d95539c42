"""GPU parity of the multi-phase path (eqs. 3-4 with Nphase phases) against
oracle/nphase.py: per-phase filter counts bit-exact; FP64 mean stress,
error and strain field within 1e-10 at fixed iteration counts for Voigt
and Reuss on a four-phase cell (pure phase-3 voxels through the reserved
table rows); tolerance stops in the same iteration; mixed precision within
1e-5; two phases through the multi-phase entry points equal the two-phase
solve; conjugate gradients reach the same tensor; bad input is refused."""
import numpy as np
import pytest
import torch

from gpu_helpers import COMPS, log, oracle_fields_to_comps, rel
from oracle import nphase as NP, solver as osolver
from workloads import lame

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
N_CELL = (15, 9, 21)
SPH = np.array([[3.5, 2.5, 4.0, 2.2], [10.0, 6.0, 5.5, 2.6], [7.5, 4.5, 13.0, 3.1], [12.5, 2.0, 17.5, 1.8],
                [2.5, 6.5, 16.0, 1.9]])
LAB = np.array([1, 2, 1, 3, 2])
PH4 = [lame(1.0, 0.3), lame(15.0, 0.25), lame(0.1, 0.35), lame(4.0, 0.2)]


@pytest.fixture(scope="module")
def hm():
    import paper_1412_3228_amd as hm_mod
    assert torch.cuda.is_available() and hm_mod.device_ok()
    return hm_mod


def _sig6(s):
    return np.array([s[i, j] for (i, j) in COMPS])


@pytest.mark.parametrize("radius,S,rule", [(1.0, 4, "voigt"), (0.55, 8, "reuss"), (1.0, 4, "none")])
def test_phase_counts_bit_exact(hm, radius, S, rule):
    log("phase counts r=%g S=%d %s" % (radius, S, rule))
    cnt, frac = hm.hm_filter_phases(N_CELL, 3, SPH, LAB, 4, radius, S, rule, "fp64", DEV)
    ref, M = NP.phase_counts(N_CELL, 3, SPH, LAB, 4, radius if rule != "none" else 0.0, S)
    assert np.array_equal(cnt.cpu().numpy(), ref)
    assert np.array_equal(frac.cpu().numpy(), NP.fractions(ref, M))
    _, f32 = hm.hm_filter_phases(N_CELL, 3, SPH, LAB, 4, radius, S, rule, "mixed", DEV)
    assert np.array_equal(f32.cpu().numpy(), NP.fractions(ref, M, "f32"))


@pytest.mark.parametrize("rule", ["voigt", "reuss"])
@pytest.mark.parametrize("k", [0, 1, 5])
def test_fixed_iterations_match_oracle(hm, rule, k):
    log("nphase fixed iterations %s k=%d" % (rule, k))
    cnt, frac = hm.hm_filter_phases(N_CELL, 3, SPH, LAB, 4, 1.0, 4, rule, "fp64", DEV)
    ref, M = NP.phase_counts(N_CELL, 3, SPH, LAB, 4, 1.0, 4)
    fld = NP.NPhaseField(N_CELL, 3, PH4, rule, NP.fractions(ref, M))
    assert np.any(NP.fractions(ref, M)[2] == 1.0)  # pure phase-3 voxels exist
    E = np.array([[0.01, -0.004, 0.002, 0.001, -0.003, 0.005], [0.0, 0.0, 0.0, 0.0, 0.0, 0.01]])
    out = hm.hm_solve_phases(N_CELL, 3, PH4, rule, frac, E, prec="fp64", tol=0.0, max_iter=k, want_eps=True)
    c0 = NP.reference_medium(PH4)
    for l in range(2):
        r = osolver.solve(fld, E[l], c0, 0.0, k)
        rep = out["reports"][l]
        assert rep["iters"] == r["iters"] == k
        assert rel(out["sig_mean"][l], _sig6(r["sig_mean"])) < 1e-10
        assert abs(rep["err"] - r["err"]) <= 1e-10 * r["err"] + 1e-13
        assert rel(out["eps"][l].cpu().numpy(), oracle_fields_to_comps(r["eps"])) < 1e-10


@pytest.mark.parametrize("prec,tol,tol_c", [("fp64", 1e-6, 1e-9), ("mixed", 1e-4, 1e-5)])
def test_effective_tensor_tolerance_stop(hm, prec, tol, tol_c):
    log("nphase effective tensor %s" % prec)
    cnt, frac = hm.hm_filter_phases(N_CELL, 3, SPH, LAB, 4, 1.0, 4, "voigt", prec, DEV)
    ref, M = NP.phase_counts(N_CELL, 3, SPH, LAB, 4, 1.0, 4)
    fld = NP.NPhaseField(N_CELL, 3, PH4, "voigt", NP.fractions(ref, M, "f32" if prec == "mixed" else "f64"))
    C, reps = osolver.effective_tensor(fld, NP.reference_medium(PH4), tol, 5000, 3)
    out = hm.hm_effective_tensor_phases(N_CELL, 3, PH4, "voigt", frac, prec=prec, tol=tol, max_iter=5000,
                                        use_graph=True, check_every=4)
    assert out["status"] == 0
    assert rel(out["C"], C) < tol_c
    if prec == "fp64":
        # (single precision: near e = 1e-4 its residual carries rounding noise
        # of that order at this contrast, so the stop iteration moves)
        assert [r["iters"] for r in out["reports"]] == [r["iters"] for r in reps]


@pytest.mark.parametrize("rule", ["voigt", "reuss"])
def test_two_phases_equal_the_two_phase_solve(hm, rule):
    ph2 = PH4[:2]
    lab = np.ones(len(SPH), dtype=int)
    _, frac_p = hm.hm_filter_phases(N_CELL, 3, SPH, lab, 2, 1.0, 4, rule, "fp64", DEV)
    _, frac, incl = hm.hm_filter(N_CELL, 3, SPH, 1.0, 4, rule, "fp64", DEV)
    assert torch.equal(frac_p.reshape(-1), frac)
    a = hm.hm_effective_tensor_phases(N_CELL, 3, ph2, rule, frac_p, tol=1e-8, max_iter=3000)
    b = hm.hm_effective_tensor(N_CELL, 3, ph2, rule, frac, incl, SPH, tol=1e-8, max_iter=3000, autotune=False)
    assert rel(a["C"], b["C"]) < 1e-14
    assert [r["iters"] for r in a["reports"]] == [r["iters"] for r in b["reports"]]


def test_conjugate_gradients_reach_the_fixed_point_tensor(hm):
    _, frac = hm.hm_filter_phases(N_CELL, 3, SPH, LAB, 4, 1.0, 4, "reuss", "fp64", DEV)
    fp = hm.hm_effective_tensor_phases(N_CELL, 3, PH4, "reuss", frac, tol=1e-10, max_iter=20000, check_every=16,
                                       use_graph=True)
    cg = hm.hm_effective_tensor_phases(N_CELL, 3, PH4, "reuss", frac, tol=1e-10, max_iter=2000, method="cg",
                                       check_every=8, use_graph=True)
    assert fp["status"] == 0 and cg["status"] == 0
    assert rel(cg["C"], fp["C"]) < 1e-7
    assert max(r["iters"] for r in cg["reports"]) < max(r["iters"] for r in fp["reports"])


def test_bad_input_is_refused(hm):
    with pytest.raises(hm.HmError) as e:  # spheres of phases 1 and 2 overlapping
        hm.hm_filter_phases(N_CELL, 3, np.array([[5.0, 4.0, 5.0, 2.5], [7.0, 4.0, 5.0, 2.5]]), [1, 2], 3, 1.0, 4,
                            "voigt", "fp64", DEV)
    assert e.value.code == -1
    _, frac = hm.hm_filter_phases(N_CELL, 3, SPH, LAB, 4, 1.0, 4, "voigt", "fp64", DEV)
    with pytest.raises(hm.HmError) as e:
        hm.hm_effective_tensor_phases(N_CELL, 3, PH4, "laminate", frac, max_iter=2)
    assert e.value.code == -1
    with pytest.raises(hm.HmError) as e:
        hm.hm_effective_tensor_phases(N_CELL, 3, PH4, "none", frac, max_iter=2)
    assert e.value.code == -5


def test_2d_cell_and_an_unused_phase(hm):
    # plane strain, four phases of which label 3 has no inclusion
    n = (21, 15, 1)
    sph = np.array([[5.0, 4.0, 0.5, 3.2], [15.0, 10.5, 0.5, 3.6], [14.5, 3.0, 0.5, 2.1]])
    lab = np.array([1, 2, 1])
    cnt, frac = hm.hm_filter_phases(n, 2, sph, lab, 4, 1.0, 8, "voigt", "fp64", DEV)
    ref, M = NP.phase_counts(n, 2, sph, lab, 4, 1.0, 8)
    assert np.array_equal(cnt.cpu().numpy(), ref) and not ref[2].any()
    fld = NP.NPhaseField(n, 2, PH4, "voigt", NP.fractions(ref, M))
    C, _ = osolver.effective_tensor(fld, NP.reference_medium(PH4), 0.0, 6, 2)
    out = hm.hm_effective_tensor_phases(n, 2, PH4, "voigt", frac, tol=0.0, max_iter=6)
    assert rel(out["C"], C) < 1e-10
