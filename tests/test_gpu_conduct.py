"""GPU parity of the conduction solve (the scalar-conductivity form of the
filtered fixed point) against oracle/thermal.py: at fixed iteration counts
the FP64 mean flux, error and gradient field agree within 1e-10 for every
rule on a cell that spans several x-sweep blocks and z tiles with ragged
tails; tolerance stops take the same iteration; mixed precision within
1e-5; grid-aligned layers give the arithmetic and harmonic means; graph
replay equals direct launches; at the 125^3 workload the first iterates
match the oracle; bad input is refused."""
import numpy as np
import pytest
import torch

from gpu_helpers import band_oracle_filter, log, rel
from oracle import filter as ofilter, thermal as othermal
from workloads import small_sphere_case, workload_c2

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
K2 = (1.0, 10.0)


@pytest.fixture(scope="module")
def hm():
    import paper_1412_3228_amd as hm_mod
    assert torch.cuda.is_available() and hm_mod.device_ok()
    return hm_mod


def _oracle_field(w, ref_f, k):
    nrm = None
    if w.rule == "laminate":
        nrm = ofilter.interface_normals(w.n, w.dim, w.spheres, ref_f["incl"], ofilter.all_voxels(w.n))
    return othermal.ConductivityField(w.n, w.dim, k, w.rule, ref_f["frac"], nrm)


def _grad_comps(g):
    """(nz, ny, nx, 3) -> (3, N)."""
    return np.moveaxis(g.reshape(-1, 3), 1, 0)


def _case(rule, n=(21, 9, 15)):
    return small_sphere_case(n=n, fraction=0.15, contrast=10.0, rule=rule, radius_vox=1.0, subsamples=4,
                             offset=(0.25, 0.5, -0.75))


@pytest.mark.parametrize("rule", ["voigt", "reuss", "laminate"])
@pytest.mark.parametrize("k", [0, 1, 7])
def test_conduction_fixed_iterations_match_oracle(hm, rule, k):
    w = _case(rule)
    log("conduction fixed iterations rule=%s k=%d n=%s" % (rule, k, w.n))
    _, frac, incl = hm.hm_filter(w.n, w.dim, w.spheres, w.radius_vox, w.subsamples, w.rule, "fp64", DEV)
    ref_f = ofilter.filter_field(w)
    fld = _oracle_field(w, ref_f, K2)
    k0 = othermal.reference_conductivity(K2)
    G = np.array([[1.0, 0.0, 0.0], [0.3, -0.7, 0.2]])
    out = hm.hm_conduct_solve(w.n, w.dim, K2, w.rule, frac, incl, w.spheres, G, prec="fp64", tol=0.0,
                              max_iter=k, want_grad=True)
    for l in range(2):
        r = othermal.solve(fld, G[l], k0, 0.0, k)
        rep = out["reports"][l]
        assert rep["iters"] == r["iters"] == k and rep["status"] == 1
        assert rel(out["flux_mean"][l], r["flux_mean"]) < 1e-10
        assert abs(rep["err"] - r["err"]) <= 1e-10 * r["err"]
        assert abs(rep["err0"] - r["errs"][0]) <= 1e-10 * r["errs"][0]
        assert rel(out["grad"][l].cpu().numpy(), _grad_comps(r["grad"])) < 1e-10


# single precision stalls near e ~ 1e-6, so its stop is taken at 1e-4
@pytest.mark.parametrize("prec,tol,tol_k", [("fp64", 1e-6, 1e-9), ("mixed", 1e-4, 1e-5)])
def test_effective_conductivity_tolerance_stop(hm, prec, tol, tol_k):
    w = _case("laminate", n=(15, 15, 15))
    log("conduction tolerance stop prec=%s" % prec)
    _, frac, incl = hm.hm_filter(w.n, w.dim, w.spheres, w.radius_vox, w.subsamples, w.rule, prec, DEV)
    ref_f = ofilter.filter_field(w)
    fld = _oracle_field(w, ref_f, K2)
    Kref, reps = othermal.effective_conductivity(fld, othermal.reference_conductivity(K2), tol, 2000, 3)
    out = hm.hm_effective_conductivity(w.n, w.dim, K2, w.rule, frac, incl, w.spheres, prec=prec, tol=tol,
                                       max_iter=2000, use_graph=True, check_every=4)
    assert out["status"] == 0
    assert rel(out["K"], Kref) < tol_k
    for J in range(3):
        it_gpu, it_ref = out["reports"][J]["iters"], reps[J]["iters"]
        assert it_gpu == it_ref if prec == "fp64" else abs(it_gpu - it_ref) <= 2


def test_conduction_2d_disk_matches_oracle(hm):
    w = small_sphere_case(n=(25, 15, 1), dim=2, fraction=0.3, contrast=0.05, rule="laminate", radius_vox=1.0,
                          subsamples=8, offset=(0.3, -0.2, 0.0))
    k = (1.0, 0.05)
    log("conduction 2d disk")
    _, frac, incl = hm.hm_filter(w.n, w.dim, w.spheres, w.radius_vox, w.subsamples, w.rule, "fp64", DEV)
    ref_f = ofilter.filter_field(w)
    fld = _oracle_field(w, ref_f, k)
    Kref, reps = othermal.effective_conductivity(fld, othermal.reference_conductivity(k), 0.0, 9, 2)
    out = hm.hm_effective_conductivity(w.n, w.dim, k, w.rule, frac, incl, w.spheres, prec="fp64", tol=0.0,
                                       max_iter=9)
    assert out["K"].shape == (2, 2)
    assert rel(out["K"], Kref) < 1e-10
    for J in range(2):
        assert abs(out["reports"][J]["err"] - reps[J]["err"]) <= 1e-10 * reps[J]["err"]


def test_grid_aligned_layers_give_the_means(hm):
    # pure-voxel layers normal to x: harmonic mean across, arithmetic along
    n = (9, 5, 3)
    rows = np.array([0, 1, 1, 0, 0, 1, 0, 0, 0], dtype=np.float64)
    frac = torch.tensor(np.broadcast_to(rows[None, None, :], (n[2], n[1], n[0])).reshape(-1).copy(),
                        dtype=torch.float64, device=DEV)
    log("conduction layered cell")
    out = hm.hm_effective_conductivity(n, 3, K2, "none", frac, None, np.zeros((0, 4)), prec="fp64", tol=1e-12,
                                       max_iter=5000)
    f = rows.mean()
    harm = 1.0 / ((1 - f) / K2[0] + f / K2[1])
    arith = (1 - f) * K2[0] + f * K2[1]
    assert np.allclose(np.diag(out["K"]), [harm, arith, arith], rtol=1e-9)
    assert np.max(np.abs(out["K"] - np.diag(np.diag(out["K"])))) < 1e-9


def test_graph_replay_equals_direct_launches(hm):
    w = _case("laminate")
    log("conduction graph replay")
    _, frac, incl = hm.hm_filter(w.n, w.dim, w.spheres, w.radius_vox, w.subsamples, w.rule, "mixed", DEV)
    a = hm.hm_effective_conductivity(w.n, w.dim, K2, w.rule, frac, incl, w.spheres, prec="mixed", tol=1e-5,
                                     max_iter=500, use_graph=False, check_every=3)
    b = hm.hm_effective_conductivity(w.n, w.dim, K2, w.rule, frac, incl, w.spheres, prec="mixed", tol=1e-5,
                                     max_iter=500, use_graph=True, check_every=3)
    c = hm.hm_effective_conductivity(w.n, w.dim, K2, w.rule, frac, incl, w.spheres, prec="mixed", tol=1e-5,
                                     max_iter=500, use_graph=True, check_every=3)
    assert np.array_equal(a["K"], b["K"]) and np.array_equal(b["K"], c["K"])
    assert [r["iters"] for r in a["reports"]] == [r["iters"] for r in b["reports"]]


def test_full_size_first_iterates_match_oracle(hm):
    # the 125^3 sphere cell of the benchmark: one FP64 iteration field by
    # field and two mixed-precision iterations against the oracle (oracle
    # fractions from its own counts near the surface, pure voxels elsewhere)
    w = workload_c2(contrast=100.0, n=125)
    k = (1.0, 100.0)
    log("conduction 125^3: oracle band filter")
    cnt_o, frac_o, incl_o, M = band_oracle_filter(w)
    nrm = ofilter.interface_normals(w.n, 3, w.spheres, incl_o, ofilter.all_voxels(w.n))
    fld = othermal.ConductivityField(w.n, 3, k, w.rule, frac_o, nrm)
    k0 = othermal.reference_conductivity(k)
    G = np.array([[0.0, 1.0, 0.0]])
    for prec, it, tol in (("fp64", 1, 1e-10), ("mixed", 2, 1e-5)):
        log("conduction 125^3: %s, %d iterations" % (prec, it))
        cnt, frac, incl = hm.hm_filter(w.n, w.dim, w.spheres, w.radius_vox, w.subsamples, w.rule, prec, DEV)
        assert np.array_equal(cnt.cpu().numpy(), cnt_o)
        r = othermal.solve(fld, G[0], k0, 0.0, it)
        out = hm.hm_conduct_solve(w.n, w.dim, k, w.rule, frac, incl, w.spheres, G, prec=prec, tol=0.0,
                                  max_iter=it, want_grad=(prec == "fp64"))
        assert rel(out["flux_mean"][0], r["flux_mean"]) < tol
        assert abs(out["reports"][0]["err"] - r["err"]) <= 10 * tol * r["err"]
        if prec == "fp64":
            assert rel(out["grad"][0].cpu().numpy(), _grad_comps(r["grad"])) < tol


def test_bad_input_is_refused(hm):
    w = _case("voigt", n=(9, 9, 9))
    _, frac, incl = hm.hm_filter(w.n, w.dim, w.spheres, w.radius_vox, w.subsamples, w.rule, "fp64", DEV)
    G = np.array([[1.0, 0.0, 0.0]])
    with pytest.raises(hm.HmError) as e:
        hm.hm_conduct_solve(w.n, w.dim, (1.0, -2.0), w.rule, frac, incl, w.spheres, G, max_iter=3)
    assert e.value.code == -1
    with pytest.raises(hm.HmError) as e:  # fractional voxels under the no-filter rule
        hm.hm_conduct_solve(w.n, w.dim, K2, "none", frac, incl, w.spheres, G, max_iter=3)
    assert e.value.code == -5
    f11 = torch.zeros(11 * 9 * 9, dtype=torch.float64, device=DEV)
    with pytest.raises(hm.HmError) as e:  # no conduction transform of length 11
        hm.hm_conduct_solve((11, 9, 9), 3, K2, "voigt", f11, None, w.spheres, G, max_iter=3)
    assert e.value.code == -2


@pytest.mark.parametrize("rule", ["voigt", "reuss", "laminate"])
def test_flux_field_matches_oracle(hm, rule):
    # local flux q = k~ g of the exported gradient fields
    w = _case(rule)
    _, frac, incl = hm.hm_filter(w.n, w.dim, w.spheres, w.radius_vox, w.subsamples, w.rule, "fp64", DEV)
    ref_f = ofilter.filter_field(w)
    fld = _oracle_field(w, ref_f, K2)
    G = np.array([[0.3, -0.7, 0.2]])
    out = hm.hm_conduct_solve(w.n, w.dim, K2, rule, frac, incl, w.spheres, G, tol=0.0, max_iter=4, want_grad=True)
    q = hm.hm_flux_field(w.n, w.dim, K2, rule, frac, incl, w.spheres, out["grad"]).cpu().numpy()
    r = othermal.solve(fld, G[0], othermal.reference_conductivity(K2), 0.0, 4)
    assert rel(q[0], _grad_comps(fld.apply(r["grad"]))) < 1e-10
