"""GPU edge cases of the solve: cells with no interface (homogeneous,
all-inclusion, contrast 1), the smallest grids (3^3, a ragged 2D 5 x 3),
against closed forms or the oracle, for both the fixed-point and the
conjugate-gradient method; sizes outside the supported set are refused."""
import numpy as np
import pytest
import torch

from gpu_helpers import oracle_fields_to_comps, oracle_solve, rel
from oracle import filter as ofilter, rules as orules
from workloads import lame, small_sphere_case

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
METHODS = ["fixed_point", "cg"]


@pytest.fixture(scope="module")
def hm():
    import paper_1412_3228_amd as hm_mod
    assert torch.cuda.is_available() and hm_mod.device_ok()
    return hm_mod


def _tensor(ph):
    return orules.to_mandel(orules.iso_tensor(*ph))


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("case", ["no-sphere", "all-inclusion", "contrast-1"])
def test_cells_without_interface_give_the_phase_tensor(hm, case, method):
    n = (9, 15, 5)
    w = small_sphere_case(n=n, fraction=0.2, contrast=7.0, rule="laminate", radius_vox=1.0, subsamples=4)
    sph = w.spheres
    phase = w.phases[0]
    if case == "no-sphere":
        sph = np.zeros((0, 4))
    elif case == "all-inclusion":
        sph = np.array([[n[0] / 2.0, n[1] / 2.0, n[2] / 2.0, 4.0 * max(n)]])
        phase = w.phases[1]
    elif case == "contrast-1":
        w = w.with_(phases=(lame(2.0, 0.25), lame(2.0, 0.25)))
        phase = w.phases[0]
    _, frac, incl = hm.hm_filter(w.n, 3, sph, w.radius_vox, w.subsamples, w.rule, "fp64", DEV)
    out = hm.hm_effective_tensor(w.n, 3, w.phases, w.rule, frac, incl, sph, prec="fp64", tol=1e-10,
                                 max_iter=50, method=method)
    assert all(r["status"] == 0 for r in out["reports"])
    assert all(r["iters"] <= 1 for r in out["reports"])
    assert rel(out["C"], _tensor(phase)) < 1e-12


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("shape", [(3, 3, 3), (5, 3, 1)])
def test_smallest_grids_match_oracle(hm, shape, method):
    dim = 2 if shape[2] == 1 else 3
    w = small_sphere_case(n=shape, dim=dim, fraction=0.3, contrast=15.0, rule="laminate",
                          radius_vox=0.7, subsamples=8)
    _, frac, incl = hm.hm_filter(w.n, dim, w.spheres, w.radius_vox, w.subsamples, w.rule, "fp64", DEV)
    ref_f = ofilter.filter_field(w)
    E = np.array([[0.01, -0.004, 0.0 if dim == 2 else 0.002, 0.0, 0.0, 0.005]])
    out = hm.hm_solve(w.n, dim, w.phases, w.rule, frac, incl, w.spheres, E, prec="fp64", tol=0.0, max_iter=4,
                      want_eps=True, method=method)
    if method == "cg":
        from oracle import solver as osolver
        from test_gpu_cg import _field
        r = osolver.solve_cg(_field(w, ref_f), E[0], 0.0, 4)
    else:
        r = oracle_solve(w, ref_f["frac"], ref_f["incl"], E, 0.0, 4)[0]
    sig = np.array([r["sig_mean"][i, j] for (i, j) in [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]])
    assert rel(out["sig_mean"][0], sig) < 1e-10
    assert rel(out["eps"][0].cpu().numpy(), oracle_fields_to_comps(r["eps"])) < 1e-10


@pytest.mark.parametrize("shape", [(1, 1, 1), (4, 9, 9), (245, 5, 5), (17, 9, 9), (143, 9, 9)])
def test_unsupported_sizes_are_refused(hm, shape):
    from paper_1412_3228_amd import HmError
    with pytest.raises(HmError) as ei:
        hm.hm_filter(shape, 3, np.zeros((0, 4)), 1.0, 4, "laminate", "fp64", DEV)
    assert ei.value.code == -2
