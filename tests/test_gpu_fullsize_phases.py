"""Full-size (125^3) checks of the anisotropic-phase and three-phase paths
at the sizes bench.py measures them:

* anisotropic cell (cubic inclusion, 2-layer rule): one FP64 iteration
  field by field against the oracle (oracle counts on the surface band,
  pure voxels elsewhere), mixed within 1e-5 of FP64 after two iterations;
* three-phase cell (20 spheres, two inclusion phases): per-phase counts at
  sampled voxels bit-exact against the oracle; making phase 2 identical to
  phase 1 reproduces the two-phase solve of the union (merging identical
  phases changes nothing); the tightly converged (1e-9) FP64 tensor is
  symmetric and inside the Voigt and Reuss bounds of the mean fractions;
  the mixed tensor is within 1e-5 of it.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import COMPS, band_oracle_filter, log, oracle_fields_to_comps, rel
from oracle import aniso as A, filter as ofilter, nphase as NP, rules, solver as osolver  # noqa: F401
from workloads import workload_aniso, workload_nphase

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def hm():
    import paper_1412_3228_amd as hm_mod
    assert torch.cuda.is_available() and hm_mod.device_ok()
    return hm_mod


def test_aniso_cell_first_iterates(hm):
    w = workload_aniso()
    cm = w.meta["C_mandel"]
    log("aniso 125^3: oracle band filter")
    cnt_o, frac_o, incl_o, M = band_oracle_filter(w)
    nrm = ofilter.interface_normals(w.n, 3, w.spheres, incl_o, ofilter.all_voxels(w.n))
    cph = [rules.from_mandel(cm[0]), rules.from_mandel(cm[1])]
    fld = A.AnisoField(w.n, 3, cph, w.rule, frac_o, nrm)
    E = np.array([[0.0, 0.0, 0.0, 0.0, 0.0, 0.01]])
    r = osolver.solve(fld, E[0], A.reference_medium(cph), 0.0, 1)
    log("aniso 125^3: GPU fp64, one iteration")
    cnt, frac, incl = hm.hm_filter(w.n, w.dim, w.spheres, w.radius_vox, w.subsamples, w.rule, "fp64", DEV)
    assert np.array_equal(cnt.cpu().numpy(), cnt_o)
    out = hm.hm_solve_aniso(w.n, 3, cm, w.rule, frac, incl, w.spheres, E, tol=0.0, max_iter=1, want_eps=True)
    sig = np.array([r["sig_mean"][i, j] for (i, j) in COMPS])
    assert rel(out["sig_mean"][0], sig) < 1e-10
    assert abs(out["reports"][0]["err"] - r["err"]) <= 1e-10 * r["err"]
    assert rel(out["eps"][0].cpu().numpy(), oracle_fields_to_comps(r["eps"])) < 1e-10
    _, f32, i32 = hm.hm_filter(w.n, w.dim, w.spheres, w.radius_vox, w.subsamples, w.rule, "mixed", DEV)
    o64 = hm.hm_solve_aniso(w.n, 3, cm, w.rule, frac, incl, w.spheres, E, tol=0.0, max_iter=2)
    o32 = hm.hm_solve_aniso(w.n, 3, cm, w.rule, f32, i32, w.spheres, E, prec="mixed", tol=0.0, max_iter=2)
    assert rel(o32["sig_mean"], o64["sig_mean"]) < 1e-5


def test_three_phase_cell_properties(hm):
    w = workload_nphase()
    lab, ph = w.meta["labels"], w.meta["phases"]
    log("nphase 125^3: sampled counts")
    cnt, frac = hm.hm_filter_phases(w.n, 3, w.spheres, lab, 3, w.radius_vox, w.subsamples, w.rule, "fp64", DEV)
    c = cnt.cpu().numpy()
    M = ofilter.stencil_offsets(w.radius_vox, w.subsamples, 3).shape[0]
    rng = np.random.default_rng(11)
    mixed = np.nonzero(((c > 0) & (c < M)).any(axis=0))[0]
    pick = np.concatenate([rng.choice(c.shape[1], 100, replace=False), rng.choice(mixed, 100, replace=False)])
    vox = ofilter.all_voxels(w.n)[pick]
    ref, M2 = NP.phase_counts(w.n, 3, w.spheres, lab, 3, w.radius_vox, w.subsamples, vox)
    assert M2 == M and np.array_equal(c[:, pick], ref)
    log("nphase 125^3: merged phases vs two-phase solve")
    ph_same = [ph[0], ph[1], ph[1]]
    a = hm.hm_effective_tensor_phases(w.n, 3, ph_same, w.rule, frac, tol=0.0, max_iter=30)
    _, fu, iu = hm.hm_filter(w.n, 3, w.spheres, w.radius_vox, w.subsamples, w.rule, "fp64", DEV)
    b = hm.hm_effective_tensor(w.n, 3, (ph[0], ph[1]), w.rule, fu, iu, w.spheres, tol=0.0, max_iter=30,
                               autotune=False)
    assert rel(a["C"], b["C"]) < 1e-12
    log("nphase 125^3: three phases, fp64 (tight) and mixed")
    o64 = hm.hm_effective_tensor_phases(w.n, 3, ph, w.rule, frac, tol=1e-9, max_iter=20000, check_every=32,
                                        use_graph=True)
    _, f32 = hm.hm_filter_phases(w.n, 3, w.spheres, lab, 3, w.radius_vox, w.subsamples, w.rule, "mixed", DEV)
    o32 = hm.hm_effective_tensor_phases(w.n, 3, ph, w.rule, f32, prec="mixed", tol=1e-4, max_iter=5000,
                                        check_every=16, stall_window=20, use_graph=True)
    C = o64["C"]
    log("nphase 125^3: fp64 iters %s, mixed statuses %s errors %s, mixed vs fp64 %.2e"
        % ([r["iters"] for r in o64["reports"]], [r["status"] for r in o32["reports"]],
           ["%.1e" % r["err"] for r in o32["reports"]], rel(o32["C"], C)))
    assert o64["status"] == 0
    assert all(r["status"] in (0, 2) for r in o32["reports"])
    assert np.allclose(C, C.T, rtol=0, atol=1e-8 * np.max(np.abs(C)))
    # Voigt and Reuss bounds of the mean phase fractions (eqs. 3-4 applied
    # to the cell averages): the filtered field's own Voigt bound is the
    # Voigt tensor of the mean fractions, and its Reuss bound lies above
    # the Reuss tensor of the mean fractions
    fm = frac.cpu().numpy().mean(axis=1)
    f_all = np.array([1.0 - fm.sum(), fm[0], fm[1]])
    cs = [rules.iso_tensor(*p) for p in ph]
    up = rules.to_mandel(NP.voigt(f_all, cs))
    lo = rules.to_mandel(NP.reuss(f_all, cs))
    Cs = 0.5 * (C + C.T)
    assert np.min(np.linalg.eigvalsh(up - Cs)) > 0.0
    assert np.min(np.linalg.eigvalsh(Cs - lo)) > 0.0
    assert rel(o32["C"], C) < 1e-5
