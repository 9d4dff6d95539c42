"""Pins of the oracle gradient: the Hill identity against central finite
differences of the effective tensor."""
import numpy as np
import pytest

from oracle import filter as F, gradient, solver
from workloads import small_sphere_case


def test_hill_gradient_matches_central_fd():
    w = small_sphere_case(n=(7, 7, 7), fraction=0.2, contrast=5.0, rule="laminate",
                          radius_vox=1.0, subsamples=4)
    flt = F.filter_field(w)
    vox = F.all_voxels(w.n)
    nrm = F.interface_normals(w.n, 3, w.spheres, flt["incl"], vox)
    c0 = solver.reference_medium(w.phases)
    fld = solver.StiffnessField(w.n, 3, w.phases, "laminate", flt["frac"], nrm)
    C, reps = solver.effective_tensor(fld, c0, 1e-12, 5000, 3, keep_fields=True)
    G = np.random.default_rng(0).standard_normal((6, 6))
    dph, dfr = gradient.hill_gradient(fld, [r["eps"] for r in reps], G, w.phases, nrm)

    def loss(ph, frac):
        f2 = solver.StiffnessField(w.n, 3, ph, "laminate", frac, nrm)
        C2, _ = solver.effective_tensor(f2, c0, 1e-12, 5000, 3)
        return float(np.sum(G * C2))

    h = 1e-5
    for q in range(4):
        pp = [list(p) for p in w.phases]
        pm = [list(p) for p in w.phases]
        pp[q // 2][q % 2] += h
        pm[q // 2][q % 2] -= h
        fd = (loss(pp, flt["frac"]) - loss(pm, flt["frac"])) / (2 * h)
        assert abs(fd - dph[q]) < 1e-6 * max(1.0, abs(fd))
    mid = np.nonzero((flt["count"] > 0) & (flt["count"] < flt["M"]))[0]
    for v in mid[[0, len(mid) // 2, -1]]:
        fp = flt["frac"].copy()
        fm = fp.copy()
        fp[v] += h
        fm[v] -= h
        fd = (loss(w.phases, fp) - loss(w.phases, fm)) / (2 * h)
        assert abs(fd - dfr[v]) < 1e-6 * max(1e-3, abs(fd))


@pytest.mark.parametrize("rule,n,dim", [("laminate", (7, 7, 7), 3), ("reuss", (9, 7, 5), 3),
                                        ("voigt", (11, 9, 1), 2)])
def test_adjoint_route_equals_hill_identity(rule, n, dim):
    """The Hill pairing of the solution fields against the adjoint route,
    which differentiates the Lippmann-Schwinger equation (eqs. 1-a, 1-b)
    through its own fixed point and pairs each field with an adjoint field
    instead of with the other load cases' fields; G is not symmetric."""
    w = small_sphere_case(n=n, dim=dim, fraction=0.2, contrast=5.0, rule=rule, radius_vox=1.0, subsamples=4,
                          offset=(0.25, -0.5, 0.0 if dim == 2 else 0.75))
    flt = F.filter_field(w)
    nrm = F.interface_normals(w.n, dim, w.spheres, flt["incl"], F.all_voxels(w.n)) if rule == "laminate" else None
    c0 = solver.reference_medium(w.phases)
    fld = solver.StiffnessField(w.n, dim, w.phases, rule, flt["frac"], nrm)
    C, reps = solver.effective_tensor(fld, c0, 1e-13, 20000, dim, keep_fields=True)
    k = C.shape[0]
    G = np.random.default_rng(3).standard_normal((k, k))
    eps = [r["eps"] for r in reps]
    dh, fh = gradient.hill_gradient(fld, eps, G, w.phases, nrm)
    da, fa, its = gradient.adjoint_gradient(fld, eps, G, w.phases, c0, nrm)
    assert max(its) < 20000
    assert np.max(np.abs(da - dh)) <= 1e-9 * np.max(np.abs(dh))
    assert np.max(np.abs(fa - fh)) <= 1e-9 * np.max(np.abs(fh))
    assert np.max(np.abs(fh)) > 0
