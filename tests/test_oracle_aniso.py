"""Pins of the anisotropic-phase oracle: the isotropic projection (identity
on isotropic tensors, the cubic closed form), the 2-layer rule of two
anisotropic layers against the Backus-type block formula in the normal
frame, Reuss <= 2-layer <= Voigt, the isotropic special case of the field,
and a cell's effective tensor within the Voigt and Reuss bounds."""
import numpy as np
import pytest

from oracle import aniso as A, filter as ofilter, rules, solver as osolver
from workloads import lame, small_sphere_case


def _rot(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    return q * np.sign(np.diag(r))[None, :]


def test_isotropic_projection():
    lam, mu = 1.7, 0.9
    assert np.allclose(A.isotropic_projection(rules.iso_tensor(lam, mu)), (lam, mu), atol=1e-14)
    c11, c12, c44 = 168.0, 121.0, 75.0  # a copper-like cubic crystal
    c = A.cubic_tensor(c11, c12, c44, _rot(3))
    l, m = A.isotropic_projection(c)
    assert np.isclose(l + 2.0 * m / 3.0, (c11 + 2.0 * c12) / 3.0)
    assert np.isclose(m, (c11 - c12 + 3.0 * c44) / 5.0)


def _block_laminate(f, n, c0, c1):
    """Continuous in-plane strain and out-of-plane stress: with the layers'
    normal-frame Mandel blocks A_PP, A_PO, A_OO,
    C_OO = S^-1, C_OP = S^-1 T, C_PP = <A_PP - A_PO A_OO^-1 A_OP> + T' S^-1 T,
    S = <A_OO^-1>, T = <A_OO^-1 A_OP>."""
    R = rules.normal_frame(n)[0]
    P, O = [0, 1, 5], [2, 3, 4]
    S = np.zeros((3, 3))
    T = np.zeros((3, 3))
    Q = np.zeros((3, 3))
    for w, c in ((1.0 - f, c0), (f, c1)):
        M = rules.to_mandel(rules.rotate(c, R[None])[0])
        iOO = np.linalg.inv(M[np.ix_(O, O)])
        S += w * iOO
        T += w * iOO @ M[np.ix_(O, P)]
        Q += w * (M[np.ix_(P, P)] - M[np.ix_(P, O)] @ iOO @ M[np.ix_(O, P)])
    Si = np.linalg.inv(S)
    C = np.zeros((6, 6))
    C[np.ix_(O, O)] = Si
    C[np.ix_(O, P)] = Si @ T
    C[np.ix_(P, O)] = T.T @ Si
    C[np.ix_(P, P)] = Q + T.T @ Si @ T
    return rules.unrotate(rules.from_mandel(C)[None], R[None])[0]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_anisotropic_laminate_block_formula_and_order(seed):
    rng = np.random.default_rng(seed)
    c0 = A.cubic_tensor(10.0, 6.0, 3.0, _rot(seed + 10))
    c1 = A.cubic_tensor(200.0, 90.0, 140.0, _rot(seed + 20))
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    f = rng.uniform(0.1, 0.9)
    L = rules.two_layer(f, n, c0, c1)
    assert np.allclose(rules.to_mandel(L), rules.to_mandel(_block_laminate(f, n, c0, c1)), atol=1e-11)
    V = rules.to_mandel(rules.voigt(f, c0, c1))
    Rr = rules.to_mandel(rules.reuss(f, c0, c1))
    Lm = rules.to_mandel(L)
    assert np.min(np.linalg.eigvalsh(V - Lm)) > -1e-10
    assert np.min(np.linalg.eigvalsh(Lm - Rr)) > -1e-10


def test_isotropic_phases_reduce_to_the_isotropic_field():
    w = small_sphere_case(n=(9, 7, 5), fraction=0.2, contrast=10.0, rule="laminate", radius_vox=1.0, subsamples=4)
    ff = ofilter.filter_field(w)
    nrm = ofilter.interface_normals(w.n, 3, w.spheres, ff["incl"], ofilter.all_voxels(w.n))
    a = A.AnisoField(w.n, 3, [rules.iso_tensor(*p) for p in w.phases], "laminate", ff["frac"], nrm)
    b = osolver.StiffnessField(w.n, 3, w.phases, "laminate", ff["frac"], nrm)
    assert np.allclose(a.voxel_tensors(), b.voxel_tensors(), atol=1e-12)
    # both reference media converge to the same effective tensor
    Ca, _ = osolver.effective_tensor(a, A.reference_medium(a.c_ph), 1e-10, 5000, 3)
    Cb, _ = osolver.effective_tensor(b, osolver.reference_medium(w.phases), 1e-10, 5000, 3)
    assert np.max(np.abs(Ca - Cb)) < 1e-8 * np.max(np.abs(Cb))


def test_reference_medium_bounds_every_phase():
    c0 = rules.iso_tensor(*lame(1.0, 0.3))
    c1 = A.cubic_tensor(30.0, 12.0, 20.0, _rot(7))
    lam0, mu0 = A.reference_medium([c0, c1])
    C0 = rules.to_mandel(rules.iso_tensor(lam0, mu0))
    for c in (c0, c1):
        ev = np.linalg.eigvalsh(np.linalg.solve(C0, rules.to_mandel(c)))
        assert ev.min() > 0.0 and ev.max() < 2.0  # c - c0 within (-c0, c0)


@pytest.mark.parametrize("rule", ["voigt", "reuss", "laminate"])
def test_cell_within_voigt_and_reuss_bounds(rule):
    w = small_sphere_case(n=(9, 9, 9), fraction=0.2, contrast=10.0, rule=rule, radius_vox=1.0, subsamples=4)
    ff = ofilter.filter_field(w)
    nrm = ofilter.interface_normals(w.n, 3, w.spheres, ff["incl"], ofilter.all_voxels(w.n))
    c0 = rules.iso_tensor(*lame(1.0, 0.3))
    c1 = A.cubic_tensor(30.0, 12.0, 20.0, _rot(7))
    fld = A.AnisoField(w.n, 3, [c0, c1], rule, ff["frac"], nrm)
    C, reps = osolver.effective_tensor(fld, A.reference_medium([c0, c1]), 1e-9, 5000, 3)
    assert all(r["status"] == 0 for r in reps)
    fm = ff["frac"].mean()
    up = rules.to_mandel(rules.voigt(fm, c0, c1))
    lo = rules.to_mandel(rules.reuss(fm, c0, c1))
    assert np.min(np.linalg.eigvalsh(up - C)) > -1e-8
    assert np.min(np.linalg.eigvalsh(C - lo)) > -1e-8
    assert np.allclose(C, C.T, atol=1e-7)
