"""Pins of the oracle's Green operator (eq. 2): identities that the
periodic Green operator of an isotropic medium must satisfy."""
import numpy as np
import pytest

from oracle import rules, solver

LAM0, MU0 = 1.7, 0.9


def _xi(m=16, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, 3)) * 5.0


def _c0():
    return rules.iso_tensor(LAM0, MU0)


def test_projector_identity():
    G = solver.gamma_hat(_xi(), LAM0, MU0)
    GcG = np.einsum("mabij,ijkl,mklcd->mabcd", G, _c0(), G)
    assert np.max(np.abs(GcG - G)) < 1e-13


def test_reproduces_compatible_strains():
    xi = _xi()
    rng = np.random.default_rng(4)
    u = rng.standard_normal((xi.shape[0], 3))
    eps = 0.5 * (np.einsum("mi,mj->mij", xi, u) + np.einsum("mi,mj->mij", u, xi))
    G = solver.gamma_hat(xi, LAM0, MU0)
    out = np.einsum("mkhij,ijpq,mpq->mkh", G, _c0(), eps)
    assert np.max(np.abs(out - eps)) < 1e-12 * np.max(np.abs(eps))


def test_equilibrium_of_c0_gamma():
    xi = _xi()
    rng = np.random.default_rng(5)
    t = rng.standard_normal((xi.shape[0], 3, 3))
    tau = t + np.transpose(t, (0, 2, 1))
    G = solver.gamma_hat(xi, LAM0, MU0)
    s = np.einsum("abkh,mkhij,mij->mab", _c0(), G, tau)
    assert np.max(np.abs(np.einsum("mj,mij->mi", xi, s) - np.einsum("mj,mij->mi", xi, tau))) < 1e-11


def test_symmetries_and_homogeneity():
    xi = _xi()
    G = solver.gamma_hat(xi, LAM0, MU0)
    assert np.max(np.abs(G - np.transpose(G, (0, 3, 4, 1, 2)))) < 1e-15
    assert np.max(np.abs(G - np.transpose(G, (0, 2, 1, 3, 4)))) < 1e-15
    assert np.max(np.abs(G - np.transpose(G, (0, 1, 2, 4, 3)))) < 1e-15
    assert np.max(np.abs(solver.gamma_hat(3.7 * xi, LAM0, MU0) - G)) < 1e-15
    assert np.max(np.abs(solver.gamma_hat(-xi, LAM0, MU0) - G)) < 1e-15


def test_gamma_along_axis_closed_form():
    # for n = e1 the only nonzero entries follow from the textbook expression:
    # G_1111 = 1/(lam0+2mu0), G_1212 = 1/(4 mu0), others of type (1,2,1,2) likewise.
    G = solver.gamma_hat(np.array([[2.0, 0.0, 0.0]]), LAM0, MU0)[0]
    assert G[0, 0, 0, 0] == pytest.approx(1.0 / (LAM0 + 2 * MU0), rel=1e-14)
    assert G[0, 1, 0, 1] == pytest.approx(1.0 / (4 * MU0), rel=1e-14)
    assert G[1, 1, 1, 1] == 0.0
