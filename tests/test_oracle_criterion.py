"""Pins of the stress-equilibrium criterion's absolute scale (Section 2,
numerical setup: the criterion of the cited reference, read as the
root-mean-square divergence of the stress over the norm of its mean).

For a trigonometric polynomial stress field on the unit cell whose
frequencies lie in the grid's set J, the discrete sum over frequencies is
exact, so the criterion equals a closed form written from calculus alone:
e = sqrt(<|div sigma|^2>) / |<sigma>|_F, with <.> the cell average.  These
tests fix the 2 pi of the frequencies, the N of the unnormalised transform,
the contraction index of xi . sigma^ and the full-spectrum sum; a slip in any
of them changes e by a constant factor.
"""
import math

import numpy as np
import pytest

from oracle import filter as F, rules, solver
from workloads import lame


def _coords(n):
    """Voxel-centre coordinates (nz, ny, nx) of the unit cell, per axis."""
    nx, ny, nz = n
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    z = (np.arange(nz) + 0.5) / nz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


@pytest.mark.parametrize("n", [(9, 7, 5), (15, 9, 11), (7, 7, 1)])
def test_equilibrium_error_of_trigonometric_stress(n):
    nx, ny, nz = n
    X, Y, Z = _coords(n)
    s0 = np.array([[1.5, 0.2, -0.3], [0.2, -0.7, 0.4], [-0.3, 0.4, 0.9]])
    A, B, C = 0.37, 0.21, 0.11
    sig = np.broadcast_to(s0, (nz, ny, nx, 3, 3)).copy()
    # sigma_11 += A sin(2 pi x): (div sigma)_1 = 2 pi A cos(2 pi x)
    sig[..., 0, 0] += A * np.sin(2 * math.pi * X)
    # sigma_12 = sigma_21 += B cos(4 pi y): (div sigma)_1 += -4 pi B sin(4 pi y)
    sig[..., 0, 1] += B * np.cos(4 * math.pi * Y)
    sig[..., 1, 0] += B * np.cos(4 * math.pi * Y)
    cases = 2
    if nz >= 3:
        # sigma_33 += C sin(2 pi z) (3D only): (div sigma)_3 = 2 pi C cos(2 pi z)
        sig[..., 2, 2] += C * np.sin(2 * math.pi * Z)
        cases = 3
    # mean squares of the three mutually orthogonal divergence terms
    ms = (2 * math.pi * A) ** 2 / 2 + (4 * math.pi * B) ** 2 / 2
    if cases == 3:
        ms += (2 * math.pi * C) ** 2 / 2
    expect = math.sqrt(ms) / np.linalg.norm(s0)
    xi = solver.frequency_grid(n)
    got = solver.equilibrium_error(sig, xi)
    assert got == pytest.approx(expect, rel=1e-12)


def test_equilibrium_error_of_divergence_free_stress_is_zero():
    # sigma_12 depending on z only, sigma_11 on y only: divergence free
    n = (9, 7, 5)
    X, Y, Z = _coords(n)
    sig = np.zeros((5, 7, 9, 3, 3))
    sig[..., 0, 0] = 1.0 + 0.3 * np.sin(2 * math.pi * Y)
    sig[..., 0, 1] = sig[..., 1, 0] = 0.2 * np.cos(2 * math.pi * Z)
    assert solver.equilibrium_error(sig, solver.frequency_grid(n)) < 1e-14


@pytest.mark.parametrize("n", [(9, 7, 5), (11, 5, 1)])
def test_first_iterate_error_of_a_sinusoidal_voigt_cell(n):
    """The solver's own criterion at iterate 0 (uniform strain E), on a cell
    whose Voigt-filtered stiffness varies as a sine along x.

    With f(x) = 1/2 + a sin(2 pi x) and eq. 3, c~ = c_bar + a sin(2 pi x) dc
    (dc = c_1 - c_0), so sigma_0 = c~ : E and, for E = e_1 (x) e_1 and
    isotropic phases, (div sigma_0)_1 = 2 pi a cos(2 pi x) (d lambda + 2 d mu)
    is its only component: e_0 = sqrt(2) pi a (d lambda + 2 d mu) / |c_bar : E|.
    """
    nx, ny, nz = n
    X, _, _ = _coords(n)
    a = 0.3
    f = 0.5 + a * np.sin(2 * math.pi * X)
    assert np.all((f > 0) & (f < 1))
    ph = (lame(1.0, 0.3), lame(7.0, 0.25))
    fld = solver.StiffnessField(n, 3 if nz > 1 else 2, ph, "voigt", f.reshape(-1), None)
    E = np.zeros((3, 3))
    E[0, 0] = 1.0
    r = solver.solve(fld, E, solver.reference_medium(ph), 0.0, 0)
    dl, dm = ph[1][0] - ph[0][0], ph[1][1] - ph[0][1]
    cbar = 0.5 * (rules.iso_tensor(*ph[0]) + rules.iso_tensor(*ph[1]))
    sbar = np.einsum("ijkl,kl->ij", cbar, E)
    expect = math.sqrt(2.0) * math.pi * a * (dl + 2 * dm) / np.linalg.norm(sbar)
    assert r["errs"][0] == pytest.approx(expect, rel=1e-12)
    assert np.allclose(r["sig_mean"], sbar, rtol=0, atol=1e-14)


def test_first_iterate_error_of_a_sinusoidal_conduction_cell():
    """Conduction form of the same pin: k~ = k_bar + a sin(2 pi x) dk under a
    mean gradient G = e_1 gives div q_0 = 2 pi a dk cos(2 pi x), so
    e_0 = sqrt(2) pi a dk / k_bar."""
    from oracle import thermal as T
    n = (9, 7, 5)
    X, _, _ = _coords(n)
    a = 0.25
    f = 0.5 + a * np.sin(2 * math.pi * X)
    k = (1.0, 9.0)
    fld = T.ConductivityField(n, 3, k, "voigt", f.reshape(-1))
    r = T.solve(fld, [1.0, 0.0, 0.0], T.reference_conductivity(k), 0.0, 0)
    kbar = 0.5 * (k[0] + k[1])
    assert r["errs"][0] == pytest.approx(math.sqrt(2.0) * math.pi * a * (k[1] - k[0]) / kbar, rel=1e-12)


def test_conduction_oracle_refuses_fractional_voxels_without_a_rule():
    from oracle import thermal as T
    with pytest.raises(ValueError):
        T.ConductivityField((3, 3, 3), 3, (1.0, 2.0), "none", np.full(27, 0.5))
