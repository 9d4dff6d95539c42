"""Pins of the Fourier-series extrapolation oracle (Figure 4): the Dirichlet
kernel closed form for a unit impulse, exact reproduction of trigonometric
polynomials in J at arbitrary points, interpolation of the grid values,
real values, preserved mean and whole-voxel translation covariance."""
import math

import numpy as np
import pytest

from oracle import extrapolate as X


def dirichlet(n, t):
    """(1/n) sum_{a in J} exp(2 pi i a t) = sin(pi n t) / (n sin(pi t)), 1 at integer t."""
    t = np.asarray(t, dtype=np.float64)
    s = np.sin(math.pi * t)
    out = np.ones_like(t)
    nz = np.abs(s) > 1e-15
    out[nz] = np.sin(math.pi * n * t[nz]) / (n * s[nz])
    return out


def test_unit_impulse_is_the_dirichlet_kernel():
    n = (7, 5, 3)
    f = np.zeros((n[2], n[1], n[0]))
    a0 = (4, 1, 2)  # x, y, z voxel
    f[a0[2], a0[1], a0[0]] = 1.0
    rng = np.random.default_rng(1)
    pts = rng.random((200, 3))
    got = X.evaluate(X.coefficients(f), pts)
    ref = np.ones(200)
    for d in range(3):
        ref *= dirichlet(n[d], pts[:, d] - (a0[d] + 0.5) / n[d])
    assert np.max(np.abs(got.imag)) < 1e-14
    assert np.max(np.abs(got.real - ref)) < 1e-13


def test_trigonometric_polynomials_in_J_are_reproduced_everywhere():
    n = (9, 7, 5)
    rng = np.random.default_rng(2)
    terms = [((3, -2, 1), 0.7, -0.2), ((0, 3, -2), -0.4, 0.9), ((4, 0, 0), 0.25, 0.1), ((0, 0, 0), 1.3, 0.0)]

    def poly(p):
        v = np.zeros(p.shape[0])
        for a, A, B in terms:
            ph = 2 * math.pi * (p @ np.array(a, dtype=np.float64))
            v += A * np.cos(ph) + B * np.sin(ph)
        return v
    grid = X.fine_points(n)
    f = poly(grid).reshape(n[2], n[1], n[0])
    pts = rng.random((300, 3))
    got = X.evaluate(X.coefficients(f), pts)
    assert np.max(np.abs(got.real - poly(pts))) < 1e-12
    assert np.max(np.abs(got.imag)) < 1e-12


@pytest.mark.parametrize("k", [3, 5])
def test_interpolates_grid_values_mean_and_translation(k):
    n = (7, 5, 3)
    rng = np.random.default_rng(3)
    f = rng.random((n[2], n[1], n[0]))
    m = tuple(k * v for v in n)
    F = X.extrapolate(f, m)
    c = (k - 1) // 2
    assert np.max(np.abs(F[c::k, c::k, c::k] - f)) < 1e-13  # the grid points are fine points
    assert abs(F.mean() - f.mean()) < 1e-14
    g = np.roll(f, shift=(1, 2, 3), axis=(0, 1, 2))  # whole-voxel shift (z 1, y 2, x 3)
    G = X.extrapolate(g, m)
    assert np.max(np.abs(G - np.roll(F, shift=(k, 2 * k, 3 * k), axis=(0, 1, 2)))) < 1e-13


def test_figure4_oscillations_fall_with_the_filter_radius():
    # Section 6 / Figure 4: the series of the unfiltered property oscillates
    # strongly, the 0.55-radius filter reduces the oscillations and the
    # 1.0-radius one almost removes them (Voigt-filtered C_11 of the 2D disk
    # at contrast 10^-3, 63 grid, series evaluated 3x finer)
    from oracle import filter as ofilter, rules as orules, solver as osolver
    from workloads import fig1_disk_case
    over = []
    for rule, r in (("none", 0.55), ("voigt", 0.55), ("voigt", 1.0)):
        w = fig1_disk_case(63, 1e-3, rule, r)
        ff = ofilter.filter_field(w)
        c = orules.to_mandel(osolver.StiffnessField(w.n, 2, w.phases, rule, ff["frac"]).voxel_tensors())[:, 0, 0]
        F = X.extrapolate(c.reshape(1, 63, 63), (189, 189, 1))
        over.append((F.max() - c.max()) / (c.max() - c.min()))
    assert over[0] > 2 * over[1] > 4 * over[2]
