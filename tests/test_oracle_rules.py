"""Pins of the homogenisation rules (Section 2, eqs. 3-5) against textbook
closed forms, bounds and invariances."""
import math

import numpy as np
import pytest

from oracle import rules
from workloads import lame

PH0 = lame(1.0, 0.3)
PH1 = lame(20.0, 0.3)
C0 = rules.iso_tensor(*PH0)
C1 = rules.iso_tensor(*PH1)


def _rand_normal(seed):
    v = np.random.default_rng(seed).standard_normal(3)
    return v / np.linalg.norm(v)


def test_lame_from_young_poisson():
    # uniaxial stress: the compliance gives 1/E on the axis and -nu/E across
    E, nu = 3.5, 0.27
    S = np.linalg.inv(rules.to_mandel(rules.iso_tensor(*lame(E, nu))))
    assert S[0, 0] == pytest.approx(1.0 / E, rel=1e-13)
    assert S[0, 1] == pytest.approx(-nu / E, rel=1e-13)


def test_mandel_roundtrip():
    m = np.random.default_rng(0).standard_normal((6, 6))
    m = m + m.T
    assert np.max(np.abs(rules.to_mandel(rules.from_mandel(m)) - m)) < 1e-15


@pytest.mark.parametrize("f", [0.1, 0.5, 0.83])
def test_voigt_reuss_isotropic_closed_forms(f):
    (l0, m0), (l1, m1) = PH0, PH1
    v = rules.voigt(f, C0, C1)
    assert np.max(np.abs(v - rules.iso_tensor((1 - f) * l0 + f * l1, (1 - f) * m0 + f * m1))) < 1e-13
    K0, K1 = l0 + 2 * m0 / 3, l1 + 2 * m1 / 3
    K = 1.0 / ((1 - f) / K0 + f / K1)
    mu = 1.0 / ((1 - f) / m0 + f / m1)
    r = rules.reuss(f, C0, C1)
    assert np.max(np.abs(r - rules.iso_tensor(K - 2 * mu / 3, mu))) < 1e-12


@pytest.mark.parametrize("f", [0.2, 0.64])
def test_laminate_textbook_coefficients_normal_e3(f):
    # Layered isotropic media (Backus averages): with M = lam + 2 mu,
    # C3333 = <1/M>^-1, C1133 = C3333 <lam/M>, C2323 = <1/mu>^-1, C1212 = <mu>,
    # C1111 = <M - lam^2/M> + C3333 <lam/M>^2, C1122 = <lam - lam^2/M> + C3333 <lam/M>^2.
    (l0, m0), (l1, m1) = PH0, PH1
    w = np.array([1 - f, f])
    lam = np.array([l0, l1])
    mu = np.array([m0, m1])
    M = lam + 2 * mu
    avg = lambda a: float(np.sum(w * a))
    c33 = 1.0 / avg(1.0 / M)
    c = rules.two_layer(f, np.array([0.0, 0.0, 1.0]), C0, C1)
    assert c[2, 2, 2, 2] == pytest.approx(c33, rel=1e-13)
    assert c[0, 0, 2, 2] == pytest.approx(c33 * avg(lam / M), rel=1e-13)
    assert c[1, 2, 1, 2] == pytest.approx(1.0 / avg(1.0 / mu), rel=1e-13)
    assert c[0, 1, 0, 1] == pytest.approx(avg(mu), rel=1e-13)
    assert c[0, 0, 0, 0] == pytest.approx(avg(M - lam ** 2 / M) + c33 * avg(lam / M) ** 2, rel=1e-13)
    assert c[0, 0, 1, 1] == pytest.approx(avg(lam - lam ** 2 / M) + c33 * avg(lam / M) ** 2, rel=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_laminate_equal_shear_is_hill_isotropic(seed):
    # Hill: phases with equal shear modulus give an isotropic composite with
    # mu_eff = mu and 1/(K_eff + 4mu/3) = <1/(K + 4mu/3)>, for any geometry.
    mu = 0.8
    la, lb = 0.5, 7.0
    f = 0.37
    ca, cb = rules.iso_tensor(la, mu), rules.iso_tensor(lb, mu)
    Ka, Kb = la + 2 * mu / 3, lb + 2 * mu / 3
    Keff = 1.0 / ((1 - f) / (Ka + 4 * mu / 3) + f / (Kb + 4 * mu / 3)) - 4 * mu / 3
    c = rules.two_layer(f, _rand_normal(seed), ca, cb)
    assert np.max(np.abs(c - rules.iso_tensor(Keff - 2 * mu / 3, mu))) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_reuss_le_laminate_le_voigt(seed):
    rng = np.random.default_rng(seed)
    f = float(rng.uniform(0.05, 0.95))
    nh = _rand_normal(seed + 10)
    v = rules.to_mandel(rules.voigt(f, C0, C1))
    r = rules.to_mandel(rules.reuss(f, C0, C1))
    l = rules.to_mandel(rules.two_layer(f, nh, C0, C1))
    assert np.min(np.linalg.eigvalsh(v - l)) > -1e-12
    assert np.min(np.linalg.eigvalsh(l - r)) > -1e-12


@pytest.mark.parametrize("rule", ["voigt", "reuss", "laminate"])
def test_formula_endpoints_and_equal_phases(rule):
    nh = _rand_normal(7)
    for f, ref in [(0.0, C0), (1.0, C1)]:
        c = rules.rule_tensor(rule, f, nh, C0, C1)
        assert np.max(np.abs(c - ref)) < 1e-12 * np.max(np.abs(C1))
    c = rules.rule_tensor(rule, 0.42, nh, C1, C1)
    assert np.max(np.abs(c - C1)) < 1e-12 * np.max(np.abs(C1))


def test_laminate_rotation_covariance():
    rng = np.random.default_rng(11)
    nh = _rand_normal(12)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    f = 0.3
    a = rules.two_layer(f, q @ nh, C0, C1)
    b = rules.two_layer(f, nh, C0, C1)
    rb = np.einsum("ia,jb,kc,ld,abcd->ijkl", q, q, q, q, b)
    assert np.max(np.abs(a - rb)) < 1e-12 * np.max(np.abs(b))


def test_laminate_batched_equals_scalar():
    rng = np.random.default_rng(13)
    f = rng.uniform(0, 1, 5)
    nh = rng.standard_normal((5, 3))
    nh /= np.linalg.norm(nh, axis=1, keepdims=True)
    b = rules.two_layer(f, nh, C0, C1)
    for i in range(5):
        assert np.max(np.abs(b[i] - rules.two_layer(float(f[i]), nh[i], C0, C1))) < 1e-14


def test_filtered_stiffness_pure_shortcut():
    assert np.array_equal(rules.filtered_stiffness("reuss", 1.0, None, C0, C1), C1)
    assert np.array_equal(rules.filtered_stiffness("laminate", 0.0, None, C0, C1), C0)
    with pytest.raises(ValueError):
        rules.filtered_stiffness("none", 0.5, None, C0, C1)
