"""Pins of the N-phase oracle (eqs. 3-4 for any number of phases):
isotropic closed forms, the two-phase special case, merging identical
phases, Reuss <= Voigt, per-phase counts against the two-phase filter, and
the effective tensor of a three-phase cell within the Voigt and Reuss
bounds of its phase fractions."""
import numpy as np
import pytest

from oracle import filter as ofilter, nphase as NP, rules, solver as osolver
from workloads import lame

PH3 = [lame(1.0, 0.3), lame(12.0, 0.25), lame(0.2, 0.35)]


def _kmu(c):
    m = rules.to_mandel(c)
    mu = m[3, 3] / 2.0
    lam = m[0, 1]
    return lam + 2.0 * mu / 3.0, mu


def test_isotropic_closed_forms():
    f = np.array([0.5, 0.3, 0.2])
    cs = [rules.iso_tensor(*p) for p in PH3]
    V = NP.voigt(f, cs)
    lam = sum(fi * p[0] for fi, p in zip(f, PH3))
    mu = sum(fi * p[1] for fi, p in zip(f, PH3))
    assert np.allclose(V, rules.iso_tensor(lam, mu), atol=1e-13)
    R = NP.reuss(f, cs)
    K = 1.0 / sum(fi / (p[0] + 2.0 * p[1] / 3.0) for fi, p in zip(f, PH3))
    mu_r = 1.0 / sum(fi / p[1] for fi, p in zip(f, PH3))
    assert np.allclose(R, rules.iso_tensor(K - 2.0 * mu_r / 3.0, mu_r), atol=1e-13)


def test_two_phases_reduce_to_the_two_phase_rules():
    c0, c1 = rules.iso_tensor(*PH3[0]), rules.iso_tensor(*PH3[1])
    for f in (0.1, 0.5, 0.93):
        fa = np.array([1.0 - f, f])
        assert np.allclose(NP.voigt(fa, [c0, c1]), rules.voigt(f, c0, c1), atol=1e-13)
        assert np.allclose(NP.reuss(fa, [c0, c1]), rules.reuss(f, c0, c1), atol=1e-12)


def test_merging_identical_phases_and_order():
    cs = [rules.iso_tensor(*p) for p in PH3]
    f = np.array([0.4, 0.35, 0.25])
    cs4 = cs + [cs[1]]
    f4 = np.array([0.4, 0.2, 0.25, 0.15])  # phase 1 split over two identical phases
    for rule in (NP.voigt, NP.reuss):
        assert np.allclose(rule(f, cs), rule(f4, cs4), atol=1e-12)
    d = rules.to_mandel(NP.voigt(f, cs)) - rules.to_mandel(NP.reuss(f, cs))
    assert np.min(np.linalg.eigvalsh(d)) > 0.0


def _three_phase_cell(n=(9, 9, 9)):
    sph = np.array([[2.5, 2.5, 2.5, 1.7], [6.5, 6.0, 6.5, 2.1], [6.5, 2.5, 2.0, 1.4], [2.0, 6.5, 6.5, 1.5]])
    labels = np.array([1, 1, 2, 2])
    return n, sph, labels


def test_phase_counts_partition_the_two_phase_count():
    n, sph, labels = _three_phase_cell()
    cnt, M = NP.phase_counts(n, 3, sph, labels, 3, 1.0, 4)
    union, M2 = ofilter.counts_at(n, 3, sph, 1.0, 4, ofilter.all_voxels(n))
    assert M == M2
    assert np.array_equal(cnt.sum(axis=0), union)  # disjoint phases
    assert np.all(cnt <= M)
    one, _ = NP.phase_counts(n, 3, sph, np.ones(4, dtype=int), 2, 1.0, 4)
    assert np.array_equal(one[0], union)


@pytest.mark.parametrize("rule", ["voigt", "reuss"])
def test_three_phase_cell_within_the_global_bounds(rule):
    n, sph, labels = _three_phase_cell()
    cnt, M = NP.phase_counts(n, 3, sph, labels, 3, 1.0, 4)
    fr = NP.fractions(cnt, M)
    fld = NP.NPhaseField(n, 3, PH3, rule, fr)
    C, reps = osolver.effective_tensor(fld, NP.reference_medium(PH3), 1e-9, 5000, 3)
    assert all(r["status"] == 0 for r in reps)
    f_all = np.concatenate([NP.matrix_fraction(fr)[None], fr], axis=0).mean(axis=1)
    cs = [rules.iso_tensor(*p) for p in PH3]
    up = rules.to_mandel(NP.voigt(f_all, cs))
    lo = rules.to_mandel(NP.reuss(f_all, cs))
    assert np.min(np.linalg.eigvalsh(up - C)) > -1e-8
    assert np.min(np.linalg.eigvalsh(C - lo)) > -1e-8
    assert np.allclose(C, C.T, atol=1e-7)


def test_pure_and_fractional_voxels():
    fr = np.array([[0.0, 1.0, 0.0, 0.25], [0.0, 0.0, 1.0, 0.5]])
    fld = NP.NPhaseField((4, 1, 1), 3, PH3, "voigt", fr)
    cs = [rules.iso_tensor(*p) for p in PH3]
    assert np.array_equal(fld.kt[0], cs[0]) and np.array_equal(fld.kt[1], cs[1]) and np.array_equal(fld.kt[2], cs[2])
    assert np.allclose(fld.kt[3], 0.25 * cs[0] + 0.25 * cs[1] + 0.5 * cs[2], atol=1e-13)
    with pytest.raises(ValueError):
        NP.NPhaseField((4, 1, 1), 3, PH3, "none", fr)
