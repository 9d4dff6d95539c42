"""Pins of the oracle's transforms and frequency set (Section 2: FFT on the
truncated odd frequency set J)."""
import math

import numpy as np
import pytest

from oracle import solver


@pytest.mark.parametrize("shape", [(3, 5, 7), (9, 9, 9), (7, 9, 1)])
def test_naive_dft_equals_fft(shape):
    rng = np.random.default_rng(1)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    a = solver.naive_dft(x)
    b = np.fft.fftn(x)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_naive_dft_brute_force_single_coefficient():
    # one coefficient by the triple sum written out
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, 5, 7))
    k = (1, 3, 5)
    s = 0j
    for a in range(3):
        for b in range(5):
            for c in range(7):
                s += x[a, b, c] * np.exp(-2j * math.pi * (a * k[0] / 3 + b * k[1] / 5 + c * k[2] / 7))
    assert abs(solver.naive_dft(x)[k] - s) < 1e-12


def test_parseval_hermitian_roundtrip():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((5, 7, 9))
    X = solver.naive_dft(x)
    assert abs(np.sum(np.abs(X) ** 2) / x.size - np.sum(x ** 2)) < 1e-10
    # Hermitian symmetry of a real input: X(-k) = conj X(k)
    Xm = X[(-np.arange(5)) % 5][:, (-np.arange(7)) % 7][:, :, (-np.arange(9)) % 9]
    assert np.max(np.abs(Xm - np.conj(X))) < 1e-12
    back = solver.naive_dft(X, sign=+1) / x.size
    assert np.max(np.abs(back - x)) < 1e-13


@pytest.mark.parametrize("n", [(5, 7, 9), (81, 81, 1)])
def test_frequency_set_is_symmetric_odd_range(n):
    xi = solver.frequency_grid(n)
    for ax, m in enumerate(n):
        a = np.unique(np.round(xi[..., ax] / (2 * math.pi)).astype(int))
        assert list(a) == list(range(-(m - 1) // 2, (m - 1) // 2 + 1))


def test_even_grid_rejected():
    with pytest.raises(AssertionError):
        solver.frequency_grid((4, 5, 5))
