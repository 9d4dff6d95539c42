"""Truncated Fourier series of a grid field evaluated off the grid (oracle;
test infrastructure only).

The conclusion (Section 6, Figure 4) looks at the filtered material
properties through their extrapolation: the truncated Fourier series whose
coefficients are the FFT of the field c~(x_alpha) on the grid, evaluated
anywhere in the cell.  With the grid points at the voxel centres
x = (alpha + 1/2) / n of the unit cell and the odd frequency set J of
Section 2, the series is

    F(y) = sum_{a in J} c^(a) exp(2 pi i a . y),
    c^(a) = (1/N) sum_x c(x) exp(-2 pi i a . x),

real because J is symmetric, and equal to c at the grid points.  Off-grid
evaluation points are the voxel centres (beta + 1/2) / m of a finer grid.
Fields are arrays (nz, ny, nx).
"""
from __future__ import annotations

import math

import numpy as np


def _freqs(n: int) -> np.ndarray:
    assert n % 2 == 1, "the truncated frequency set J needs odd grids"
    h = (n - 1) // 2
    return np.arange(-h, h + 1, dtype=np.float64)


def coefficients(field: np.ndarray):
    """c^(a) for a in J (axes ordered z, y, x, each -h..h) from numpy's FFT
    of the grid values, with the phase of the half-voxel offset of the
    grid points."""
    nz, ny, nx = field.shape
    F = np.fft.fftn(np.asarray(field, dtype=np.float64)) / field.size
    F = np.fft.fftshift(F)  # frequencies -h..h on every axis (odd n)
    for ax, n in zip((0, 1, 2), (nz, ny, nx)):
        a = _freqs(n)
        shape = [1, 1, 1]
        shape[ax] = n
        F = F * np.exp(-1j * math.pi * a / n).reshape(shape)
    return F


def evaluate(coefs: np.ndarray, points: np.ndarray) -> np.ndarray:
    """F at cell points (k, 3) given as (x, y, z) in [0, 1): the explicit
    sum over J; returns the complex values (the imaginary part is rounding)."""
    nz, ny, nx = coefs.shape
    ax, ay, az = _freqs(nx), _freqs(ny), _freqs(nz)
    Z, Y, X = np.meshgrid(az, ay, ax, indexing="ij")
    a = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)  # (N, 3)
    c = coefs.ravel()
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.empty(pts.shape[0], dtype=np.complex128)
    step = max(1, 4_000_000 // a.shape[0])
    for s in range(0, pts.shape[0], step):
        ph = np.exp(2j * math.pi * (pts[s:s + step] @ a.T))
        out[s:s + step] = ph @ c
    return out


def fine_points(m) -> np.ndarray:
    """Voxel centres of an (mx, my, mz) grid as (x, y, z), x fastest."""
    mx, my, mz = m
    gz, gy, gx = np.meshgrid((np.arange(mz) + 0.5) / mz, (np.arange(my) + 0.5) / my,
                             (np.arange(mx) + 0.5) / mx, indexing="ij")
    return np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)


def extrapolate(field: np.ndarray, m) -> np.ndarray:
    """The series of `field` on the voxel centres of the m grid, (mz, my, mx), real part."""
    vals = evaluate(coefficients(field), fine_points(m))
    mx, my, mz = m
    return vals.real.reshape(mz, my, mx)
