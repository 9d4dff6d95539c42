"""Filtered stiffness with any number of phases (oracle; test infrastructure
only).

Section 2 writes the Voigt rule (eq. 3) as the fraction-weighted sum of the
phase stiffnesses and the Reuss rule (eq. 4) as the inverse of the
fraction-weighted sum of the phase compliances, for Nphase phases.  Here
phase 0 is the matrix and inclusion k belongs to phase labels[k] in
1..P-1.  The fraction of phase p >= 1 in the filter around a voxel is the
number of refined points inside the inclusions of phase p over M, counted
as the two-phase filter counts the inclusion set; the matrix takes
f_0 = 1 - (f_1 + ... + f_(P-1)) (summed in that order).

Readings taken where the paper is silent:
* inclusions of different phases do not overlap (a refined point inside
  two phases would count twice); inclusions of one phase may;
* a voxel whose fractions are all 0 is pure matrix, one with f_p = 1 is pure
  phase p (the phase tensor, no rule); fractional voxels need a rule;
* the reference medium is alpha times the mean of the smallest and largest
  Lame parameters over all phases;
* the 2-layer rule (eq. 5) is written for two phases and is not extended.
"""
from __future__ import annotations

import numpy as np

from . import filter as ofilter
from . import rules


def phase_counts(n, dim: int, spheres: np.ndarray, labels, n_phases: int, radius_vox: float,
                 subsamples: int, voxels: np.ndarray = None):
    """Counts (P-1, k) of refined points inside each inclusion phase, and M."""
    if voxels is None:
        voxels = ofilter.all_voxels(n)
    sph = np.asarray(spheres, dtype=np.float64).reshape(-1, 4)
    lab = np.asarray(labels, dtype=np.int64).reshape(-1)
    out = []
    M = None
    for p in range(1, n_phases):
        sel = sph[lab == p]
        if sel.shape[0] == 0:
            c = np.zeros(voxels.shape[0], dtype=np.int64)
            _, M = ofilter.counts_at(n, dim, sph[:1], radius_vox, subsamples, voxels[:1])
        else:
            c, M = ofilter.counts_at(n, dim, sel, radius_vox, subsamples, voxels)
        out.append(c)
    return np.stack(out, axis=0), M


def fractions(counts: np.ndarray, M: int, prec: str = "f64") -> np.ndarray:
    """count / M per phase as one IEEE division in float64 or float32."""
    if prec == "f32":
        return counts.astype(np.float32) / np.float32(M)
    return counts.astype(np.float64) / np.float64(M)


def matrix_fraction(fr: np.ndarray) -> np.ndarray:
    """f_0 = 1 - (f_1 + ... + f_(P-1)), summed in phase order, float64."""
    s = np.zeros(fr.shape[1:], dtype=np.float64)
    for p in range(fr.shape[0]):
        s = s + fr[p].astype(np.float64)
    return 1.0 - s


def voigt(f_all: np.ndarray, c_list) -> np.ndarray:
    """Eq. 3: sum_i f_i c_i for fractions f_all (P, ...) and phase tensors."""
    return sum(np.asarray(f_all[i])[..., None, None, None, None] * c_list[i] for i in range(len(c_list)))


def reuss(f_all: np.ndarray, c_list) -> np.ndarray:
    """Eq. 4: (sum_i f_i c_i^-1)^-1 with the inverses taken as Mandel matrices."""
    s = sum(np.asarray(f_all[i])[..., None, None] * np.linalg.inv(rules.to_mandel(c_list[i]))
            for i in range(len(c_list)))
    return rules.from_mandel(np.linalg.inv(s))


def reference_medium(phases, alpha: float = 1.0):
    lam = [p[0] for p in phases]
    mu = [p[1] for p in phases]
    return alpha * 0.5 * (min(lam) + max(lam)), alpha * 0.5 * (min(mu) + max(mu))


class NPhaseField:
    """c~ on the grid for P isotropic phases (Lame pairs) and fractions (P-1, N)."""

    def __init__(self, n, dim, phases, rule, fr):
        self.n = tuple(n)
        self.dim = dim
        fr = np.asarray(fr)
        P = len(phases)
        assert fr.shape[0] == P - 1
        c_ph = [rules.iso_tensor(*p) for p in phases]
        f0 = matrix_fraction(fr)
        f_all = np.concatenate([f0[None], fr.astype(np.float64)], axis=0)  # (P, N)
        N = f_all.shape[1]
        self.kt = np.zeros((N, 3, 3, 3, 3))
        pure = np.zeros(N, dtype=bool)
        allzero = np.all(fr == 0, axis=0)
        self.kt[allzero] = c_ph[0]
        pure |= allzero
        for p in range(1, P):
            one = (fr[p - 1] == 1) & ~pure
            self.kt[one] = c_ph[p]
            pure |= one
        mid = np.nonzero(~pure)[0]
        if mid.size:
            if rule == "voigt":
                self.kt[mid] = voigt(f_all[:, mid], c_ph)
            elif rule == "reuss":
                self.kt[mid] = reuss(f_all[:, mid], c_ph)
            else:
                raise ValueError("fractional voxels need the Voigt or Reuss rule (got %r)" % rule)
        self.mid = mid

    def apply(self, eps: np.ndarray) -> np.ndarray:
        e = eps.reshape(-1, 3, 3)
        return np.einsum("mijkl,mkl->mij", self.kt, e).reshape(eps.shape)

    def voxel_tensors(self) -> np.ndarray:
        return self.kt
