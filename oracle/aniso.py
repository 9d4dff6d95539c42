"""Filtered stiffness of two anisotropic phases (oracle; test infrastructure
only).

Section 2's rules are written for general phase tensors: Voigt (eq. 3) and
Reuss (eq. 4) average stiffnesses and compliances, and the 2-layer rule
(eq. 5) imposes continuous out-of-plane stress and in-plane strain across
the interface.  ``rules.voigt``, ``rules.reuss`` and ``rules.two_layer``
already take full tensors; this module supplies the phase tensors, the
reference medium and the stiffness field for anisotropic phases.

Reading where the paper is silent: the reference medium is the multiple
of the identity on symmetric tensors (lambda0 = 0) whose value 2 mu0 is
alpha times the mean of the smallest and largest eigenvalue of the phases'
Mandel matrices, so that c - c0 stays within (-c0, c0) for every phase and
the basic scheme contracts by (M - m) / (M + m).  (The mean of the Lame
parameters used for isotropic phases does not bound anisotropic ones: a
stiff shear eigenvalue can exceed 2 c0.)  ``isotropic_projection`` (the
orthogonal projection onto isotropic tensors) is kept for the pins.
"""
from __future__ import annotations

import numpy as np

from . import rules


def isotropic_projection(c: np.ndarray):
    """(lambda, mu) of the isotropic tensor nearest to c (Frobenius norm)."""
    tr1 = np.einsum("iijj->", c)
    tr2 = np.einsum("ijij->", c)
    kappa = tr1 / 9.0
    mu = (tr2 - tr1 / 3.0) / 10.0
    return kappa - 2.0 * mu / 3.0, mu


def reference_medium(c_list, alpha: float = 1.0):
    """(lambda0, mu0) = (0, alpha (m + M) / 4) from the extreme Mandel eigenvalues."""
    ev = np.concatenate([np.linalg.eigvalsh(rules.to_mandel(c)) for c in c_list])
    return 0.0, alpha * 0.25 * (ev.min() + ev.max())


class AnisoField:
    """c~ on the grid for two phase tensors (3x3x3x3): the phase tensor where
    f is 0 or 1, else the rule (the normal per voxel for the 2-layer rule)."""

    def __init__(self, n, dim, c_phases, rule, frac, normals=None):
        self.n = tuple(n)
        self.dim = dim
        self.c_ph = [np.asarray(c_phases[0], dtype=np.float64), np.asarray(c_phases[1], dtype=np.float64)]
        f = np.asarray(frac, dtype=np.float64).reshape(-1)
        self.frac = f
        self.mask0 = f == 0.0
        self.mask1 = f == 1.0
        self.mid = np.nonzero(~(self.mask0 | self.mask1))[0]
        if self.mid.size and rule == "none":
            raise ValueError("fractional voxels need a homogenisation rule")
        if self.mid.size:
            nh = None if normals is None else np.asarray(normals)[self.mid]
            if rule == "laminate" and nh is None:
                raise ValueError("the 2-layer rule needs interface normals")
            self.c_mid = rules.rule_tensor(rule, f[self.mid], nh, self.c_ph[0], self.c_ph[1])
        else:
            self.c_mid = np.zeros((0, 3, 3, 3, 3))

    def apply(self, eps: np.ndarray) -> np.ndarray:
        e = eps.reshape(-1, 3, 3)
        s = np.zeros_like(e)
        s[self.mask0] = np.einsum("ijkl,mkl->mij", self.c_ph[0], e[self.mask0])
        s[self.mask1] = np.einsum("ijkl,mkl->mij", self.c_ph[1], e[self.mask1])
        if self.mid.size:
            s[self.mid] = np.einsum("mijkl,mkl->mij", self.c_mid, e[self.mid])
        return s.reshape(eps.shape)

    def voxel_tensors(self) -> np.ndarray:
        N = self.frac.size
        c = np.zeros((N, 3, 3, 3, 3))
        c[self.mask0] = self.c_ph[0]
        c[self.mask1] = self.c_ph[1]
        c[self.mid] = self.c_mid
        return c


def cubic_tensor(c11: float, c12: float, c44: float, R=None) -> np.ndarray:
    """Cubic crystal (Voigt constants C11, C12, C44) in the cube frame, or
    with its cube axes along the columns of the rotation R."""
    m = np.zeros((6, 6))
    m[:3, :3] = c12
    for i in range(3):
        m[i, i] = c11
        m[3 + i, 3 + i] = 2.0 * c44  # Mandel shear entries carry the factor 2
    c = rules.from_mandel(m)
    if R is None:
        return c
    return np.einsum("ai,bj,ck,dl,ijkl->abcd", R, R, R, R, c)
