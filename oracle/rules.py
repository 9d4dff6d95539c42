"""Homogenisation rules of the filter (oracle).

Section 2 of the paper: the filtered stiffness c~(x_a) = HR(c, omega(x_a))
uses the phase volume fractions in the filter and one of three rules:
Voigt (eq. 3, fraction-weighted mean of stiffnesses), Reuss (eq. 4, inverse
of the fraction-weighted mean of compliances) and the 2-layer rule (eq. 5:
a two-phase laminate whose interface is the local planar approximation,
with continuous out-of-plane stress and in-plane strain across it and
fraction-weighted averages of the other parts).

Reading of eq. 5-b (its printed form repeats f_1): the averages are
f_1 s_1^P + f_2 s_2^P = s^P and f_1 e_1^OP + f_2 e_2^OP = e^OP.

Tensors are full 3x3x3x3 arrays c[..., i, j, k, l] (a leading batch axis is
allowed everywhere); Mandel 6x6 forms use the order (11, 22, 33, 23, 13, 12)
with sqrt(2) on the shear rows/columns.  Phase 0 is the matrix, phase 1 the
inclusion; f is the inclusion fraction.  All functions accept complex
inputs so that derivatives can be taken by the complex step.
"""
from __future__ import annotations

import math

import numpy as np

MANDEL = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))
_W = np.array([1.0, 1.0, 1.0, math.sqrt(2.0), math.sqrt(2.0), math.sqrt(2.0)])


def iso_tensor(lam, mu) -> np.ndarray:
    """c_ijkl = lam d_ij d_kl + mu (d_ik d_jl + d_il d_jk)."""
    d = np.eye(3)
    return (lam * np.einsum("ij,kl->ijkl", d, d)
            + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def to_mandel(c: np.ndarray) -> np.ndarray:
    """(..., 3, 3, 3, 3) -> (..., 6, 6)."""
    m = np.zeros(c.shape[:-4] + (6, 6), dtype=c.dtype)
    for A, (i, j) in enumerate(MANDEL):
        for B, (k, l) in enumerate(MANDEL):
            m[..., A, B] = _W[A] * _W[B] * c[..., i, j, k, l]
    return m


def from_mandel(m: np.ndarray) -> np.ndarray:
    """(..., 6, 6) -> (..., 3, 3, 3, 3) with both minor symmetries."""
    c = np.zeros(m.shape[:-2] + (3, 3, 3, 3), dtype=m.dtype)
    for A, (i, j) in enumerate(MANDEL):
        for B, (k, l) in enumerate(MANDEL):
            v = m[..., A, B] / (_W[A] * _W[B])
            for (p, q) in {(i, j), (j, i)}:
                for (r, s) in {(k, l), (l, k)}:
                    c[..., p, q, r, s] = v
    return c


def rotate(c: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Components in the frame whose basis vectors are the columns of R.

    c'_abcd = R_ia R_jb R_kc R_ld c_ijkl  (R may carry a leading batch axis).
    """
    if R.ndim == 2:
        return np.einsum("ia,jb,kc,ld,ijkl->abcd", R, R, R, R, c, optimize=True)
    cb = np.broadcast_to(c, R.shape[:-2] + (3, 3, 3, 3))
    return np.einsum("mia,mjb,mkc,mld,mijkl->mabcd", R, R, R, R, cb, optimize=True)


def unrotate(cp: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Inverse of rotate: c_ijkl = R_ia R_jb R_kc R_ld c'_abcd."""
    if R.ndim == 2:
        return np.einsum("ia,jb,kc,ld,abcd->ijkl", R, R, R, R, cp, optimize=True)
    return np.einsum("mia,mjb,mkc,mld,mabcd->mijkl", R, R, R, R, cp, optimize=True)


def _fr(f):
    f = np.asarray(f)
    return f[..., None, None, None, None]


def voigt(f, c0: np.ndarray, c1: np.ndarray) -> np.ndarray:
    """Eq. 3: fraction-weighted mean of the phase stiffnesses."""
    return (1.0 - _fr(f)) * c0 + _fr(f) * c1


def reuss(f, c0: np.ndarray, c1: np.ndarray) -> np.ndarray:
    """Eq. 4: inverse of the fraction-weighted mean of the phase compliances (Mandel inverse)."""
    f = np.asarray(f)[..., None, None]
    s = (1.0 - f) * np.linalg.inv(to_mandel(c0)) + f * np.linalg.inv(to_mandel(c1))
    return from_mandel(np.linalg.inv(s))


def normal_frame(nhat: np.ndarray) -> np.ndarray:
    """Orthonormal frames (t1, t2, n) as columns, n being the unit normal; batched over rows."""
    n = np.atleast_2d(np.asarray(nhat, dtype=np.float64))
    n = n / np.linalg.norm(n, axis=1, keepdims=True)
    e = np.where((np.abs(n[:, 0]) < 0.9)[:, None], np.array([1.0, 0.0, 0.0]),
                 np.array([0.0, 1.0, 0.0]))
    t1 = e - np.sum(e * n, axis=1, keepdims=True) * n
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(n, t1)
    return np.stack([t1, t2, n], axis=2)


# In the normal frame (n along the third axis), Mandel indices of the
# in-plane ("P": 11, 22, 12) and out-of-plane ("OP": 33, 23, 13) parts.
_P = [0, 1, 5]
_OP = [2, 3, 4]


def two_layer(f, nhat: np.ndarray, c0: np.ndarray, c1: np.ndarray) -> np.ndarray:
    """Eq. 5: stiffness of a two-phase laminate with interface normal nhat.

    Batched over a leading axis of f (m,) and nhat (m, 3); a scalar f and a
    single normal give one tensor.  In the frame of the normal, for each
    unit macroscopic Mandel strain, solves the six linear conditions for the
    out-of-plane strains of the two layers: equal out-of-plane stress in
    both layers, and the fraction-weighted mean of their out-of-plane
    strains equal to the macroscopic one (both layers carry the macroscopic
    in-plane strain).  The macroscopic stress is the fraction-weighted mean
    of the in-plane stresses together with the common out-of-plane stress.
    """
    scalar = np.ndim(f) == 0
    fv = np.atleast_1d(np.asarray(f))
    R = normal_frame(nhat)
    if R.shape[0] == 1 and fv.shape[0] > 1:
        R = np.broadcast_to(R, (fv.shape[0], 3, 3))
    A = to_mandel(rotate(c0, R))   # layer 1: matrix, fraction 1 - f
    B = to_mandel(rotate(c1, R))   # layer 2: inclusion, fraction f
    f1 = (1.0 - fv)[:, None, None]
    f2 = fv[:, None, None]
    m = fv.shape[0]
    dt = np.result_type(A, fv)
    eye3 = np.eye(3)
    # unknowns x = [e1_OP (3), e2_OP (3)] for each of the 6 unit strains
    K = np.zeros((m, 6, 6), dtype=dt)
    K[:, 0:3, 0:3] = A[:, _OP][:, :, _OP]
    K[:, 0:3, 3:6] = -B[:, _OP][:, :, _OP]
    K[:, 3:6, 0:3] = f1 * eye3
    K[:, 3:6, 3:6] = f2 * eye3
    Eu = np.eye(6)
    eP = Eu[_P, :]     # (3, 6): in-plane part of each unit strain (columns)
    eOP = Eu[_OP, :]
    rhs = np.zeros((m, 6, 6), dtype=dt)
    rhs[:, 0:3, :] = -(A[:, _OP][:, :, _P] - B[:, _OP][:, :, _P]) @ eP
    rhs[:, 3:6, :] = eOP
    x = np.linalg.solve(K, rhs)            # (m, 6 unknowns, 6 loads)
    e1 = np.zeros((m, 6, 6), dtype=dt)
    e2 = np.zeros((m, 6, 6), dtype=dt)
    e1[:, _P, :] = eP
    e2[:, _P, :] = eP
    e1[:, _OP, :] = x[:, 0:3, :]
    e2[:, _OP, :] = x[:, 3:6, :]
    s1 = A @ e1
    s2 = B @ e2
    Cl = np.zeros((m, 6, 6), dtype=dt)
    Cl[:, _P, :] = f1 * s1[:, _P, :] + f2 * s2[:, _P, :]
    Cl[:, _OP, :] = s1[:, _OP, :]
    out = unrotate(from_mandel(Cl), R)
    return out[0] if scalar else out


def rule_tensor(rule: str, f, nhat, c0: np.ndarray, c1: np.ndarray) -> np.ndarray:
    """The rule's formula (no pure-phase shortcut), batched; used for values and derivatives."""
    if rule == "voigt":
        return voigt(f, c0, c1)
    if rule == "reuss":
        return reuss(f, c0, c1)
    if rule == "laminate":
        return two_layer(f, nhat, c0, c1)
    raise ValueError("rule %r has no formula" % rule)


def filtered_stiffness(rule: str, f, nhat, c0: np.ndarray, c1: np.ndarray) -> np.ndarray:
    """c~ at one voxel: the pure phase tensor when f is exactly 0 or 1, else the rule."""
    if f == 0.0:
        return c0.copy()
    if f == 1.0:
        return c1.copy()
    if rule == "none":
        raise ValueError("rule 'none' needs a pure voxel (f in {0, 1})")
    return rule_tensor(rule, f, nhat, c0, c1)
