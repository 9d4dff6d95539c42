"""Derivatives of the effective tensor (oracle).

Plain definition used: at the discrete solution the effective tensor is the
minimum of the strain energy over compatible fields of prescribed mean, so
by the Hill (energy) identity

    dC_KL / dtheta = (1 / N) sum_x eps^K(x) : dc~(x)/dtheta : eps^L(x)

where eps^K is the solution field under the K-th unit Mandel strain and the
derivative of c~ is taken at fixed fields.  The reference medium c0 does not
enter the discrete solution and is held fixed.  Derivatives of the
homogenisation rules (eqs. 3-5) are taken by the complex step on the rule
formulas of ``rules`` (exact to rounding, no subtraction).

For a loss L(C_eff) with G = dL/dC (Mandel), dL/dtheta = sum_KL G_KL dC_KL/dtheta.
"""
from __future__ import annotations

import numpy as np

from . import rules

H_CS = 1e-30


def _pair_tensor(eps_fields, G):
    """P_x[i,j,k,l] = sum_KL G_KL eps^K_ij(x) eps^L_kl(x), shape (N, 3, 3, 3, 3)."""
    E = np.stack([e.reshape(-1, 3, 3) for e in eps_fields], axis=0)   # (K, N, 3, 3)
    GE = np.einsum("KL,Lnkl->Knkl", G, E)
    return np.einsum("Knij,Knkl->nijkl", E, GE)


def hill_gradient(field, eps_fields, G, phases, normals=None):
    """dL/d(lambda_0, mu_0, lambda_1, mu_1) and dL/df(x) for every voxel.

    ``field`` is an oracle StiffnessField, ``eps_fields`` the K solution
    fields in the order of the unit Mandel strains, ``G`` = dL/dC (K x K).
    dL/df uses the derivative of the rule formula at the voxel's fraction and
    normal (also at pure voxels); it is zero for rule "none".
    """
    N = field.frac.size
    P = _pair_tensor(eps_fields, np.asarray(G, dtype=np.float64))
    f = field.frac
    rule = field.rule
    (l0, m0), (l1, m1) = phases
    dphase = np.zeros(4)
    params = np.array([l0, m0, l1, m1], dtype=np.float64)
    mid = field.mid
    nh = None if normals is None else np.asarray(normals)[mid]
    for q in range(4):
        pc = params.astype(np.complex128)
        pc[q] += 1j * H_CS
        c0c = rules.iso_tensor(pc[0], pc[1])
        c1c = rules.iso_tensor(pc[2], pc[3])
        d0 = np.imag(c0c) / H_CS
        d1 = np.imag(c1c) / H_CS
        tot = np.einsum("nijkl,ijkl->", P[field.mask0], d0) + np.einsum("nijkl,ijkl->", P[field.mask1], d1)
        if mid.size:
            cm = rules.rule_tensor(rule, f[mid].astype(np.complex128), nh, c0c, c1c)
            tot += np.einsum("nijkl,nijkl->", P[mid], np.imag(cm) / H_CS)
        dphase[q] = tot / N
    dfrac = np.zeros(N)
    if rule != "none":
        c0r = rules.iso_tensor(l0, m0)
        c1r = rules.iso_tensor(l1, m1)
        nall = None if normals is None else np.asarray(normals)
        cm = rules.rule_tensor(rule, f.astype(np.complex128) + 1j * H_CS, nall, c0r, c1r)
        dfrac = np.einsum("nijkl,nijkl->n", P, np.imag(cm) / H_CS) / N
    return dphase, dfrac
