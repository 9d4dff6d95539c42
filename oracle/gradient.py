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

A second route, kept as a cross-check, differentiates the discrete
Lippmann-Schwinger equation itself (eqs. 1-a, 1-b): with C_LK = <e_L : c~ :
eps^K> and eps^K = E_K - Gamma0 * ((c~ - c0) : eps^K), the change of eps^K is
eliminated through the adjoint field w_K = g_K - (c~ - c0) : (Gamma0 * w_K),
g_K = c~ : H_K, H_K = sum_L G_LK e_L, which gives
dL/dtheta = sum_K <(H_K - Gamma0 * w_K) : dc~/dtheta : eps^K>.
"""
from __future__ import annotations

import numpy as np

from . import rules
from . import solver

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
    return _contract(field, _pair_tensor(eps_fields, np.asarray(G, dtype=np.float64)), phases, normals)


def _contract(field, P, phases, normals):
    """(1/N) sum_x P_x :: dc~(x)/dtheta for the four phase parameters and
    for the fraction of every voxel."""
    N = field.frac.size
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


def _gamma0(t, xi, lam0, mu0):
    """Gamma0 * t for a real tensor field t (zero-mean part only, eq. 2)."""
    th = np.fft.fftn(t, axes=(0, 1, 2))
    return -np.real(np.fft.ifftn(solver._apply_gamma(th, xi, lam0, mu0), axes=(0, 1, 2)))


def adjoint_gradient(field, eps_fields, G, phases, c0, normals=None, tol=1e-13, max_iter=20000):
    """dL/d(lambda_0, mu_0, lambda_1, mu_1) and dL/df(x) by the adjoint route.

    ``eps_fields`` are the converged solution fields under the unit Mandel
    strains (3D: 6, 2D: 3), ``c0`` the reference medium (lambda0, mu0) of the
    fixed point.  Each adjoint field is found by the fixed point
    w <- g - (c~ - c0) : (Gamma0 * w) from w = g, stopped when a step changes
    w by less than ``tol`` relative (the same contraction as the forward
    scheme, so it converges whenever that does).  Returns
    (dphase, dfrac, iterations per load case).
    """
    G = np.asarray(G, dtype=np.float64)
    units = solver.unit_mandel_strains(field.dim)
    n = field.n
    nx, ny, nz = n
    lam0, mu0 = c0
    C0 = rules.iso_tensor(lam0, mu0)
    xi = solver.frequency_grid(n)
    P = np.zeros((field.frac.size, 3, 3, 3, 3))
    its = []
    for K, eps in enumerate(eps_fields):
        H = sum(G[L, K] * units[L] for L in range(len(units)))
        Hf = np.broadcast_to(H, (nz, ny, nx, 3, 3)).copy()
        g = field.apply(Hf)
        w = g.copy()
        it = 0
        while True:
            u = _gamma0(w, xi, lam0, mu0)
            w_new = g - (field.apply(u) - np.einsum("ijkl,zyxkl->zyxij", C0, u))
            it += 1
            step = float(np.linalg.norm(w_new - w))
            w = w_new
            if step <= tol * float(np.linalg.norm(w)) or it >= max_iter:
                break
        its.append(it)
        v = Hf - _gamma0(w, xi, lam0, mu0)
        P += np.einsum("nij,nkl->nijkl", v.reshape(-1, 3, 3), eps.reshape(-1, 3, 3))
    dphase, dfrac = _contract(field, P, phases, normals)
    return dphase, dfrac, its
