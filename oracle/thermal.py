"""Scalar conductivity (thermal / electrical) counterpart of the filtered
Lippmann-Schwinger fixed point (oracle; test infrastructure only).

The paper's study is elastic, but its abstract expects the filters to
help in the same way for thermal or electrical conduction.  For conduction the unknown is the gradient field g = grad T with
mean G, the flux is q = k~ g, equilibrium is div q = 0, the polarization is
tau = (k~ - k0) g with a scalar reference k0, and the Green operator is
Gamma0^(xi) = n (x) n / k0 (n = xi / |xi|):  g^(xi) = -Gamma0^ tau^ for
xi != 0 and g^(0) = N G (the counterparts of eqs. 1-2).  The filtered
conductivity of a fractional voxel follows the three rules of Section 2:
Voigt (eq. 3) k~ = <k> I, Reuss (eq. 4) k~ = <1/k>^-1 I, and the 2-layer
rule (eq. 5: continuous normal flux, continuous tangential gradient) whose
layers in parallel give k~ = <k> (I - n (x) n) + <1/k>^-1 n (x) n.  The
error of iterate i is sqrt(sum_xi |xi . q^_i|^2) / |q^_i(0)|, and the same
stop rules as the elastic solve apply (divergence judged on the residual).
Fields are arrays (nz, ny, nx, 3); 2D cells are one voxel thick.
"""
from __future__ import annotations

import math

import numpy as np

from . import solver as osolver

STATUS_CONVERGED = osolver.STATUS_CONVERGED
STATUS_NOT_CONVERGED = osolver.STATUS_NOT_CONVERGED
STATUS_STALLED = osolver.STATUS_STALLED
STATUS_DIVERGED = osolver.STATUS_DIVERGED


def reference_conductivity(k, alpha: float = 1.0) -> float:
    """k0 = alpha times the mean of the smallest and largest phase conductivity."""
    return alpha * 0.5 * (min(k) + max(k))


def rule_tensor(rule: str, f: float, nhat, k) -> np.ndarray:
    """Filtered conductivity (3x3) of a voxel with inclusion fraction f."""
    g = 1.0 - f
    arith = g * k[0] + f * k[1]
    harm = 1.0 / (g / k[0] + f / k[1])
    if rule in ("none", "voigt"):
        return arith * np.eye(3)
    if rule == "reuss":
        return harm * np.eye(3)
    if rule == "laminate":
        n = np.asarray(nhat, dtype=np.float64)
        N = np.outer(n, n)
        return arith * (np.eye(3) - N) + harm * N
    raise ValueError(rule)


class ConductivityField:
    """k~ on the grid: pure voxels carry k_p I, fractional ones the rule's tensor."""

    def __init__(self, n, dim, k, rule, frac, normals=None):
        self.n = tuple(n)
        self.dim = dim
        f = np.asarray(frac, dtype=np.float64).reshape(-1)
        self.kt = np.zeros((f.size, 3, 3))
        self.kt[f == 0.0] = k[0] * np.eye(3)
        self.kt[f == 1.0] = k[1] * np.eye(3)
        mid = np.nonzero((f > 0.0) & (f < 1.0))[0]
        if mid.size and rule == "none":
            # without a filter every voxel is pure (the indicator at its centre)
            raise ValueError("fractional voxels need a homogenisation rule")
        for v in mid:
            nh = normals[v] if normals is not None else np.array([1.0, 0.0, 0.0])
            self.kt[v] = rule_tensor(rule, f[v], nh, k)

    def apply(self, g: np.ndarray) -> np.ndarray:
        """q = k~ g for a field (nz, ny, nx, 3)."""
        return np.einsum("mij,mj->mi", self.kt, g.reshape(-1, 3)).reshape(g.shape)


def _gamma(tau_hat: np.ndarray, xi: np.ndarray, k0: float) -> np.ndarray:
    """-Gamma0^ tau^ = -n (n . tau^) / k0 at every nonzero frequency (zero frequency left at 0)."""
    x = xi.reshape(-1, 3)
    t = tau_hat.reshape(-1, 3)
    out = np.zeros_like(t)
    nz = np.any(x != 0.0, axis=1)
    q2 = np.sum(x[nz] ** 2, axis=1)
    proj = np.einsum("mi,mi->m", x[nz], t[nz]) / q2
    out[nz] = -x[nz] * proj[:, None] / k0
    return out.reshape(tau_hat.shape)


def solve(field: ConductivityField, G, k0: float, tol: float, max_iter: int):
    """Basic fixed point for a mean gradient G (3 components); returns
    dict(iters, err, status, flux_mean, errs, grad=g_{i+1})."""
    G = np.asarray(G, dtype=np.float64)
    nx, ny, nz = field.n
    N = nx * ny * nz
    xi = osolver.frequency_grid(field.n)
    g = np.broadcast_to(G, (nz, ny, nx, 3)).copy()
    errs = []
    r0 = None
    i = 0
    while True:
        q = field.apply(g)
        qh = np.fft.fftn(q, axes=(0, 1, 2))
        num = math.sqrt(float(np.sum(np.abs(np.einsum("zyxj,zyxj->zyx", xi, qh)) ** 2)))
        den = float(np.linalg.norm(qh[0, 0, 0]))
        e = num / den if den > 0 else (0.0 if num == 0.0 else math.inf)
        errs.append(e)
        if r0 is None:
            r0 = num
        status = None
        if e < tol:
            status = STATUS_CONVERGED
        elif not math.isfinite(e) or (r0 > 0 and num > osolver.DIVERGENCE_FACTOR * r0):
            status = STATUS_DIVERGED
        elif i >= max_iter:
            status = STATUS_NOT_CONVERGED
        tau = q - k0 * g
        gh = _gamma(np.fft.fftn(tau, axes=(0, 1, 2)), xi, k0)
        gh[0, 0, 0] = N * G
        g_next = np.real(np.fft.ifftn(gh, axes=(0, 1, 2)))
        if status is not None:
            return {"iters": i, "err": e, "status": status, "flux_mean": np.mean(q.reshape(-1, 3), axis=0),
                    "errs": errs, "grad": g_next}
        g = g_next
        i += 1


def effective_conductivity(field: ConductivityField, k0: float, tol: float, max_iter: int, dim: int):
    """K_eff: column J is <q> under the J-th unit mean gradient (3 in 3D, 2 in 2D)."""
    k = 2 if dim == 2 else 3
    K = np.zeros((k, k))
    reps = []
    for J in range(k):
        G = np.zeros(3)
        G[J] = 1.0
        r = solve(field, G, k0, tol, max_iter)
        K[:, J] = r["flux_mean"][:k]
        reps.append(r)
    return K, reps
