"""Lippmann-Schwinger fixed point with the filtered stiffness (oracle).

Follows Section 2 of the paper: the periodic cell loaded by a macroscopic
strain E satisfies eps = -Gamma0 * tau + E with tau = (c - c0) : eps
(eq. 1-a, 1-b); in Fourier space eps^(k) = -Gamma0^(k) : tau^(k) for k != 0
and eps^(0) = E (eq. 2); on an odd grid the frequencies are the integer
set J = prod_d {-(N_d-1)/2 .. (N_d-1)/2}.  The polarization is evaluated at
the grid points with the filtered stiffness c~ in place of c.

Readings taken where the paper is silent:
* grid points are voxel centres, the cell is [0,1)^d, frequencies
  xi = 2 pi a for a in J; 2D is plane strain (a 3D cell one voxel thick);
* the reference medium is the mean of the phases' smallest and largest
  Lame parameters, times alpha (Section 5 / Figure 3 caption);
* the stress-equilibrium error of iterate i is
  e_i = sqrt(sum_xi |xi . sigma^_i(xi)|^2) / |sigma^_i(0)|_F
  with the unnormalised DFT (the Moulinec-Suquet criterion);
* the reported mean stress is that of the iterate whose error passed; the
  returned strain field is the one produced by the update from it.

Storage: fields are arrays (nz, ny, nx, 3, 3) of full symmetric tensors.
FFTs are numpy's (a library step); ``naive_dft`` is the O(N^2) definition.
"""
from __future__ import annotations

import math

import numpy as np

from . import filter as ofilter
from . import rules

STATUS_CONVERGED = 0
STATUS_NOT_CONVERGED = 1
STATUS_STALLED = 2
STATUS_DIVERGED = 3

DIVERGENCE_FACTOR = 1.0e3
STALL_DECREASE = 0.99


def reference_medium(phases, alpha: float = 1.0):
    """(lambda0, mu0) = alpha * mean of the phases' smallest and largest Lame parameters."""
    lams = [p[0] for p in phases]
    mus = [p[1] for p in phases]
    return alpha * 0.5 * (min(lams) + max(lams)), alpha * 0.5 * (min(mus) + max(mus))


def naive_dft(x: np.ndarray, axes=(0, 1, 2), sign: int = -1) -> np.ndarray:
    """Unnormalised multidimensional DFT by its definition, one axis at a time.

    X[k] = sum_j x[j] exp(sign 2 pi i j k / n) along each of the given axes.
    """
    out = np.asarray(x, dtype=np.complex128)
    for ax in axes:
        n = out.shape[ax]
        j = np.arange(n)
        W = np.exp(sign * 2j * math.pi * np.outer(j, j) / n)
        out = np.moveaxis(np.tensordot(W, np.moveaxis(out, ax, 0), axes=(1, 0)), 0, ax)
    return out


def frequency_grid(n) -> np.ndarray:
    """xi = 2 pi a on the integer set J, shape (nz, ny, nx, 3) as (xi_x, xi_y, xi_z)."""
    nx, ny, nz = n
    ax = [np.round(np.fft.fftfreq(m, d=1.0 / m)) for m in (nx, ny, nz)]
    for m, a in zip((nx, ny, nz), ax):
        assert m % 2 == 1, "the truncated frequency set J needs odd grids"
        assert a.max() == (m - 1) // 2
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return 2.0 * math.pi * np.stack([X, Y, Z], axis=-1)


def gamma_hat(xi: np.ndarray, lam0: float, mu0: float) -> np.ndarray:
    """Green operator of the isotropic medium (lam0, mu0) at frequencies xi (m, 3) != 0.

    Gamma_khij = (d_ki n_h n_j + d_hi n_k n_j + d_kj n_h n_i + d_hj n_k n_i) / (4 mu0)
                 - (lam0 + mu0) / (mu0 (lam0 + 2 mu0)) n_i n_j n_k n_h,   n = xi / |xi|.
    """
    nv = xi / np.linalg.norm(xi, axis=1, keepdims=True)
    d = np.eye(3)
    t = (np.einsum("ki,mh,mj->mkhij", d, nv, nv)
         + np.einsum("hi,mk,mj->mkhij", d, nv, nv)
         + np.einsum("kj,mh,mi->mkhij", d, nv, nv)
         + np.einsum("hj,mk,mi->mkhij", d, nv, nv)) / (4.0 * mu0)
    t -= (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0)) * np.einsum("mi,mj,mk,mh->mkhij", nv, nv, nv, nv)
    return t


class StiffnessField:
    """The filtered stiffness c~ on the grid.

    Pure voxels (fraction exactly 0 or 1) carry the phase tensor; every other
    voxel carries the rule's tensor for its fraction and interface normal.
    """

    def __init__(self, n, dim, phases, rule, frac, normals=None):
        self.n = tuple(n)
        self.dim = dim
        self.rule = rule
        self.c_ph = [rules.iso_tensor(*phases[0]), rules.iso_tensor(*phases[1])]
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
        """sigma = c~ : eps for a field (nz, ny, nx, 3, 3)."""
        e = eps.reshape(-1, 3, 3)
        s = np.zeros_like(e)
        s[self.mask0] = np.einsum("ijkl,mkl->mij", self.c_ph[0], e[self.mask0])
        s[self.mask1] = np.einsum("ijkl,mkl->mij", self.c_ph[1], e[self.mask1])
        if self.mid.size:
            s[self.mid] = np.einsum("mijkl,mkl->mij", self.c_mid, e[self.mid])
        return s.reshape(eps.shape)

    def voxel_tensors(self) -> np.ndarray:
        """(N, 3, 3, 3, 3) tensors of every voxel (small grids only)."""
        N = self.frac.size
        c = np.zeros((N, 3, 3, 3, 3))
        c[self.mask0] = self.c_ph[0]
        c[self.mask1] = self.c_ph[1]
        c[self.mid] = self.c_mid
        return c


def build_field(w, frac=None, incl=None):
    """Stiffness field of a workload: filter (unless frac is given), normals, rule."""
    vox = ofilter.all_voxels(w.n)
    if frac is None:
        flt = ofilter.filter_field(w, "f64", vox)
        frac, incl = flt["frac"], flt["incl"]
    frac = np.asarray(frac).reshape(-1)
    normals = None
    if w.rule == "laminate":
        if incl is None:
            incl = np.full(frac.shape, -1, dtype=np.int64)
        normals = ofilter.interface_normals(w.n, w.dim, w.spheres, np.asarray(incl).reshape(-1), vox)
    return StiffnessField(w.n, w.dim, w.phases, w.rule, frac, normals)


def strain_tensor(comp6) -> np.ndarray:
    """Tensor components (11, 22, 33, 23, 13, 12) -> symmetric 3x3."""
    a11, a22, a33, a23, a13, a12 = [float(v) for v in comp6]
    return np.array([[a11, a12, a13], [a12, a22, a23], [a13, a23, a33]])


def _apply_gamma(tau_hat, xi, lam0, mu0, chunk=65536):
    """eps^ = -Gamma0^ : tau^ at every nonzero frequency (zero frequency left at 0)."""
    sh = tau_hat.shape
    t = tau_hat.reshape(-1, 3, 3)
    x = xi.reshape(-1, 3)
    out = np.zeros_like(t)
    nz = np.nonzero(np.any(x != 0.0, axis=1))[0]
    for s in range(0, nz.size, chunk):
        idx = nz[s:s + chunk]
        G = gamma_hat(x[idx], lam0, mu0)
        out[idx] = -np.einsum("mkhij,mij->mkh", G, t[idx])
    return out.reshape(sh)


def equilibrium_error(sig: np.ndarray, xi: np.ndarray) -> float:
    """sqrt(sum_xi |xi . sigma^(xi)|^2) / |sigma^(0)|_F with the unnormalised DFT."""
    sh = np.fft.fftn(sig, axes=(0, 1, 2))
    div = np.einsum("zyxj,zyxij->zyxi", xi, sh)
    num = math.sqrt(float(np.sum(np.abs(div) ** 2)))
    den = float(np.sqrt(np.sum(np.abs(sh[0, 0, 0]) ** 2)))
    return num / den if den > 0 else (0.0 if num == 0.0 else math.inf)


def solve(field: StiffnessField, E, c0, tol: float, max_iter: int,
          stall_window: int = 0, eps0=None, dft=None):
    """Basic fixed-point scheme for one macroscopic strain E (3x3 or 6 components).

    Iterate i computes sigma_i = c~ : eps_i and its error e_i = r_i / |<sigma_i>|
    with the equilibrium residual r_i = sqrt(sum_xi |xi . sigma^_i|^2); it
    stops when e_i < tol (converged), when e_i is not finite or r_i exceeds
    1e3 r_0 (diverged: the residual, not e_i, because the mean stress of an
    iterate can pass close to zero at high contrast and make e_i spike while
    the iteration converges), when with stall_window > 0 the error has not dropped by 1%
    below its last reference value for stall_window iterations (stalled),
    or when i == max_iter (not converged).  Otherwise
    tau_i = sigma_i - c0 : eps_i, eps^_{i+1} = -Gamma0^ : tau^_i (xi != 0),
    eps^_{i+1}(0) = N E, eps_{i+1} = real inverse DFT.

    Returns dict(iters=i, err=e_i, status, sig_mean=<sigma_i> (3x3),
    errs=[e_0..e_i], eps=eps_{i+1}).
    """
    E = np.asarray(E, dtype=np.float64)
    if E.shape != (3, 3):
        E = strain_tensor(E)
    n = field.n
    nx, ny, nz = n
    N = nx * ny * nz
    lam0, mu0 = c0
    C0 = rules.iso_tensor(lam0, mu0)
    xi = frequency_grid(n)
    fwd = (lambda a: np.fft.fftn(a, axes=(0, 1, 2))) if dft is None else dft[0]
    inv = (lambda a: np.fft.ifftn(a, axes=(0, 1, 2))) if dft is None else dft[1]
    if eps0 is None:
        eps = np.broadcast_to(E, (nz, ny, nx, 3, 3)).copy()
    else:
        eps = np.array(eps0, dtype=np.float64)
    errs = []
    r0 = None
    ref, iref = None, 0
    i = 0
    while True:
        sig = field.apply(eps)
        sh = fwd(sig)
        div = np.einsum("zyxj,zyxij->zyxi", xi, sh)
        num = math.sqrt(float(np.sum(np.abs(div) ** 2)))
        den = float(np.sqrt(np.sum(np.abs(sh[0, 0, 0]) ** 2)))
        e = num / den if den > 0 else (0.0 if num == 0.0 else math.inf)
        errs.append(e)
        if r0 is None:
            r0 = num
        status = None
        if e < tol:
            status = STATUS_CONVERGED
        elif not math.isfinite(e) or (r0 > 0 and num > DIVERGENCE_FACTOR * r0):
            status = STATUS_DIVERGED
        else:
            if ref is None or e < STALL_DECREASE * ref:
                ref, iref = e, i
            if stall_window > 0 and i - iref >= stall_window:
                status = STATUS_STALLED
            elif i >= max_iter:
                status = STATUS_NOT_CONVERGED
        tau = sig - np.einsum("ijkl,zyxkl->zyxij", C0, eps)
        tau_hat = fwd(tau)
        eps_hat = _apply_gamma(tau_hat, xi, lam0, mu0)
        eps_hat[0, 0, 0] = N * E
        eps_next = np.real(inv(eps_hat))
        if status is not None:
            return {"iters": i, "err": e, "status": status,
                    "sig_mean": np.mean(sig.reshape(-1, 3, 3), axis=0),
                    "errs": errs, "eps": eps_next}
        eps = eps_next
        i += 1


def project_compatible(t: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """G t: orthogonal projection (sum over voxels of u : v) of a real
    symmetric tensor field onto compatible strain fields of zero mean.  It
    is Gamma0 of the reference medium lambda0 = 0, mu0 = 1/2 (c0 = identity
    on symmetric tensors), applied at every nonzero frequency (eq. 2)."""
    th = np.fft.fftn(t, axes=(0, 1, 2))
    return np.real(np.fft.ifftn(-_apply_gamma(th, xi, 0.0, 0.5), axes=(0, 1, 2)))


def field_dot(u: np.ndarray, v: np.ndarray) -> float:
    """sum over voxels of u : v for (nz, ny, nx, 3, 3) fields."""
    return float(np.sum(u * v))


def solve_cg(field: StiffnessField, E, tol: float, max_iter: int, keep_residuals: bool = False):
    """Conjugate gradients on the same Lippmann-Schwinger operator (the Krylov
    alternative named in Section 5).

    With c0 = identity, the strain eps = E + x whose stress is in
    equilibrium satisfies G(c~ : x) = -G(c~ : E) with x compatible and of
    zero mean, where G is project_compatible; G c~ G is symmetric positive
    definite for sum_v u : v on that space, so plain CG applies:
    x_0 = 0, r_0 = p_0 = -G(c~ : E); q = G(c~ : p), alpha = (r.r)/(p.q),
    x += alpha p, r -= alpha q, beta = (r.r)_new/(r.r), p = r + beta p.
    Iterate k (k operator applications after the start) has the error
    e_k = sqrt(<r_k : r_k>) / |<sigma_k>| (r = -G sigma_k, the compatible part
    of the stress, vanishes at equilibrium; <.> voxel mean, Frobenius norm);
    the solve stops when e_k < tol or k == max_iter.

    Returns dict(iters=k, err=e_k, status, sig_mean=<sigma_k> (3x3),
    errs=[e_0..e_k], eps=E + x_k) and, with keep_residuals, the r_k fields.
    """
    E = np.asarray(E, dtype=np.float64)
    if E.shape != (3, 3):
        E = strain_tensor(E)
    nx, ny, nz = field.n
    N = nx * ny * nz
    xi = frequency_grid(field.n)
    Eb = np.broadcast_to(E, (nz, ny, nx, 3, 3))
    x = np.zeros((nz, ny, nx, 3, 3))
    r = -project_compatible(field.apply(Eb), xi)
    p = r.copy()
    rr = field_dot(r, r)
    errs, rs = [], []
    k = 0
    while True:
        if keep_residuals:
            rs.append(r.copy())
        sig_mean = np.mean(field.apply(Eb + x).reshape(-1, 3, 3), axis=0)
        fro = float(np.sqrt(np.sum(sig_mean * sig_mean)))
        e = math.sqrt(rr / N) / fro if fro > 0 else (0.0 if rr == 0.0 else math.inf)
        errs.append(e)
        status = None
        if e < tol:
            status = STATUS_CONVERGED
        elif k >= max_iter:
            status = STATUS_NOT_CONVERGED
        if status is not None:
            out = {"iters": k, "err": e, "status": status, "sig_mean": sig_mean, "errs": errs, "eps": Eb + x}
            if keep_residuals:
                out["residuals"] = rs
            return out
        q = project_compatible(field.apply(p), xi)
        alpha = rr / field_dot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = field_dot(r, r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        k += 1


def unit_mandel_strains(dim: int):
    """Unit Mandel strains as 3x3 tensors: 6 in 3D, the 3 in-plane ones (11, 22, 12) in 2D."""
    s = 1.0 / math.sqrt(2.0)
    out = []
    for (i, j) in rules.MANDEL:
        E = np.zeros((3, 3))
        if i == j:
            E[i, i] = 1.0
        else:
            E[i, j] = E[j, i] = s
        out.append(E)
    if dim == 2:
        return [out[0], out[1], out[5]]
    return out


def mandel_vector(t: np.ndarray, dim: int) -> np.ndarray:
    """Mandel components of a symmetric tensor (the in-plane three in 2D)."""
    v = np.array([t[i, j] * (1.0 if i == j else math.sqrt(2.0)) for (i, j) in rules.MANDEL])
    return v[[0, 1, 5]] if dim == 2 else v


def effective_tensor(field: StiffnessField, c0, tol: float, max_iter: int, dim: int,
                     keep_fields: bool = False, stall_window: int = 0):
    """C_eff in Mandel form: column J is Mandel(<sigma>) under the J-th unit Mandel strain."""
    loads = unit_mandel_strains(dim)
    k = len(loads)
    C = np.zeros((k, k))
    reps = []
    for J, E in enumerate(loads):
        r = solve(field, E, c0, tol, max_iter, stall_window=stall_window)
        C[:, J] = mandel_vector(r["sig_mean"], dim)
        if not keep_fields:
            r = dict(r)
            r.pop("eps")
        reps.append(r)
    return C, reps
