"""Shared helpers of the GPU parity tests: oracle runs and field conversions."""
import math

import numpy as np

from oracle import filter as ofilter, solver as osolver

COMPS = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def oracle_fields_to_comps(eps):
    """(nz, ny, nx, 3, 3) -> (6, N) tensor components (11, 22, 33, 23, 13, 12)."""
    e = eps.reshape(-1, 3, 3)
    return np.stack([e[:, i, j] for (i, j) in COMPS], axis=0)


def oracle_solve(w, frac, incl, E, tol, max_iter, alpha=1.0, stall_window=0):
    vox = ofilter.all_voxels(w.n)
    normals = None
    if w.rule == "laminate":
        normals = ofilter.interface_normals(w.n, w.dim, w.spheres, np.asarray(incl).reshape(-1), vox)
    fld = osolver.StiffnessField(w.n, w.dim, w.phases, w.rule, np.asarray(frac, dtype=np.float64), normals)
    c0 = osolver.reference_medium(w.phases, alpha)
    return [osolver.solve(fld, e, c0, tol, max_iter, stall_window=stall_window) for e in np.asarray(E).reshape(-1, 6)]


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    s = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (s if s > 0 else 1.0))


def log(msg):
    print(msg, flush=True)


def band_oracle_filter(w, margin=2.0):
    """Oracle counts on the voxels near the single sphere's surface; pure elsewhere."""
    vox = ofilter.all_voxels(w.n)
    c = w.spheres[0, :3]
    R = w.spheres[0, 3]
    d = np.linalg.norm(vox + 0.5 - c, axis=1)
    near = np.abs(d - R) <= w.radius_vox + margin
    cnt = np.where(d < R, 1, 0).astype(np.int64)
    M = ofilter.stencil_offsets(w.radius_vox, w.subsamples, w.dim).shape[0]
    cnt *= M
    cb, M2 = ofilter.counts_at(w.n, w.dim, w.spheres, w.radius_vox, w.subsamples, vox[near])
    assert M2 == M
    cnt[near] = cb
    frac = cnt.astype(np.float64) / np.float64(M)
    incl = np.where((cnt > 0) & (cnt < M), 0, -1)
    return cnt, frac, incl, M
