"""Filter of material properties: sub-voxel phase fractions (oracle).

Follows Section 2 of the paper: the filtered behaviour at grid point x_a is
HR(c, omega(x_a)) where omega is a uniform filter centred on x_a, acting on
the phase indicator functions to give volume fractions, which may be
estimated by averaging the indicators over a refined grid.  The numerical
setup of Section 2 fixes the filter radius in pixel units (0.5 being the
circle inscribed in a pixel) and the interface normal as the unit vector
from the inclusion centre to x_a.

Integer lattice (this reading of the refined grid):
lengths are measured in units u = h / (2 S) where h is the voxel size and S
the number of sub-samples per voxel and axis (S even).  Voxel a has its
centre at (2 a + 1) S; the refined grid is the global lattice of spacing
2u whose points sit at odd coordinates; the filter of radius r voxels keeps
the refined points at offsets o (odd integers per axis) with |o|^2 <= (2 r S)^2
(closed ball).  A refined point is inside the inclusion set when, for some
sphere k, its periodic minimum-image squared distance to the quantised
centre is <= R_k^2.  All distances are exact integers, so counts are exact.

Plain brute force: every voxel tests every stencil offset against every
sphere.  No classification shortcut.
"""
from __future__ import annotations

import numpy as np


def quantise_spheres(spheres: np.ndarray, subsamples: int):
    """Sphere table in lattice units: integer centres and squared radii.

    Centre c (voxel units) becomes round(c * 2S) (ties away from zero); the
    radius becomes t = r * 2S and the squared radius t * t, both in float64.
    """
    s2 = 2.0 * subsamples
    sph = np.asarray(spheres, dtype=np.float64).reshape(-1, 4)
    c = sph[:, :3] * s2
    cu = (np.sign(c) * np.floor(np.abs(c) + 0.5)).astype(np.int64)
    t = sph[:, 3] * s2
    return cu, t, t * t


def stencil_offsets(radius_vox: float, subsamples: int, dim: int) -> np.ndarray:
    """Offsets (odd integers, lattice units) of the refined points inside the filter ball.

    Returns an (M, 3) int64 array; the third column is 0 in 2D.
    """
    S = subsamples
    rho = radius_vox * 2.0 * S
    m = int(np.floor(rho))
    odd = np.arange(-m, m + 1, dtype=np.int64)
    odd = odd[odd % 2 != 0]
    if dim == 2:
        ox, oy = np.meshgrid(odd, odd, indexing="ij")
        o = np.stack([ox.ravel(), oy.ravel(), np.zeros(ox.size, np.int64)], axis=1)
    else:
        ox, oy, oz = np.meshgrid(odd, odd, odd, indexing="ij")
        o = np.stack([ox.ravel(), oy.ravel(), oz.ravel()], axis=1)
    d2 = np.sum(o * o, axis=1).astype(np.float64)
    keep = d2 <= rho * rho
    return o[keep]


def _min_image_int(d: np.ndarray, period: np.ndarray) -> np.ndarray:
    """Periodic minimum image of integer differences into [-P/2, P/2)."""
    return np.mod(d + period // 2, period) - period // 2


def voxel_centres_u(n, subsamples: int, voxels: np.ndarray) -> np.ndarray:
    """Lattice coordinates (2a+1)S of voxel centres for (k, 3) voxel indices (x, y, z)."""
    return (2 * np.asarray(voxels, dtype=np.int64) + 1) * subsamples


def inside_any(points_u: np.ndarray, cu: np.ndarray, R2: np.ndarray, period: np.ndarray,
               dim: int) -> np.ndarray:
    """Indicator of the inclusion set at integer points (..., 3)."""
    res = np.zeros(points_u.shape[:-1], dtype=bool)
    axes = 2 if dim == 2 else 3
    for k in range(cu.shape[0]):
        d = _min_image_int(points_u[..., :axes] - cu[k, :axes], period[:axes])
        d2 = np.sum(d * d, axis=-1).astype(np.float64)
        res |= d2 <= R2[k]
    return res


def all_voxels(n) -> np.ndarray:
    """(N, 3) voxel indices (x, y, z) in memory order z-major, x fastest."""
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def counts_at(n, dim: int, spheres: np.ndarray, radius_vox: float, subsamples: int,
              voxels: np.ndarray, chunk: int = 256):
    """Brute-force sub-sample counts for the given voxels.

    Returns (count, M).  With radius 0 (no filter) the single point is the
    voxel centre itself and M = 1.
    """
    cu, _, R2 = quantise_spheres(spheres, subsamples)
    period = 2 * subsamples * np.asarray(n, dtype=np.int64)
    X = voxel_centres_u(n, subsamples, voxels)
    if radius_vox <= 0.0:
        return inside_any(X, cu, R2, period, dim).astype(np.int64), 1
    off = stencil_offsets(radius_vox, subsamples, dim)
    M = off.shape[0]
    out = np.zeros(X.shape[0], dtype=np.int64)
    for s in range(0, X.shape[0], chunk):
        P = X[s:s + chunk, None, :] + off[None, :, :]
        out[s:s + chunk] = np.sum(inside_any(P, cu, R2, period, dim), axis=1)
    return out, M


def normal_sphere(n, dim: int, spheres: np.ndarray, subsamples: int,
                  voxels: np.ndarray) -> np.ndarray:
    """Index of the inclusion that defines the interface normal at each voxel.

    The sphere whose surface is nearest to the voxel centre,
    k = argmin_k | |d_k| - t_k | with d_k the minimum-image lattice vector
    from the quantised centre and t_k the radius in lattice units; ties go
    to the lowest index.  Where the voxel straddles one surface only this is
    the inclusion the paper's normal belongs to (pinned against per-sphere
    counts); where several surfaces are within the filter's reach the
    nearest one is a convention of this implementation (a reading, not
    pinned).
    """
    cu, t, _ = quantise_spheres(spheres, subsamples)
    period = 2 * subsamples * np.asarray(n, dtype=np.int64)
    X = voxel_centres_u(n, subsamples, voxels)
    axes = 2 if dim == 2 else 3
    best = np.full(X.shape[0], np.inf)
    arg = np.full(X.shape[0], -1, dtype=np.int64)
    for k in range(cu.shape[0]):
        d = _min_image_int(X[:, :axes] - cu[k, :axes], period[:axes])
        dist = np.abs(np.sqrt(np.sum(d * d, axis=1).astype(np.float64)) - t[k])
        better = dist < best
        best[better] = dist[better]
        arg[better] = k
    return arg


def filter_field(w, prec: str = "f64", voxels: np.ndarray = None):
    """Counts, fractions and normal-sphere ids of a workload (all voxels by default).

    Returns dict(count, frac, incl, M).  frac = count / M as one IEEE
    division in float64 (prec "f64") or float32 (prec "f32").  incl is the
    normal sphere for voxels with 0 < count < M and -1 elsewhere.
    """
    if voxels is None:
        voxels = all_voxels(w.n)
    count, M = counts_at(w.n, w.dim, w.spheres, w.radius_vox if w.rule != "none" else 0.0,
                         w.subsamples, voxels)
    if prec == "f32":
        frac = count.astype(np.float32) / np.float32(M)
    else:
        frac = count.astype(np.float64) / np.float64(M)
    incl = np.full(count.shape, -1, dtype=np.int64)
    mixed = (count > 0) & (count < M)
    if np.any(mixed):
        incl[mixed] = normal_sphere(w.n, w.dim, w.spheres, w.subsamples, voxels[mixed])
    return {"count": count, "frac": frac, "incl": incl, "M": M}


def interface_normals(n, dim: int, spheres: np.ndarray, incl: np.ndarray,
                      voxels: np.ndarray) -> np.ndarray:
    """Unit normals from the inclusion centre to the voxel centre (Section 2 setup).

    Voxel-unit coordinates: x_a = a + 0.5, d = x_a - c_k folded once into
    [-n/2, n/2) per axis; n = d / |d|, and e_1 where d = 0.  Rows with
    incl < 0 are returned as e_1 (unused).
    """
    sph = np.asarray(spheres, dtype=np.float64).reshape(-1, 4)
    nn = np.asarray(n, dtype=np.float64)
    x = np.asarray(voxels, dtype=np.float64) + 0.5
    out = np.zeros((x.shape[0], 3))
    out[:, 0] = 1.0
    sel = incl >= 0
    if not np.any(sel):
        return out
    d = x[sel] - sph[incl[sel], :3]
    for a in range(3):
        da = d[:, a]
        da = np.where(da >= nn[a] / 2.0, da - nn[a], da)
        da = np.where(da < -nn[a] / 2.0, da + nn[a], da)
        d[:, a] = da
    if dim == 2:
        d[:, 2] = 0.0
    norm = np.sqrt(np.sum(d * d, axis=1))
    nz = norm > 0
    res = np.zeros_like(d)
    res[:, 0] = 1.0
    res[nz] = d[nz] / norm[nz, None]
    out[sel] = res
    return out
