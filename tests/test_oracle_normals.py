"""Pins of the interface normal (Section 2 numerical setup: the normal at an
interface voxel points from the inclusion centre to the voxel).

Where a voxel straddles the surface of one inclusion only, which inclusion
supplies the normal is fixed by the paper, and so is the vector: these
tests check both against geometry computed here independently of the
oracle's lattice code (nearest periodic image by enumeration, per-sphere
counts).  The choice between several surfaces within the filter's reach is
a convention of the oracle (the nearest surface) and is not tested here.
"""
import itertools

import numpy as np

from oracle import filter as F


def _fractional(n, dim, spheres, r, S):
    vox = F.all_voxels(n)
    cnt, M = F.counts_at(n, dim, spheres, r, S, vox)
    sel = (cnt > 0) & (cnt < M)
    return vox[sel]


def _nearest_image(x, c, n, dim):
    """Periodic image of centre c nearest to x, by enumerating the 27 (or 9) shifts."""
    best, arg = np.inf, None
    shifts = itertools.product((-1, 0, 1), repeat=3 if dim == 3 else 2)
    for sh in shifts:
        s = np.zeros(3)
        s[:len(sh)] = sh
        ci = c + s * np.asarray(n, dtype=np.float64)
        d = np.linalg.norm(x - ci)
        if d < best:
            best, arg = d, ci
    return arg


def test_single_inclusion_normal_is_the_outward_radial_direction_across_the_period():
    # a sphere over a corner of the cell: its interface wraps across all faces
    n, S, r = (15, 13, 11), 4, 1.0
    c = np.array([1.25, 2.5, 0.75])
    spheres = np.array([[c[0], c[1], c[2], 3.0]])
    vox = _fractional(n, 3, spheres, r, S)
    assert len(vox) > 100
    k = F.normal_sphere(n, 3, spheres, S, vox)
    assert np.all(k == 0)
    nrm = F.interface_normals(n, 3, spheres, k, vox)
    for v, nv in zip(vox, nrm):
        x = v + 0.5
        d = x - _nearest_image(x, c, n, 3)
        assert np.allclose(nv, d / np.linalg.norm(d), rtol=0, atol=1e-14)
    # voxels on opposite faces of the period see opposite normals
    assert np.any(nrm[:, 0] > 0.5) and np.any(nrm[:, 0] < -0.5)


def test_single_inclusion_normal_in_2d_lies_in_the_plane():
    n, S, r = (17, 15, 1), 8, 1.0
    c = np.array([16.5, 7.25, 0.0])
    spheres = np.array([[c[0], c[1], c[2], 4.0]])
    vox = _fractional(n, 2, spheres, r, S)
    k = F.normal_sphere(n, 2, spheres, S, vox)
    assert np.all(k == 0)
    nrm = F.interface_normals(n, 2, spheres, k, vox)
    assert np.all(nrm[:, 2] == 0.0)
    for v, nv in zip(vox, nrm):
        x = v + 0.5
        x[2] = 0.0
        d = x - _nearest_image(x, c, n, 2)
        d[2] = 0.0
        assert np.allclose(nv, d / np.linalg.norm(d), rtol=0, atol=1e-14)


def test_normal_comes_from_the_surface_the_voxel_straddles():
    """A large and a small inclusion whose surfaces are further apart than
    the filter reaches: each fractional voxel straddles exactly one surface
    (found from each sphere's own counts) and takes that inclusion's normal,
    including voxels on the large surface that lie nearer the small centre."""
    n, S, r = (25, 23, 21), 4, 1.0
    big = [8.0, 11.5, 10.25, 6.0]
    small = [18.5, 11.75, 10.5, 1.5]
    spheres = np.array([big, small])
    vox = _fractional(n, 3, spheres, r, S)
    owner = np.full(len(vox), -1)
    for k, sph in enumerate(spheres):
        cnt, M = F.counts_at(n, 3, sph[None, :], r, S, vox)
        alone = (cnt > 0) & (cnt < M)
        assert not np.any(alone & (owner >= 0)), "surfaces within the filter's reach of each other"
        owner[alone] = k
    assert np.all(owner >= 0)
    got = F.normal_sphere(n, 3, spheres, S, vox)
    assert np.array_equal(got, owner)
    # the case a nearest-centre rule would get wrong is present
    x = vox + 0.5
    d_big = np.linalg.norm(x - np.array(big[:3]), axis=1)
    d_small = np.linalg.norm(x - np.array(small[:3]), axis=1)
    assert np.any((owner == 0) & (d_small < d_big))
    # and the order of the list does not matter
    got_swapped = F.normal_sphere(n, 3, spheres[::-1], S, vox)
    assert np.array_equal(got_swapped, 1 - owner)
