"""Pins of the filter (Section 2: uniform filter of radius given in pixel
units, phase fractions by averaging indicators on a refined grid)."""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import filter as F
from workloads import small_sphere_case, workload_c1

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "filter_small_2d.json")


def _enumerate_stencil(r, S, dim):
    # independent brute force in plain Python
    rho2 = (2 * r * S) ** 2
    lim = int(2 * r * S) + 1
    vals = [o for o in range(-lim, lim + 1) if o % 2 != 0]
    cnt = 0
    for o in itertools.product(vals, repeat=dim):
        if sum(v * v for v in o) <= rho2:
            cnt += 1
    return cnt


@pytest.mark.parametrize("r,S,dim", [(1.0, 16, 2), (0.55, 16, 2), (1.0, 8, 3), (0.5, 4, 3)])
def test_stencil_size_brute_force(r, S, dim):
    assert F.stencil_offsets(r, S, dim).shape[0] == _enumerate_stencil(r, S, dim)


def test_stencil_size_close_to_ball_volume():
    # a dense refined lattice approaches the area/volume of the ball in voxel units
    M2 = F.stencil_offsets(1.0, 64, 2).shape[0]
    assert abs(M2 / 64 ** 2 - math.pi) < 0.01
    M3 = F.stencil_offsets(1.0, 32, 3).shape[0]
    assert abs(M3 / 32 ** 3 - 4 * math.pi / 3) < 0.02


def test_golden_counts():
    g = json.load(open(GOLDEN))
    vox = F.all_voxels(g["n"])
    for case in g["cases"]:
        cnt, M = F.counts_at(g["n"], g["dim"], np.array(g["spheres"]), case["radius_vox"],
                             g["subsamples"], vox)
        assert M == case["M"]
        assert cnt.reshape(3, 3).tolist() == case["count"]


def test_pointwise_brute_force_tiny():
    # plain loops over refined points for a 5^3 cell
    w = small_sphere_case(n=(5, 5, 5), fraction=0.15, radius_vox=0.75, subsamples=2,
                          offset=(0.25, -0.125, 0.0))
    vox = F.all_voxels(w.n)
    cnt, M = F.counts_at(w.n, 3, w.spheres, w.radius_vox, w.subsamples, vox)
    S = w.subsamples
    cu = [int(round(v * 2 * S)) for v in w.spheres[0, :3]]
    R2 = (w.spheres[0, 3] * 2 * S) ** 2
    P = 2 * S * 5
    offs = [o for o in itertools.product(range(-3, 4), repeat=3)
            if all(v % 2 for v in o) and sum(v * v for v in o) <= (2 * w.radius_vox * S) ** 2]
    assert len(offs) == M
    for idx in [0, 17, 31, 62, 93, 124]:
        x, y, z = vox[idx]
        X = [(2 * x + 1) * S, (2 * y + 1) * S, (2 * z + 1) * S]
        c = 0
        for o in offs:
            d2 = 0
            for a in range(3):
                d = (X[a] + o[a] - cu[a] + P // 2) % P - P // 2
                d2 += d * d
            c += d2 <= R2
        assert c == cnt[idx]


def test_pure_voxels_away_from_interface():
    w = small_sphere_case(n=(15, 15, 15), fraction=0.2, radius_vox=1.0, subsamples=4)
    flt = F.filter_field(w)
    vox = F.all_voxels(w.n) + 0.5
    d = np.linalg.norm(vox - w.spheres[0, :3], axis=1)
    R = w.spheres[0, 3]
    far_in = d < R - 1.0 - 1e-9
    far_out = d > R + 1.0 + 1e-9
    assert np.all(flt["frac"][far_in] == 1.0)
    assert np.all(flt["frac"][far_out] == 0.0)
    mixed = (flt["count"] > 0) & (flt["count"] < flt["M"])
    assert np.all(flt["incl"][mixed] == 0) and np.all(flt["incl"][~mixed] == -1)


def test_centred_sphere_symmetry_bitwise():
    w = small_sphere_case(n=(13, 13, 13), fraction=0.2, radius_vox=1.0, subsamples=4)
    c = F.filter_field(w)["count"].reshape(13, 13, 13)
    for perm in itertools.permutations(range(3)):
        assert np.array_equal(np.transpose(c, perm), c)
    for ax in range(3):
        assert np.array_equal(np.flip(c, ax), c)


def test_shift_covariance_and_periodic_wrap():
    w = small_sphere_case(n=(11, 11, 11), fraction=0.1, radius_vox=1.0, subsamples=4)
    c = F.filter_field(w)["count"].reshape(11, 11, 11)
    ws = w.with_(spheres=w.spheres + np.array([[1.0, -2.0, 5.0, 0.0]]))
    cs = F.filter_field(ws)["count"].reshape(11, 11, 11)
    # arrays are [z][y][x]
    assert np.array_equal(np.roll(c, (5, -2, 1), axis=(0, 1, 2)), cs)


def test_no_filter_is_point_indicator():
    w = workload_c1("none")
    flt = F.filter_field(w)
    assert flt["M"] == 1
    vox = F.all_voxels(w.n) + 0.5
    d2 = np.sum((vox[:, :2] - w.spheres[0, :2]) ** 2, axis=1)
    assert np.array_equal(flt["count"], (d2 <= w.spheres[0, 3] ** 2).astype(np.int64))


def test_fraction_division_precisions():
    w = small_sphere_case(n=(9, 9, 9), radius_vox=1.0, subsamples=4)
    f64 = F.filter_field(w, "f64")
    f32 = F.filter_field(w, "f32")
    assert f32["frac"].dtype == np.float32
    assert np.array_equal(f64["count"], f32["count"])
    assert np.all(np.abs(f64["frac"] - f32["frac"]) <= 6e-8)


def test_normals_point_outward_unit():
    w = small_sphere_case(n=(15, 15, 15), fraction=0.2, radius_vox=1.0, subsamples=4)
    flt = F.filter_field(w)
    vox = F.all_voxels(w.n)
    nrm = F.interface_normals(w.n, 3, w.spheres, flt["incl"], vox)
    mixed = flt["incl"] >= 0
    d = vox[mixed] + 0.5 - w.spheres[0, :3]
    assert np.allclose(np.linalg.norm(nrm, axis=1), 1.0)
    assert np.all(np.sum(nrm[mixed] * d, axis=1) > 0)
