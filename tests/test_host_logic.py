"""Host-side logic that runs without a GPU: the benchmark's byte and flop
accounting and profile-name normalisation, and the seeded workloads
(reproducible, non-overlapping inclusions, valid phase matrices)."""
import math

import numpy as np
import pytest

import bench
from workloads import cubic_mandel, iso_mandel, lame, rotation_from_seed, workload_aniso, workload_c2, workload_nphase


def test_kernel_bytes_by_hand():
    n = (125, 125, 125)
    plane = 125 * 125 * 63
    # FP32 elastic z-sweep: spectrum 6 components and 3 history components, read and written
    assert bench.kernel_bytes(n, "mixed", "zsweep") == 2 * 6 * plane * 8 + 2 * 3 * plane * 8
    # FP64 conduction x-sweep with 1000 fractional voxels: 3 components, ids, 8-real rows
    assert bench.kernel_bytes(n, "fp64", "xsweep", 1000, nc=3, nh=1) == 2 * 3 * plane * 16 + 4 * 125 ** 3 + 1000 * 64
    # anisotropic rows hold 24 reals
    assert (bench.kernel_bytes(n, "mixed", "xsweep", 10, row_reals=24) -
            bench.kernel_bytes(n, "mixed", "xsweep", 0)) == 10 * 24 * 4
    assert bench.kernel_bytes(n, "mixed", "ysweep_fwd") == 2 * 6 * plane * 8


def test_series_flops_and_profile_names():
    assert bench.series_flops((125, 125, 125), (375, 375, 375)) == 2.0 * (
        125 * 125 * 125 * 375 + 125 * 375 * 125 * 375 + 375 * 375 * 125 * 375)
    assert bench._short("void hm::k_xsweep<float, 125, 8, 256, 1, 27, false>(hm::SolveArgs)") == \
        "xsweep<float,125,8,256,1,27>"
    assert bench._short("void hm::k_xsweep<double, 125, 8, 256, 1, 9, true>(hm::SolveArgs)") == \
        "xsweep<double,125,8,256,1,9,1>"
    assert bench._short("void hm::k_zsweep<float, 125, 16, 512, 1, 2, 1>(hm::SolveArgs)") == \
        "zsweep<float,125,16,512,1,2,1>"


def _min_gap(sph, n):
    gaps = []
    for i in range(len(sph)):
        for j in range(i):
            d = sph[i, :3] - sph[j, :3]
            d -= np.asarray(n) * np.round(d / np.asarray(n))
            gaps.append(np.linalg.norm(d) - sph[i, 3] - sph[j, 3])
    return min(gaps)


def test_workloads_are_seeded_and_valid():
    a, b = workload_nphase(), workload_nphase()
    assert np.array_equal(a.spheres, b.spheres) and np.array_equal(a.meta["labels"], b.meta["labels"])
    assert _min_gap(a.spheres, a.n) >= 2.0 - 1e-9
    assert set(a.meta["labels"].tolist()) == {1, 2}
    w = workload_aniso()
    for m in w.meta["C_mandel"]:
        assert np.allclose(m, m.T) and np.linalg.eigvalsh(m).min() > 0.0
    R = rotation_from_seed(8)
    assert np.allclose(R.T @ R, np.eye(3)) and np.isclose(np.linalg.det(R), 1.0)
    # rotation leaves the cubic invariants: trace and Frobenius norm of the Mandel matrix
    c0, c1 = cubic_mandel(30.0, 12.0, 20.0), cubic_mandel(30.0, 12.0, 20.0, R)
    assert np.isclose(np.trace(c0), np.trace(c1)) and np.isclose(np.linalg.norm(c0), np.linalg.norm(c1))
    lam, mu = lame(1.0, 0.3)
    assert np.allclose(np.linalg.eigvalsh(iso_mandel(lam, mu)), sorted([2 * mu] * 5 + [3 * lam + 2 * mu]))
    c2 = workload_c2(100.0)
    assert math.isclose(4.0 / 3.0 * math.pi * c2.spheres[0, 3] ** 3 / 125 ** 3, 0.25, rel_tol=1e-6)


def test_effective_tensor_trajectory_and_iterations_to_error():
    # two load cases: the first stops after iterate 2, the second runs to 4
    nan = float("nan")
    hsig = np.full((6, 5, 6), nan)
    for J in range(6):
        last = 2 if J == 0 else 4
        for i in range(last + 1):
            hsig[J, i] = (1.0 + 0.1 * (J + 1) / (i + 1)) * np.eye(6)[J]
    traj = bench.ceff_trajectory(hsig)
    assert traj.shape == (5, 6, 6)
    # a stopped load case keeps its last column; shear columns carry sqrt(2)
    assert np.allclose(traj[4, :, 0], traj[2, :, 0])
    assert traj[4, 3, 3] == pytest.approx(np.sqrt(2.0) * (1.0 + 0.4 / 5))
    Cref = traj[-1]
    e = np.linalg.norm(traj - Cref, axis=(1, 2)) / np.linalg.norm(Cref)
    assert bench.iterations_to(traj, Cref, 0.0) == 4
    k = bench.iterations_to(traj, Cref, float(e[2]))
    assert k == 2 and np.all(e[k:] <= e[2])
    assert bench.iterations_to(traj, Cref * 2.0, 1e-3) is None


def test_floor_fraction_and_design_bytes():
    assert bench.floor_fraction(8e12 / 52.0, "mixed") == pytest.approx(1.0)
    assert bench.floor_fraction(1e10, "fp64") == pytest.approx(104.0 * 1e10 / 8e12)
    n = (125, 125, 125)
    plane = 125 * 125 * 63
    # four sweeps over the six-component half spectrum plus the history and the ids
    want = (4 * 2 * 6 * plane * 8 + 2 * 3 * plane * 8 + 4 * 125 ** 3) / 125 ** 3
    assert bench.design_bytes_per_voxel_it(n, "mixed") == pytest.approx(want)


def test_abi_argument_battery():
    """Every entry point rejects each bad argument with its code and message,
    and calls with valid arguments fail cleanly at the first device call
    when no GPU is usable (tests/host_battery.py)."""
    import os

    import host_battery

    L = host_battery.load_decls()
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libhm.so not built")
    if L.load(L.LIB_PATH).hm_device_ok():
        pytest.skip("a GPU is usable here: the battery's stand-in device pointers must not reach it")
    # on a thread of its own: the library's last-error and timing state is
    # per thread, and other tests expect this thread's to be untouched
    import threading

    res = {}
    t = threading.Thread(target=lambda: res.update(out=host_battery.run()))
    t.start()
    t.join()
    n, bad = res["out"]
    assert n > 50 and not bad, bad
