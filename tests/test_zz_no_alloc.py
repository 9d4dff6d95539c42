"""hm_filter_noalloc (the filter for callers that cannot allocate) against
hm_filter through the C ABI: two calls in a row on one device, the second
with a smaller grid and fewer spheres, bit-exact counts, fractions and
normal-sphere ids in both precisions; the sphere limit is refused."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_helpers import log
from workloads import rsa_spheres, small_sphere_case

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def lib():
    import paper_1412_3228_amd as hm_mod
    from paper_1412_3228_amd import _lib
    assert torch.cuda.is_available() and hm_mod.device_ok()
    return _lib.load()


def _call(lib, fn, w, prec):
    from paper_1412_3228_amd import _lib
    from paper_1412_3228_amd.api import _grid, _spheres, _stream, _ptr
    N = int(np.prod(w.n))
    count = torch.full((N,), -7, dtype=torch.int32, device=DEV)
    frac = torch.full((N,), -7.0, dtype=torch.float64 if prec == "fp64" else torch.float32, device=DEV)
    incl = torch.full((N,), -7, dtype=torch.int32, device=DEV)
    g = _grid(w.n, w.dim)
    sph, ns = _spheres(w.spheres)
    rc = getattr(lib, fn)(ctypes.byref(g), sph, ns, float(w.radius_vox), int(w.subsamples), _lib.RULES[w.rule],
                          _lib.PRECS[prec], _ptr(count), _ptr(frac), _ptr(incl), _stream(torch.device(DEV)))
    torch.cuda.synchronize()
    return rc, count.cpu().numpy(), frac.cpu().numpy(), incl.cpu().numpy()


def _cases():
    rng = np.random.Generator(np.random.PCG64(41))
    big = small_sphere_case(n=(45, 35, 27), rule="laminate", radius_vox=1.0, subsamples=8)
    big = big.with_(spheres=rsa_spheres(rng, big.n, [3.0 + 0.1 * k for k in range(20)], gap=0.5))
    small = small_sphere_case(n=(15, 21, 9), fraction=0.15, rule="laminate", radius_vox=0.55, subsamples=8,
                              offset=(0.3125, -0.25, 0.125))
    return big, small


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_filter_matches_filter_on_two_calls(lib, prec):
    for w in _cases():
        log("noalloc filter %s %s, %d spheres" % (prec, w.n, len(w.spheres)))
        rc0, c0, f0, i0 = _call(lib, "hm_filter", w, prec)
        rc1, c1, f1, i1 = _call(lib, "hm_filter_noalloc", w, prec)
        assert rc0 == 0 and rc1 == 0
        assert np.array_equal(c0, c1)
        assert np.array_equal(f0, f1)
        assert np.array_equal(i0, i1)
        assert np.any((c0 > 0) & (c0 < c0.max()))


def test_noalloc_filter_refuses_too_many_spheres(lib):
    from paper_1412_3228_amd import _lib
    w = small_sphere_case(n=(9, 9, 9), rule="voigt", radius_vox=1.0, subsamples=4)
    many = np.tile(w.spheres, (_lib.HM_FILTER_NOALLOC_MAX_SPHERES + 1, 1))
    rc, _, _, _ = _call(lib, "hm_filter_noalloc", w.with_(spheres=many), "fp64")
    assert rc == _lib.HM_E_SIZE
    assert b"at most" in lib.hm_last_error()
