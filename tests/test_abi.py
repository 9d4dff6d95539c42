"""The C-ABI library loads and exports every symbol include/hm.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for f in ("hm_filter", "hm_solve", "hm_effective_tensor", "hm_solve_adjoint"):
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_1412_3228_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libhm.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(_lib.EXPORTS)


def test_last_error_starts_empty_and_loader_reports_missing_library(tmp_path):
    from paper_1412_3228_amd import _lib
    if os.path.exists(_lib.LIB_PATH):
        lib = ctypes.CDLL(_lib.LIB_PATH)
        lib.hm_last_error.restype = ctypes.c_char_p
        assert lib.hm_last_error() == b""
    with pytest.raises(ImportError):
        _lib._lib = None
        try:
            _lib.load(str(tmp_path / "missing.so"))
        finally:
            _lib._lib = None


def test_argument_errors_without_gpu():
    """Host-side validation rejects bad grids before touching the device."""
    from paper_1412_3228_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libhm.so not built")
    lib = _lib.load()
    g = _lib.HmGrid()
    g.dim = 3
    g.n[0], g.n[1], g.n[2] = 16, 15, 15
    sph = (_lib.HmSphere * 1)()
    rc = lib.hm_filter(ctypes.byref(g), sph, 0, 1.0, 8, 1, 0, None, None, None, None)
    assert rc == _lib.HM_E_SIZE and b"odd" in lib.hm_last_error()
    for bad in (17, 143, 245):  # a prime above 13, a length with no compiled transform, beyond 243
        g.n[0] = bad
        rc = lib.hm_filter(ctypes.byref(g), sph, 0, 1.0, 8, 1, 0, None, None, None, None)
        assert rc == _lib.HM_E_SIZE and b"no compiled transform" in lib.hm_last_error()
    g.n[0] = 15
    rc = lib.hm_filter(ctypes.byref(g), sph, 0, 1.0, 7, 1, 0, None, None, None, None)
    assert rc == _lib.HM_E_ARG and b"even" in lib.hm_last_error()
    g.dim = 2
    rc = lib.hm_filter(ctypes.byref(g), sph, 0, 1.0, 8, 1, 0, None, None, None, None)
    assert rc == _lib.HM_E_ARG
