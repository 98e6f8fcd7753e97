"""The C-ABI library on a machine without a GPU: it loads, exports every entry point that
include/hk.h declares, and rejects invalid arguments on the host before any device work."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2101_02005_amd import build
    build.build()
    import paper_2101_02005_amd as hk
    return hk.load()


def test_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "hk.h")).read()
    names = set(re.findall(r"^(?:hk_status|const char\*|int64_t)\s+(hk_\w+)\s*\(", hdr, re.M))
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n


def _grid(hk, a=0.0, d=0.1, n=100):
    return hk.grid(a, d, n)


def test_host_validation(lib):
    import paper_2101_02005_amd as hk
    sp = hk.species(18.0)
    h = ctypes.c_void_p()
    E = hk.HK_EINVAL
    assert lib.hk_prepare_lines(None, None, None, None, None, 10, ctypes.byref(sp), None, ctypes.byref(h)) == E
    fake = ctypes.c_void_p(0x1000)
    assert lib.hk_prepare_lines(fake, fake, fake, fake, fake, 0, ctypes.byref(sp), None, ctypes.byref(h)) == E
    bad_sp = hk.species(-1.0)
    assert lib.hk_prepare_lines(fake, fake, fake, fake, fake, 5, ctypes.byref(bad_sp), None, ctypes.byref(h)) == E
    assert b"species" in lib.hk_last_error()
    g = _grid(hk)
    ws = ctypes.c_void_p(0x100000)
    k = ctypes.c_void_p(0x200000)
    for T, P, grd, cut, msg in [(-1.0, 1.0, g, 25.0, b"T"), (math.nan, 1.0, g, 25.0, b"T"),
                                (1000.0, -1.0, g, 25.0, b"P"), (1000.0, 1.0, _grid(hk, d=0.0), 25.0, b"grid"),
                                (1000.0, 1.0, _grid(hk, n=0), 25.0, b"grid"), (1000.0, 1.0, g, 0.0, b"cutoff"),
                                (1000.0, 1.0, g, math.nan, b"cutoff"), (1000.0, 1.0, g, -math.inf, b"cutoff")]:
        assert lib.hk_opacity(None, None, T, P, grd, cut, k, ws, 1 << 20, None) == E
        assert msg in lib.hk_last_error(), lib.hk_last_error()
    assert lib.hk_opacity(None, None, 1000.0, 1.0, g, 25.0, k, ctypes.c_void_p(0x100010), 1 << 20, None) == E
    assert b"aligned" in lib.hk_last_error()
    assert lib.hk_opacity(None, None, 1000.0, 1.0, g, 25.0, k, ws, 1 << 20, None) == E
    assert b"handle" in lib.hk_last_error()
    Ta = (ctypes.c_double * 2)(1000.0, 800.0)
    Pa = (ctypes.c_double * 2)(1.0, 1.0)
    Ga = (hk.Grid * 2)(g, g)
    Oa = (ctypes.c_int64 * 2)(0, 50)  # overlapping outputs
    assert lib.hk_opacity_batched(None, 2, Ta, Pa, Ga, Oa, 25.0, k, ws, 1 << 20, None) == E
    assert b"overlap" in lib.hk_last_error()
    assert lib.hk_opacity_batched(None, 0, Ta, Pa, Ga, Oa, 25.0, k, ws, 1 << 20, None) == E
    assert lib.hk_release_lines(None) == hk.HK_OK


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_2101_02005_amd._lib as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        L.load()
