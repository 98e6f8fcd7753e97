"""Error paths of the C ABI on a device: a workspace smaller than the call's plan needs, or
misaligned, is rejected with HK_EINVAL before anything is launched (k keeps the caller's values);
a batched call with one bad pair launches nothing either."""
import ctypes

import numpy as np
import pytest

from gpu_util import prepare, workload_lines

pytestmark = pytest.mark.gpu

SP = (18.0, 296.0, 1.0, 0.05, 1.5)


def _call(hk, lines, grd, k, ws_ptr, ws_bytes, opts=None):
    lib = hk._lib.load()
    if opts is None:
        return lib.hk_opacity(ctypes.c_void_p(lines.handle), None, 1000.0, 1.0, grd, 25.0, hk._lib._ptr(k),
                              ctypes.c_void_p(ws_ptr), ws_bytes, None)
    return lib.hk_opacity_ex(ctypes.c_void_p(lines.handle), None, 1000.0, 1.0, grd, 25.0, hk._lib._opts(opts),
                             hk._lib._ptr(k), ctypes.c_void_p(ws_ptr), ws_bytes, None)


@pytest.mark.parametrize("opts", [None, {"profile": 1, "plinth": 1}])
def test_workspace_too_small_or_misaligned(opts):
    import torch

    import paper_2101_02005_amd as hk
    w, L = workload_lines("c1")
    lines = prepare(L, SP)
    grd = hk.grid(0.0, 0.1, 20_000)
    o = None if opts is None else hk.options(**opts)
    if o is None:
        need = hk.hk_workspace_size(lines, 0, [grd], 25.0)
    else:
        need = hk.hk_workspace_size_ex(lines, 0, [1000.0], [1.0], [grd], 25.0, o)
    ws = hk._lib._workspace(need + 512)
    base = hk._lib._aligned(ws)
    k = torch.full((grd.n,), 7.0, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    # hk_workspace_size covers every tuning the library may pick; a call checks the size its own
    # tuning needs, so a few KB is short of it whatever the tuning
    st = _call(hk, lines, grd, k, base, 4096, o)
    assert st == hk.HK_EINVAL, hk._lib.load().hk_last_error()
    assert b"too small" in hk._lib.load().hk_last_error()
    st = _call(hk, lines, grd, k, base + 8, need, o)  # not 256-byte aligned
    assert st == hk.HK_EINVAL
    torch.cuda.synchronize()
    assert bool((k == 7.0).all())  # nothing was launched
    st = _call(hk, lines, grd, k, base, need, o)  # the size it asked for
    assert st == hk.HK_OK, hk._lib.load().hk_last_error()
    torch.cuda.synchronize()
    assert np.isfinite(k.cpu().numpy()).all() and float(k.max()) > 0.0 and not bool((k == 7.0).any())
    lines.release()


def test_batched_bad_pair_launches_nothing():
    import torch

    import paper_2101_02005_amd as hk
    w, L = workload_lines("c1")
    lines = prepare(L, SP)
    grids = [hk.grid(0.0, 0.1, 20_000)] * 3
    k = torch.full((60_000,), 7.0, dtype=torch.float32, device="cuda")
    with pytest.raises(hk.HkError) as ei:
        hk.hk_opacity_batched(lines, [800.0, -1.0, 1200.0], [1.0, 1.0, 1.0], grids, 25.0, k=k)  # T < 0
    assert ei.value.status == hk.HK_EINVAL
    torch.cuda.synchronize()
    assert bool((k == 7.0).all())
    lines.release()
