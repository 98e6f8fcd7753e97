"""The allocation-free entry point (hk_opacity_noalloc) against hk_opacity, called through the C
ABI: two calls in a row, the second on a smaller input, each bitwise equal to hk_opacity on the
same input (the same kernels and tuning); and a problem beyond the scratch array's size rejected
with HK_ENOMEM before any launch, its output untouched."""
import ctypes

import pytest

from gpu_util import prepare, workload_lines

pytestmark = pytest.mark.gpu


def _noalloc(lib, lines, T, P, g, cut, k):
    import torch
    return lib.hk_opacity_noalloc(ctypes.c_void_p(lines.handle), None, float(T), float(P), g, float(cut),
                                  ctypes.c_void_p(k.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_noalloc_matches_workspace_entry_point():
    import torch

    import linegen
    import paper_2101_02005_amd as hk
    lib = hk.load()
    assert hk.hk_noalloc_max_bytes() == 64 << 20
    for N, n, dnu, T, P in ((10_000, 20_000, 0.1, 1000.0, 1.0), (3_000, 5_001, 0.37, 400.0, 0.2)):
        w, L = workload_lines("c1", N=N)
        lines = prepare(L, w.species_tuple())
        g = hk.grid(0.0, dnu, n)
        ref = hk.hk_opacity(lines, T, P, g, 25.0)
        k = torch.full((n,), -1.0, dtype=torch.float32, device="cuda")
        st = _noalloc(lib, lines, T, P, g, 25.0, k)
        assert st == hk.HK_OK, lib.hk_last_error()
        torch.cuda.synchronize()
        assert torch.equal(k, ref), (N, n)
        lines.release()
    # beyond the scratch array: HK_ENOMEM, nothing launched
    w = linegen.workload("c3", N=4_000_000)
    dev = [torch.empty(w.N, dtype=torch.float64, device="cuda") for _ in range(5)]
    linegen.generate_device(w.recipe(), w.seed, w.N, [t.data_ptr() for t in dev],
                            stream=torch.cuda.current_stream().cuda_stream)
    lines = hk.hk_prepare_lines(*dev, hk.species(*w.species_tuple()))
    k = torch.full((w.n_grid,), -1.0, dtype=torch.float32, device="cuda")
    st = _noalloc(lib, lines, 800.0, 0.1, hk.grid(w.nu_start, w.dnu, w.n_grid), w.cut, k)
    assert st == hk.HK_ENOMEM, lib.hk_last_error()
    torch.cuda.synchronize()
    assert bool((k == -1.0).all())
    lines.release()
