"""GPU parity of the streamed form (a line list in host memory, processed in chunks whose copies
overlap the computation) against one-call results on the whole list and against the FP64
oracle, through the C ABI."""
import numpy as np
import pytest

import linegen
import oracle
from gpu_util import TOL_K, prepare, rel_err, workload_lines

pytestmark = pytest.mark.gpu

SP = (18.0, 296.0, 1.0, 0.05, 1.5)


def _host(L, order=None):
    idx = np.arange(len(L["nu"])) if order is None else order
    return [np.ascontiguousarray(L[k][idx]) for k in ("nu", "S_ref", "E", "gamma_ref", "n")]


@pytest.mark.parametrize("chunk", [10_000, 3_333, 1_000])
@pytest.mark.parametrize("sort", [False, True])
def test_stream_c1_vs_one_call_and_oracle(chunk, sort):
    import paper_2101_02005_amd as hk
    w, L = workload_lines("c1")
    g = hk.grid(0.0, 0.1, 20_000)
    order = np.argsort(L["nu"], kind="stable") if sort else None
    ks = hk.hk_opacity_stream(*_host(L, order), hk.species(*SP), 1000.0, 1.0, g, 25.0, chunk)
    ks = ks.cpu().numpy().astype(np.float64)
    lines = prepare(L, SP)
    k1 = hk.hk_opacity(lines, 1000.0, 1.0, g, 25.0).cpu().numpy().astype(np.float64)
    lines.release()
    assert np.max(np.abs(ks - k1)) <= 1e-6 * k1.max()
    ko = oracle.opacity(L, oracle.species(*SP), 1000.0, 1.0, 0.0, 0.1, 25.0, np.arange(20_000))
    assert rel_err(ks, ko) <= TOL_K
    # no line reaches a point outside the union of its cut: exact zero there too
    assert np.all(ks[ko == 0.0] == 0.0)


def test_stream_options_sorted_bands():
    """Plinth removal and Lorentz-multiple cuts through the streamed form, on a sorted list whose
    chunks each touch a narrow band of the grid."""
    import paper_2101_02005_amd as hk
    w, L = workload_lines("c1")
    order = np.argsort(L["nu"], kind="stable")
    g = hk.grid(0.0, 0.05, 40_000)
    opts = hk.options(profile=0, cut_mode=2, plinth=1)
    ks = hk.hk_opacity_stream(*_host(L, order), hk.species(*SP), 800.0, 2.0, g, 150.0, 700, opts=opts)
    ks = ks.cpu().numpy().astype(np.float64)
    sp = oracle.species(*SP)
    pts = np.arange(40_000)
    ko = oracle.opacity_ex(L, sp, 800.0, 2.0, 0.0, 0.05, 150.0, pts, cut_mode=2, plinth=True)
    scale = oracle.opacity_ex(L, sp, 800.0, 2.0, 0.0, 0.05, 150.0, pts, cut_mode=2, plinth=False).max()
    assert np.max(np.abs(ks - ko)) <= TOL_K * scale


def test_stream_large_pinned_list():
    """2e7 lines in pinned host memory, four chunks: equal to the one-call result on the device."""
    import torch

    import paper_2101_02005_amd as hk
    w = linegen.workload("c3", N=20_000_000)
    dev = [torch.empty(w.N, dtype=torch.float64, device="cuda") for _ in range(5)]
    linegen.generate_device(w.recipe(), w.seed, w.N, [t.data_ptr() for t in dev],
                            stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    host = [torch.empty(w.N, dtype=torch.float64, pin_memory=True) for _ in range(5)]
    for h, d in zip(host, dev):
        h.copy_(d)
    sp = hk.species(*w.species_tuple())
    g = hk.grid(w.nu_start, w.dnu, w.n_grid)
    lines = hk.hk_prepare_lines(*dev, sp)
    k1 = hk.hk_opacity(lines, 1200.0, 0.5, g, w.cut)
    torch.cuda.synchronize()
    lines.release()
    del dev
    ks = hk.hk_opacity_stream(*host, sp, 1200.0, 0.5, g, w.cut, 5_000_000)
    torch.cuda.synchronize()
    d = (ks.double() - k1.double()).abs().max().item()
    assert d <= 1e-6 * k1.double().max().item()


def test_stream_invalid_chunk():
    import paper_2101_02005_amd as hk
    w, L = workload_lines("c1")
    arrs = _host(L)
    arrs[0][7_777] = -1.0  # nu <= 0 in the fourth chunk
    k = None
    with pytest.raises(hk.HkError) as ei:
        k = hk.hk_opacity_stream(*arrs, hk.species(*SP), 1000.0, 1.0, hk.grid(0.0, 0.1, 20_000), 25.0, 2_500)
    assert ei.value.status == hk.HK_EINVAL
    assert k is None
