"""The batched form: many (T, P) pairs and uneven grids in one persistent launch, recorded in a
hipGraph and replayed. Parity with the FP64 oracle on sampled windows, agreement with plain
calls, and bitwise-stable graph replays interleaved with eager work."""
import os

import numpy as np
import pytest

import linegen
import oracle
from gpu_util import TOL_K, rel_err

pytestmark = pytest.mark.gpu


def _prep_device(w):
    import torch

    import paper_2101_02005_amd as hk
    out = [torch.empty(w.N, dtype=torch.float64, device="cuda") for _ in range(5)]
    linegen.generate_device(w.recipe(), w.seed, w.N, [t.data_ptr() for t in out],
                            stream=torch.cuda.current_stream().cuda_stream)
    return hk.hk_prepare_lines(*out, hk.species(*w.species_tuple()))


def _pairs_subset(w):
    T, P = w.T, w.P
    sel = [(T[0], P[0]), (T[-1], P[-1]), (T[0], P[-1]), (T[-1], P[0]), (T[8], P[7]), (T[13], P[3])]
    return [t for t, _ in sel], [p for _, p in sel]


def test_batched_full_list_windows_vs_oracle():
    import paper_2101_02005_amd as hk
    w = linegen.workload("c3")
    lines = _prep_device(w)
    T, P = _pairs_subset(w)
    # uneven grids: the full range for most pairs, sub-ranges for two
    grids = [hk.grid(w.nu_start, w.dnu, w.n_grid)] * len(T)
    grids[2] = hk.grid(1000.0, w.dnu, 300_000)
    grids[5] = hk.grid(2.5, 0.013, 123_457)
    k = hk.hk_opacity_batched(lines, T, P, grids, w.cut).cpu().numpy()
    lines.release()
    sp = oracle.species(*w.species_tuple())
    rng = np.random.default_rng(30)
    off = 0
    for p, (t, pr, g) in enumerate(zip(T, P, grids)):
        kp = k[off:off + g.n]
        starts = [0, g.n - 16, int(np.argmax(kp)) - 8] + list(rng.integers(0, g.n - 16, 4))
        worst = 0.0
        for s0 in sorted(set(min(max(int(s), 0), g.n - 16) for s in starts)):
            lo = g.nu_start + s0 * g.dnu - w.cut - 0.5
            hi = g.nu_start + (s0 + 16) * g.dnu + w.cut + 0.5
            _, L = linegen.select(w.recipe(), w.seed, w.N, max(lo, 0.0), hi, cap=1 << 24)
            pts = np.arange(s0, s0 + 16)
            ko = oracle.opacity(L, sp, t, pr, g.nu_start, g.dnu, w.cut, pts)
            e = rel_err(kp[pts].astype(np.float64), ko)
            worst = max(worst, e)
            assert e <= TOL_K, (t, pr, s0, e)
        print("pair T=%.1f K P=%.3g atm grid %g+%g*[0,%d): worst window err %.3e" % (t, pr, g.nu_start, g.dnu, g.n,
                                                                                        worst))
        off += g.n


def test_batched_matches_plain_and_graph_replays():
    import torch

    import paper_2101_02005_amd as hk
    w = linegen.workload("c3", N=200_000)
    lines = _prep_device(w)
    T = [100.0, 700.0, 700.0, 3000.0]
    P = [1e-6, 0.1, 30.0, 100.0]
    grids = [hk.grid(0.0, 0.01, 500_000), hk.grid(0.0, 0.01, 500_000), hk.grid(250.0, 0.02, 77_777),
             hk.grid(0.0, 0.05, 200_000)]
    ref = hk.hk_opacity_batched(lines, T, P, grids, w.cut).clone()
    # plain calls agree within FP32 accumulation tolerance (work items may be split differently)
    off = 0
    for t, pr, g in zip(T, P, grids):
        kp = hk.hk_opacity(lines, t, pr, g, w.cut)
        a, b = kp.cpu().numpy().astype(np.float64), ref[off:off + g.n].cpu().numpy().astype(np.float64)
        assert np.max(np.abs(a - b)) <= 1e-6 * max(b.max(), 1e-300)
        off += g.n
    # graph replays with eager work and synchronizations in between: bitwise identical
    out = torch.empty_like(ref)
    for r in range(4):
        out.fill_(-1.0)
        hk.hk_opacity_batched(lines, T, P, grids, w.cut, k=out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), r
        _ = hk.hk_opacity(lines, 500.0, 1.0, hk.grid(0.0, 0.1, 10_000), w.cut)  # eager work between replays
        torch.cuda.synchronize()
    # the eager (ungraphed) batched launch gives the same bits as the graph
    os.environ["HK_GRAPH"] = "0"
    try:
        eager = hk.hk_opacity_batched(lines, T, P, grids, w.cut, k=torch.empty_like(ref))
    finally:
        del os.environ["HK_GRAPH"]
    assert torch.equal(eager, ref)
    lines.release()


def test_batched_300_pairs_windows_vs_oracle():
    """The benched form: the full 1e7-line list, all 300 (T, P) pairs in one launch, checked on 12
    pairs (the corners and pairs across the grid of T and P) x 8 windows each against the oracle."""
    import paper_2101_02005_amd as hk
    w = linegen.workload("c3")
    lines = _prep_device(w)
    T = [t for t in w.T for _ in w.P]
    P = [p for _ in w.T for p in w.P]
    n_pairs = len(T)
    assert n_pairs == 300
    grd = hk.grid(w.nu_start, w.dnu, w.n_grid)
    k = hk.hk_opacity_batched(lines, T, P, [grd] * n_pairs, w.cut)
    nT, nP = len(w.T), len(w.P)
    pick = sorted(set([0, nP - 1, (nT - 1) * nP, n_pairs - 1] +
                      [it * nP + ip for it, ip in ((2, 3), (5, 11), (8, 7), (10, 0), (12, 14), (15, 5), (17, 9),
                                                   (19, 2))]))
    assert len(pick) >= 12
    rows = k.view(n_pairs, -1)[pick].cpu().numpy()
    lines.release()
    sp = oracle.species(*w.species_tuple())
    width = 16
    fixed = [0, 100_000, 250_000, 420_000, 610_000, 800_000, w.n_grid - width]  # shared window starts
    sel_cache = {}

    def lines_for(s0):
        if s0 not in sel_cache:
            lo = w.nu_start + s0 * w.dnu - w.cut - 0.5
            hi = w.nu_start + (s0 + width) * w.dnu + w.cut + 0.5
            sel_cache[s0] = linegen.select(w.recipe(), w.seed, w.N, max(lo, 0.0), hi, cap=1 << 24)[1]
        return sel_cache[s0]

    for r, p in enumerate(pick):
        kp = rows[r].astype(np.float64)
        starts = fixed + [min(max(int(np.argmax(kp)) - width // 2, 0), w.n_grid - width)]
        worst = 0.0
        for s0 in starts:
            pts = np.arange(s0, s0 + width)
            ko = oracle.opacity(lines_for(s0), sp, T[p], P[p], w.nu_start, w.dnu, w.cut, pts)
            e = rel_err(kp[pts], ko)
            worst = max(worst, e)
            assert e <= TOL_K, (T[p], P[p], s0, e)
        print("300-pair launch, pair %d (T=%.1f K, P=%.3g atm): worst of %d windows %.3e"
              % (p, T[p], P[p], len(starts), worst))
