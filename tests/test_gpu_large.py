"""GPU parity at the full sizes of the large workloads, on sampled windows the FP64 oracle
computes point by point (the whole grids are far beyond the oracle), plus the uncut
precision workload with its error reported per wavenumber decade."""
import numpy as np
import pytest

import linegen
import oracle
from gpu_util import TOL_K, rel_err

pytestmark = pytest.mark.gpu


def _device_lines(w):
    import torch
    out = [torch.empty(w.N, dtype=torch.float64, device="cuda") for _ in range(5)]
    linegen.generate_device(w.recipe(), w.seed, w.N, [t.data_ptr() for t in out],
                            stream=torch.cuda.current_stream().cuda_stream)
    return out


def _progress(capsys, msg):
    """The test's own per-window results, written as they come (not held by output capture): a
    window of the densest band takes the oracle tens of seconds."""
    with capsys.disabled():
        print(msg, flush=True)


def _windows(w, k, rng, n_rand, width):
    """Window starts: the low-wavenumber edge, the densest band, the largest k, random ones, the end."""
    n = w.n_grid
    starts = [0, int(round((100.0 - w.nu_start) / w.dnu)), int(np.argmax(k)) - width // 2, n - width]
    starts += list(rng.integers(0, n - width, n_rand))
    return sorted(set(int(min(max(s, 0), n - width)) for s in starts))


@pytest.mark.parametrize("cut,dnu,direct", [(25.0, 0.01, 0), (100.0, 0.01, 0), (25.0, 0.1, 0), (100.0, 0.1, 0),
                                             (25.0, 0.1, 1)])
def test_large_list_windows(cut, dnu, direct, capsys):
    """The full 5e8-line list at both resolutions and both cutting lengths; direct = 1: every
    (line, point) pair evaluated (no Chebyshev-node classes)."""
    import torch

    import paper_2101_02005_amd as hk
    w = linegen.workload("c2", cut=cut, dnu=dnu)
    dev = _device_lines(w)
    lines = hk.hk_prepare_lines(*dev, hk.species(*w.species_tuple()))
    del dev
    k = hk.hk_opacity(lines, w.T[0], w.P[0], hk.grid(w.nu_start, w.dnu, w.n_grid), w.cut,
                      opts=hk.options(direct=1) if direct else None).cpu().numpy()
    lines.release()
    torch.cuda.empty_cache()
    rng = np.random.default_rng(20 + int(cut) + int(100 * dnu))
    width = 24
    sp = oracle.species(*w.species_tuple())
    worst = 0.0
    for s0 in _windows(w, k, rng, 12 if cut < 50 else 6, width):
        lo = w.nu_start + s0 * w.dnu - w.cut - 0.5
        hi = w.nu_start + (s0 + width) * w.dnu + w.cut + 0.5
        _, L = linegen.select(w.recipe(), w.seed, w.N, max(lo, 0.0), hi, cap=1 << 26)
        pts = np.arange(s0, s0 + width)
        ko = oracle.opacity(L, sp, w.T[0], w.P[0], w.nu_start, w.dnu, w.cut, pts)
        e = rel_err(k[pts].astype(np.float64), ko)
        worst = max(worst, e)
        _progress(capsys, "c2 cut %g dnu %g direct %d window @%d (%.2f cm^-1): %d lines, max rel err %.3e"
                  % (cut, dnu, direct, s0, w.nu_start + s0 * w.dnu, len(L["nu"]), e))
        assert e <= TOL_K
    _progress(capsys, "c2 cut %g dnu %g direct %d: worst window %.3e" % (cut, dnu, direct, worst))


def test_uncut_precision_per_decade():
    import paper_2101_02005_amd as hk
    w = linegen.workload("c5")
    L = linegen.generate(w.recipe(), w.seed, w.N)
    from gpu_util import prepare
    lines = prepare(L, w.species_tuple())
    k = hk.hk_opacity(lines, w.T[0], w.P[0], hk.grid(w.nu_start, w.dnu, w.n_grid), w.cut).cpu().numpy()
    lines.release()
    sp = oracle.species(*w.species_tuple())
    rng = np.random.default_rng(50)
    width = 16
    for dec_lo, dec_hi in ((1000.0, 10000.0), (10000.0, 100000.0)):
        j_lo = int(round((dec_lo - w.nu_start) / w.dnu))
        j_hi = int(round((dec_hi - w.nu_start) / w.dnu)) - width
        starts = list(rng.integers(j_lo, j_hi, 9)) + [j_lo + int(np.argmax(k[j_lo:j_hi]))]
        pts = np.concatenate([np.arange(s, s + width) for s in starts])
        ko = oracle.opacity(L, sp, w.T[0], w.P[0], w.nu_start, w.dnu, w.cut, pts)
        e = float(np.max(np.abs(k[pts] - ko)) / ko.max())
        print("c5 decade %g-%g cm^-1: max |dk| / max k = %.3e over %d points" % (dec_lo, dec_hi, e, len(pts)))
        assert e <= TOL_K
