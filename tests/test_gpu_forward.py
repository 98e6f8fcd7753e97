"""GPU parity of the forward path (prep, binning, work list, Voigt kernel, combine) against
the FP64 oracle, through the C ABI. Tolerance: 1e-5 of max k over the compared points."""
import numpy as np
import pytest

import linegen
import oracle
from gpu_util import TOL_K, _lines, gpu_k, oracle_k, prepare, rel_err, to_device, workload_lines

pytestmark = pytest.mark.gpu

SP = (18.0, 296.0, 1.0, 0.05, 1.5)


def test_generator_device_twin_bitwise():
    import torch
    w = linegen.workload("c2")
    N = 300_000
    out = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in range(5)]
    linegen.generate_device(w.recipe(), w.seed, N, [t.data_ptr() for t in out], i0=123_456_789)
    torch.cuda.synchronize()
    host = linegen.generate(w.recipe(), w.seed, N, i0=123_456_789)
    for t, k in zip(out, linegen.FIELDS):
        assert np.array_equal(t.cpu().numpy(), host[k]), k


def test_binning_sorted_stable_permutation():
    import paper_2101_02005_amd as hk
    w, L = workload_lines("c1")
    lines = prepare(L, w.species_tuple())
    keys, perm = hk.hk_debug_sorted(lines)
    keys = keys.cpu().numpy().view(np.uint32).astype(np.int64)
    perm = perm.cpu().numpy().astype(np.int64)
    assert np.all(np.diff(keys) >= 0)
    assert np.array_equal(np.sort(perm), np.arange(w.N))
    same = np.diff(keys) == 0
    assert np.all(np.diff(perm)[same] > 0)  # stable: caller order within a bin
    nu = L["nu"][perm]
    binw = (nu.max() - nu.min()) / (2 ** 24 - 1)
    assert np.all(np.diff(nu) >= -2 * binw)
    lines.release()


@pytest.mark.parametrize("T,P", [(1000.0, 1.0), (100.0, 1e-6), (3000.0, 100.0), (296.0, 1.0)])
def test_line_params_vs_oracle(T, P):
    import paper_2101_02005_amd as hk
    w, L = workload_lines("c2", N=50_000)
    lines = prepare(L, w.species_tuple())
    S, a, g = (x.cpu().numpy() for x in hk.hk_debug_line_params(lines, T, P))
    So, ao, go = oracle.line_params(L, oracle.species(*w.species_tuple()), T, P)
    m = So > 1e-300
    assert np.max(np.abs(S[m] / So[m] - 1)) < 1e-12
    assert np.max(np.abs(a / ao - 1)) < 1e-14
    assert np.max(np.abs(g / go - 1)) < 1e-14
    lines.release()


@pytest.mark.parametrize("cut,nu0,dnu,n", [(25.0, 0.0, 0.1, 20000), (0.37, 99.0, 0.013, 3001),
                                           (100.0, 0.0, 0.01, 1_000_000), (np.inf, 10.0, 0.5, 77)])
def test_cut_bounds_exact(cut, nu0, dnu, n):
    import paper_2101_02005_amd as hk
    w, L = workload_lines("c1")
    lines = prepare(L, w.species_tuple())
    lo, hi = hk.hk_debug_cut_bounds(lines, hk.grid(nu0, dnu, n), cut)
    jo0, jo1 = oracle.jranges(L["nu"], nu0, dnu, n, cut)
    lo, hi = lo.cpu().numpy().astype(np.int64), hi.cpu().numpy().astype(np.int64)
    empty_o = jo1 < jo0
    assert np.array_equal(empty_o, hi < lo)
    assert np.array_equal(lo[~empty_o], jo0[~empty_o]) and np.array_equal(hi[~empty_o], jo1[~empty_o])
    lines.release()


@pytest.mark.parametrize("reading", [1, 0])
def test_small_config_all_points(reading):
    w = linegen.workload("c1", s_reading=reading)
    L = linegen.generate(w.recipe(), w.seed, w.N)
    lines = prepare(L, w.species_tuple())
    k = gpu_k(lines, w.T[0], w.P[0], w.nu_start, w.dnu, w.n_grid, w.cut)
    ko = oracle_k(L, w.species_tuple(), w.T[0], w.P[0], w.nu_start, w.dnu, w.cut, np.arange(w.n_grid))
    print("c1 reading %d: max rel err %.3e" % (reading, rel_err(k, ko)))
    assert rel_err(k, ko) <= TOL_K
    lines.release()


EDGE = [
    # (name, lines, T, P, nu_start, dnu, n, cut)
    ("one line on a grid point", _lines([50.0]), 1000.0, 1.0, 0.0, 0.1, 1000, 25.0),
    ("line beyond the grid end within the cut", _lines([102.3]), 800.0, 0.5, 0.0, 0.1, 1000, 25.0),
    ("line beyond the cut of every point", _lines([200.0]), 800.0, 0.5, 0.0, 0.1, 1000, 25.0),
    ("no cut", _lines(np.linspace(3.0, 180.0, 37)), 1500.0, 2.0, 0.0, 0.05, 4000, np.inf),
    ("single grid point", _lines([10.0, 10.02, 30.0]), 500.0, 1.0, 10.01, 0.01, 1, 5.0),
    ("ragged tile tail", _lines(np.linspace(1.0, 40.0, 200)), 700.0, 0.3, 0.0, 0.01, 2048 * 3 + 17, 2.0),
    ("narrow Doppler lines, unsampled peaks", _lines(np.linspace(5.0, 60.0, 300) + 0.0013, g=0.03),
     100.0, 1e-6, 0.0, 0.01, 7000, 10.0),
    ("zero pressure (pure Gaussian)", _lines(np.linspace(500.0, 520.0, 50)), 1000.0, 0.0, 490.0, 0.001, 30000, 3.0),
    ("very broad Lorentz lines", _lines(np.linspace(100.0, 300.0, 100)), 100.0, 100.0, 0.0, 0.01, 40000, 100.0),
    ("tiny wavenumbers", _lines(np.array([1e-13, 1e-9, 1e-5, 0.3])), 1500.0, 1.0, 0.0, 0.01, 5000, 25.0),
    ("cut shorter than the spacing", _lines(np.linspace(10.0, 11.0, 77)), 300.0, 1.0, 9.0, 0.05, 60, 0.02),
    ("exact cut boundary hits", _lines(np.array([10.0, 12.5, 15.0])), 600.0, 1.0, 0.0, 0.5, 100, 2.0),
]


@pytest.mark.parametrize("case", EDGE, ids=[c[0] for c in EDGE])
def test_edge_cases(case):
    name, L, T, P, nu0, dnu, n, cut = case
    lines = prepare(L, SP)
    k = gpu_k(lines, T, P, nu0, dnu, n, cut)
    ko = oracle_k(L, SP, T, P, nu0, dnu, cut, np.arange(n))
    if ko.max() == 0:
        assert np.all(k == 0)
    else:
        assert rel_err(k, ko) <= TOL_K, (name, rel_err(k, ko))
    # outside the union of the lines' cut ranges the GPU sum is exactly zero
    j0, j1 = oracle.jranges(L["nu"], nu0, dnu, n, cut)
    covered = np.zeros(n + 1, np.int64)
    for a, b in zip(j0, j1):
        if b >= a:
            covered[a] += 1
            covered[b + 1] -= 1
    inside = np.cumsum(covered)[:n] > 0
    assert np.all(k[~inside] == 0)
    lines.release()


def test_isolated_line_cores():
    """Lines far apart on a grid that resolves their cores (spacing alpha/16), y = gamma/alpha
    from 0 to 4.3: each line's window is its own profile, so the comparison pins the FP32
    line-core evaluation (|z| < 4.4) point by point, relative to the line's peak."""
    T, P = 1000.0, 1.0
    sp = (18.0, 296.0, 1.0, 0.05, 1.5)
    ys = np.array([0.0, 0.02, 0.1, 0.3, 0.6, 1.0, 1.5, 2.2, 3.0, 3.7, 4.1, 4.3])
    nu = 1000.0 + 2.0 * np.arange(ys.size) + 0.37e-4 * np.arange(ys.size)  # off-grid centres
    alpha = oracle.line_params(_lines(nu), oracle.species(*sp), T, P)[1]
    L = _lines(nu, S=1e-20, E=100.0, g=ys * alpha, n=0.0)  # n = 0, P = P_ref: gamma = gamma_ref
    assert np.allclose(oracle.line_params(L, oracle.species(*sp), T, P)[2], ys * alpha)
    dnu, cut = 0.0002, 0.5
    nu_start = 999.0
    n = int((nu[-1] + 1.0 - nu_start) / dnu)
    lines = prepare(L, sp)
    k = gpu_k(lines, T, P, nu_start, dnu, n, cut)
    lines.release()
    ko = oracle_k(L, sp, T, P, nu_start, dnu, cut, np.arange(n))
    worst = 0.0
    for i in range(ys.size):
        j0 = int((nu[i] - cut - nu_start) / dnu) + 2
        j1 = int((nu[i] + cut - nu_start) / dnu) - 1
        e = np.max(np.abs(k[j0:j1] - ko[j0:j1])) / ko[j0:j1].max()
        print("y = %.2f: max |dk| / line peak = %.3e" % (ys[i], e))
        worst = max(worst, e)
    assert worst <= 6e-7, worst


def test_unresolved_line_cores():
    """Strong pure-Doppler lines (P = 0) whose width is a tenth of the spacing, each alone, placed
    so that their nearest grid point sits at x = d/alpha from 0.3 to 4.3: the grid samples each
    only there, so that point is its window's max k. It pins the line-core pass's FP64 rounds
    (40 terms) for lines whose peak falls between grid points, point by point relative to that
    sampled value (FP32 rounds there would be 4e-4 off at x = 3, 18 FP64 terms 5e-5)."""
    T, P = 300.0, 0.0
    sp = (18.0, 296.0, 1.0, 0.05, 1.5)
    xs = np.array([0.3, 1.0, 2.0, 2.5, 3.0, 3.5, 4.0, 4.3])
    dnu, cut, nu_start = 0.002, 0.3, 99.0
    g = 100.0 + np.arange(xs.size)  # grid points (multiples of dnu from nu_start)
    alpha = oracle.line_params(_lines(g), oracle.species(*sp), T, P)[1]
    nu = g + xs * alpha
    for _ in range(3):  # alpha is taken at the line's own wavenumber
        alpha = oracle.line_params(_lines(nu), oracle.species(*sp), T, P)[1]
        nu = g + xs * alpha
    assert np.all(alpha < 0.1 * dnu)
    L = _lines(nu, S=1e-20, E=100.0, g=0.05, n=0.5)
    n = int((nu[-1] + 1.0 - nu_start) / dnu)
    lines = prepare(L, sp)
    k = gpu_k(lines, T, P, nu_start, dnu, n, cut)
    lines.release()
    worst = 0.0
    for i in range(xs.size):
        j0 = int((nu[i] - cut - nu_start) / dnu) + 2
        j1 = int((nu[i] + cut - nu_start) / dnu) - 1
        ko = oracle_k(L, sp, T, P, nu_start, dnu, cut, np.arange(j0, j1))
        e = np.max(np.abs(k[j0:j1] - ko)) / ko.max()
        print("x = %.1f: max |dk| / window max = %.3e" % (xs[i], e))
        worst = max(worst, e)
    assert worst <= 1e-6, worst


def test_deterministic_bitwise():
    w, L = workload_lines("c1")
    lines = prepare(L, w.species_tuple())
    k1 = gpu_k(lines, 1300.0, 3.0, 0.0, 0.01, 200_000, 25.0)
    k2 = gpu_k(lines, 1300.0, 3.0, 0.0, 0.01, 200_000, 25.0)
    assert np.array_equal(k1.view(np.uint64), k2.view(np.uint64))
    lines.release()


@pytest.mark.parametrize("field,bad", [("nu", -2.0), ("nu", np.inf), ("S_ref", -1e-20), ("S_ref", np.nan),
                                       ("E", np.inf), ("gamma_ref", -0.01), ("gamma_ref", np.nan), ("n", np.nan)])
def test_invalid_line_data_rejected(field, bad):
    """Each field's check (nu in the first pass, the others while the records are copied)."""
    import paper_2101_02005_amd as hk
    L = _lines([1.0, 2.0, 3.0, 4.0] * 100)
    L[field] = L[field].copy()
    L[field][257] = bad
    with pytest.raises(hk.HkError) as e:
        prepare(L, SP)
    assert e.value.status == hk.HK_EINVAL
    # a valid list still prepares afterwards
    lines = prepare(_lines([1.0, 2.0, 3.0]), SP)
    lines.release()


TUNINGS = [1, 2, 4, 8]  # slots P: span width 64 P, tile-far tile width 256 P


@pytest.mark.parametrize("slots", TUNINGS)
def test_every_tuning_matches_oracle(slots, monkeypatch):
    """Each span width the autotuner may pick gives the same parity."""
    monkeypatch.setenv("HK_SLOTS", str(slots))
    w, L = workload_lines("c1")
    lines = prepare(L, w.species_tuple())
    k = gpu_k(lines, w.T[0], w.P[0], w.nu_start, w.dnu, w.n_grid, w.cut)
    ko = oracle_k(L, w.species_tuple(), w.T[0], w.P[0], w.nu_start, w.dnu, w.cut, np.arange(w.n_grid))
    assert rel_err(k, ko) <= TOL_K
    lines.release()
    for name, Le, T, P, nu0, dnu, n, cut in [EDGE[i] for i in (3, 5, 6, 7, 8, 11)]:
        lines = prepare(Le, SP)
        k = gpu_k(lines, T, P, nu0, dnu, n, cut)
        ko = oracle_k(Le, SP, T, P, nu0, dnu, cut, np.arange(n))
        assert rel_err(k, ko) <= TOL_K, (name, slots, rel_err(k, ko))
        lines.release()


_CLASS_CASES = [(1000.0, 1.0), (3000.0, 10.0)]
_class_oracle = {}


@pytest.mark.parametrize("T,P", _CLASS_CASES)
@pytest.mark.parametrize("slots", TUNINGS)
def test_every_evaluation_class_vs_oracle(slots, T, P, monkeypatch):
    """Dense lines around a 2048-point grid with a 12 cm^-1 cut: every span sees direct lines,
    middle (32-node), far (16-node), very far (8-node) and, for 64- and 128-point spans, masked
    (6-node, cut bound on the span) lines, and tiles see tile-far lines; all points against the
    FP64 oracle."""
    monkeypatch.setenv("HK_SLOTS", str(slots))
    rng = np.random.default_rng(77)
    N = 40000
    L = {"nu": np.sort(rng.uniform(985.0, 1045.0, N))[rng.permutation(N)],
         "S_ref": 10.0 ** rng.uniform(-22.0, -19.0, N), "E": rng.uniform(0.0, 3000.0, N),
         "gamma_ref": rng.uniform(0.01, 0.1, N), "n": rng.uniform(0.4, 0.8, N)}
    nu0, dnu, n, cut = 1000.0, 0.01, 2048, 12.0
    key = (T, P)
    if key not in _class_oracle:
        _class_oracle[key] = oracle_k(L, SP, T, P, nu0, dnu, cut, np.arange(n))
    ko = _class_oracle[key]
    lines = prepare(L, SP)
    k = gpu_k(lines, T, P, nu0, dnu, n, cut)
    lines.release()
    e = rel_err(k, ko)
    print("span %d points, T=%g P=%g: max |dk| / max k = %.3e" % (64 * slots, T, P, e))
    assert e <= TOL_K


def test_autotuner_picks_a_candidate_and_keeps_parity(monkeypatch):
    import paper_2101_02005_amd as hk
    monkeypatch.delenv("HK_SLOTS", raising=False)
    monkeypatch.setenv("HK_AUTOTUNE", "1")
    w, L = workload_lines("c1")
    lines = prepare(L, w.species_tuple())
    k1 = gpu_k(lines, w.T[0], w.P[0], w.nu_start, w.dnu, w.n_grid, w.cut)  # tunes
    t = hk.hk_get_timings()
    assert t.tile_width // 64 in TUNINGS and t.tile_width % 64 == 0
    k2 = gpu_k(lines, w.T[0], w.P[0], w.nu_start, w.dnu, w.n_grid, w.cut)  # cached choice
    assert np.array_equal(k1, k2)
    ko = oracle_k(L, w.species_tuple(), w.T[0], w.P[0], w.nu_start, w.dnu, w.cut, np.arange(w.n_grid))
    assert rel_err(k2, ko) <= TOL_K
    lines.release()


def test_block_cache_reuse_and_empty():
    """A handle prepared into a cached block (released by an earlier handle of the same size)
    gives the same opacity, and so does one prepared after the cache is emptied."""
    import paper_2101_02005_amd as hk
    w, L = workload_lines("c1")
    ks = []
    for i in range(3):
        if i == 2:
            hk.hk_empty_cache()
        lines = prepare(L, w.species_tuple())
        ks.append(gpu_k(lines, w.T[0], w.P[0], w.nu_start, w.dnu, w.n_grid, w.cut))
        lines.release()
    assert np.array_equal(ks[0], ks[1]) and np.array_equal(ks[0], ks[2])
