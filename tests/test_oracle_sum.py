"""Pins of the oracle's opacity sum k_j = sum_{|nu_j-nu_i|<=cut} S_i V(nu_j - nu_i):
brute force with an independent Faddeeva (scipy's wofz) on tiny inputs, the inclusive
cut predicate, linearity, additivity and cut monotonicity."""
import numpy as np
import scipy.special as sc

import linegen
import oracle


def _tiny(rng, N, lo, hi):
    return {"nu": rng.uniform(lo, hi, N), "S_ref": 10 ** rng.uniform(-22, -19, N),
            "E": rng.exponential(2000.0, N), "gamma_ref": rng.uniform(0.02, 0.1, N), "n": rng.uniform(0.4, 0.8, N)}


def _brute(L, sp, T, P, nu_start, dnu, n, cut):
    S, a, g = oracle.line_params(L, sp, T, P)
    nuj = nu_start + np.arange(n) * dnu
    d = nuj[:, None] - np.asarray(L["nu"])[None, :]
    V = sc.wofz((d + 1j * g[None, :]) / a[None, :]).real / (np.sqrt(np.pi) * a[None, :])
    m = np.abs(d) <= cut
    return (np.where(m, V * S[None, :], 0.0)).sum(axis=1)


def test_brute_force_tiny():
    rng = np.random.default_rng(1)
    sp = oracle.species(18.0, 296.0, 1.0, 0.05, 1.5)
    for T, P, cut, dnu in [(1000.0, 1.0, 2.0, 0.01), (300.0, 1e-3, 0.5, 0.002), (3000.0, 30.0, 1e9, 0.05)]:
        L = _tiny(rng, 40, 100.0, 110.0)
        n = 800
        k = oracle.opacity(L, sp, T, P, 99.0, dnu, cut, np.arange(n))
        ref = _brute(L, sp, T, P, 99.0, dnu, n, cut)
        assert np.max(np.abs(k - ref)) <= 1e-12 * ref.max()


def test_inclusive_cut_boundary():
    sp = oracle.species(18.0, 296.0, 1.0, 0.05, 1.5)
    L = {"nu": [10.0], "S_ref": [1e-20], "E": [100.0], "gamma_ref": [0.05], "n": [0.5]}
    j0, j1 = oracle.jranges(L["nu"], 0.0, 0.5, 100, 2.0)
    assert (j0[0], j1[0]) == (16, 24)
    k = oracle.opacity(L, sp, 500.0, 1.0, 0.0, 0.5, 2.0, np.arange(14, 27))
    assert np.all(k[:2] == 0) and np.all(k[-2:] == 0) and np.all(k[2:11] > 0)
    assert oracle.count_evals(L["nu"], 0.0, 0.5, 100, 2.0) == 9


def test_count_evals_brute():
    rng = np.random.default_rng(4)
    nu = rng.uniform(-5, 60, 300)
    nu = np.abs(nu) + 1e-3
    for cut in (0.37, 3.0, np.inf):
        cnt = oracle.count_evals(nu, 1.0, 0.1, 500, cut)
        nuj = 1.0 + np.arange(500) * 0.1
        ref = int((np.abs(nuj[:, None] - nu[None, :]) <= cut).sum())
        assert cnt == ref


def test_linearity_additivity_monotonicity():
    rng = np.random.default_rng(9)
    sp = oracle.species(18.0, 296.0, 1.0, 0.05, 1.5)
    A, B = _tiny(rng, 30, 200.0, 230.0), _tiny(rng, 25, 205.0, 240.0)
    pts = np.arange(0, 6000, 7)
    kA = oracle.opacity(A, sp, 800.0, 0.3, 195.0, 0.01, 4.0, pts)
    kB = oracle.opacity(B, sp, 800.0, 0.3, 195.0, 0.01, 4.0, pts)
    AB = {k: np.concatenate([A[k], B[k]]) for k in A}
    kAB = oracle.opacity(AB, sp, 800.0, 0.3, 195.0, 0.01, 4.0, pts)
    assert np.max(np.abs(kAB - kA - kB)) <= 1e-14 * kAB.max()
    A2 = dict(A, S_ref=2.0 * A["S_ref"])
    assert np.max(np.abs(oracle.opacity(A2, sp, 800.0, 0.3, 195.0, 0.01, 4.0, pts) - 2 * kA)) <= 1e-15 * kA.max()
    kwide = oracle.opacity(AB, sp, 800.0, 0.3, 195.0, 0.01, 9.0, pts)
    assert np.all(kwide >= kAB)


def test_literal_and_scale_readings_small_config():
    w = linegen.workload("c1")
    sp = oracle.species(*w.species_tuple())
    pts = np.arange(0, w.n_grid, 97)
    for reading in (0, 1):
        L = linegen.generate(w.recipe(s_reading=reading), w.seed, w.N)
        k = oracle.opacity(L, sp, w.T[0], w.P[0], w.nu_start, w.dnu, w.cut, pts)
        assert np.all(np.isfinite(k)) and k.max() > 0


def test_line_functional_sums_to_weighted_opacity():
    """sum_i L_i = sum_j g_j k_j: the per-line functional (a loop over each line's cut range)
    against the per-point sum (a loop over each point's lines), on tiny lists and three cuts."""
    rng = np.random.default_rng(12)
    sp = oracle.species(18.0, 296.0, 1.0, 0.05, 1.5)
    for T, P, cut in [(700.0, 0.5, 1.5), (2000.0, 10.0, 0.2), (300.0, 1e-4, np.inf)]:
        L = _tiny(rng, 25, 50.0, 60.0)
        n = 1500
        g = rng.standard_normal(n)
        Li = oracle.line_functional(L, sp, T, P, 49.0, 0.008, n, cut, g)
        k = oracle.opacity(L, sp, T, P, 49.0, 0.008, cut, np.arange(n))
        ref = float(np.dot(g, k))
        assert abs(Li.sum() - ref) <= 1e-13 * float(np.dot(np.abs(g), k)), (T, P, cut, Li.sum(), ref)


def test_line_functional_per_line_brute_force():
    """L_i = sum over the line's cut range of g_j S_i V_ij with scipy's wofz, line by line."""
    rng = np.random.default_rng(13)
    sp = oracle.species(18.0, 296.0, 1.0, 0.05, 1.5)
    L = _tiny(rng, 12, 20.0, 22.0)
    T, P, cut, nu0, dnu, n = 900.0, 2.0, 0.6, 19.5, 0.004, 800
    g = rng.standard_normal(n)
    Li = oracle.line_functional(L, sp, T, P, nu0, dnu, n, cut, g)
    S, a, gam = oracle.line_params(L, sp, T, P)
    nuj = nu0 + np.arange(n) * dnu
    for i in range(12):
        d = nuj - L["nu"][i]
        V = sc.wofz((d + 1j * gam[i]) / a[i]).real / (np.sqrt(np.pi) * a[i])
        ref = float(np.sum(np.where(np.abs(d) <= cut, g * S[i] * V, 0.0)))
        assert abs(Li[i] - ref) <= 1e-12 * float(np.sum(np.abs(g) * S[i] * V)), (i, Li[i], ref)
