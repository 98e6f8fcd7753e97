"""Pins of the oracle's HITRAN-style widths and pressure shift (or_opacity_hitran) against the
already pinned ExoMol-form oracle: the special cases that reduce to it (no shift with equal
air and self widths, a pure self-broadened gas, an even mix), and the exact translation of k
by a shift of a whole number of grid steps (which also fixes that the strength and Doppler
width keep the unshifted wavenumber)."""
import numpy as np
import pytest

import oracle

SP = (18.0, 296.0, 1.0, 0.05, 1.5)


def _list(N, seed, lo=995.0, hi=1015.0):
    rng = np.random.default_rng(seed)
    return {"nu": rng.uniform(lo, hi, N), "S_ref": 10 ** rng.uniform(-22, -19, N), "E": rng.exponential(1500.0, N),
            "gamma_air": rng.uniform(0.02, 0.1, N), "gamma_self": rng.uniform(0.1, 0.5, N),
            "n": rng.uniform(0.4, 0.8, N), "delta": rng.uniform(-0.02, 0.01, N)}


def _exomol(L, gref):
    return {"nu": L["nu"], "S_ref": L["S_ref"], "E": L["E"], "gamma_ref": gref, "n": L["n"]}


PTS = np.arange(0, 16_000)
GRID = (1000.0, 0.000625)  # dnu = 2^-4 / 100 is not exact; the translation test uses its own grid


@pytest.mark.parametrize("profile,cut_mode,cut,plinth", [(0, 0, 2.0, False), (0, 2, 30.0, True), (1, 0, 1.0, True),
                                                         (2, 1, 5.0, False), (3, 0, 0.5, True)])
def test_reduces_to_exomol_form(profile, cut_mode, cut, plinth):
    L = _list(400, 1)
    sp = oracle.species(*SP)
    T, P = 900.0, 2.5
    kw = dict(cut_mode=cut_mode, profile=profile, plinth=plinth)
    # no shift, equal air and self widths: the ExoMol form with gamma_ref = gamma_air, any P_self
    L0 = dict(L, delta=np.zeros(400), gamma_self=L["gamma_air"])
    ref = oracle.opacity_ex(_exomol(L, L["gamma_air"]), sp, T, P, GRID[0], GRID[1], cut, PTS, **kw)
    assert np.max(np.abs(ref)) > 0
    for ps in (0.0, 1.0, P):
        k = oracle.opacity_hitran(L0, sp, T, P, ps, GRID[0], GRID[1], cut, PTS, **kw)
        assert np.max(np.abs(k - ref)) <= 1e-12 * np.max(np.abs(ref))
    # a pure self-broadened gas, and an even mix
    Lz = dict(L, delta=np.zeros(400))
    for ps, g in ((P, L["gamma_self"]), (0.5 * P, 0.5 * (L["gamma_air"] + L["gamma_self"]))):
        k = oracle.opacity_hitran(Lz, sp, T, P, ps, GRID[0], GRID[1], cut, PTS, **kw)
        r = oracle.opacity_ex(_exomol(L, g), sp, T, P, GRID[0], GRID[1], cut, PTS, **kw)
        assert np.max(np.abs(k - r)) <= 1e-12 * np.max(np.abs(r))


@pytest.mark.parametrize("profile,plinth", [(0, False), (0, True), (2, False), (1, True)])
def test_shift_translates_k(profile, plinth):
    """Every line shifted by the same m grid steps: k moves by m points, unchanged otherwise."""
    L = _list(300, 2, 1002.0, 1008.0)
    sp = oracle.species(*SP)
    T, P, m, dnu = 1200.0, 4.0, 24, 0.0078125  # dnu = 2^-7: the shifted centres stay exact
    L["nu"] = np.round(L["nu"] / dnu) * dnu + 0.3 * dnu  # on a 2^-7 lattice plus a fixed offset
    d = m * dnu / P
    Ls = dict(L, delta=np.full(300, d))
    L0 = dict(L, delta=np.zeros(300))
    pts = np.arange(0, 2000)
    nu0 = 998.0
    k0 = oracle.opacity_hitran(L0, sp, T, P, 1.0, nu0, dnu, 3.0, pts, profile=profile, plinth=plinth)
    ks = oracle.opacity_hitran(Ls, sp, T, P, 1.0, nu0, dnu, 3.0, pts + m, profile=profile, plinth=plinth)
    assert np.max(np.abs(k0)) > 0
    assert np.max(np.abs(ks - k0)) <= 1e-13 * np.max(np.abs(k0))
    # while taking the strength and Doppler width at the shifted centre instead would not be
    Lw = dict(L0, nu=L["nu"] + m * dnu)
    kw = oracle.opacity_hitran(Lw, sp, T, P, 1.0, nu0, dnu, 3.0, pts + m, profile=profile, plinth=plinth)
    assert np.max(np.abs(kw - k0)) > 1e-9 * np.max(np.abs(k0))


def test_rejects_bad_partial_pressure():
    L = _list(10, 3)
    with pytest.raises(ValueError):
        oracle.opacity_hitran(L, oracle.species(*SP), 500.0, 1.0, 2.0, 1000.0, 0.01, 1.0, np.arange(10))
