"""Pins of the oracle's options: the line profiles of Sec. 2.1 (Voigt, Lorentz, Doppler and the
binned Gaussian integrated cross section), plinth removal (Sec. 2.1.1: a line's own value at its
cutting length, subtracted inside the cut) and the cut given as a multiple of the Doppler or the
Lorentz half-width (Sec. 2.4.3 step 4), against closed forms, brute force with scipy, mpmath
quadrature, unit area per line, and central differences for the adjoint."""
import mpmath
import numpy as np
import pytest
import scipy.special as sc

import oracle

SP = oracle.species(18.0, 296.0, 1.0, 0.05, 1.5)
KB, C, AMU = 1.3806489e-16, 2.99792458e10, 1.660538921e-24
R_GAS = 8.314462618e7  # erg / (mol K): the Doppler width from the textbook gas-constant form


def _one(nu, S=1e-20, E=300.0, g=0.06, n=0.6):
    return {"nu": np.array([nu]), "S_ref": np.array([S]), "E": np.array([E]), "gamma_ref": np.array([g]),
            "n": np.array([n])}


def _tiny(rng, N, lo, hi):
    return {"nu": rng.uniform(lo, hi, N), "S_ref": 10 ** rng.uniform(-22, -19, N),
            "E": rng.exponential(2000.0, N), "gamma_ref": rng.uniform(0.02, 0.1, N), "n": rng.uniform(0.4, 0.8, N)}


def test_defaults_reduce_to_plain_opacity():
    rng = np.random.default_rng(3)
    L = _tiny(rng, 40, 100.0, 105.0)
    pts = np.arange(0, 1200, 3)
    for cut in (1.5, np.inf):
        a = oracle.opacity(L, SP, 900.0, 0.7, 99.5, 0.005, cut, pts)
        b = oracle.opacity_ex(L, SP, 900.0, 0.7, 99.5, 0.005, cut, pts)
        assert np.array_equal(a, b)


def test_plinth_is_the_value_at_the_cut():
    """One line whose cut falls exactly on grid points: k there is zero, inside it is S (V(d) -
    V(cut)) with scipy's wofz, outside zero."""
    L = _one(10.0)
    T, P, cut, nu0, dnu, n = 500.0, 1.0, 2.0, 0.0, 0.5, 100
    k = oracle.opacity_ex(L, SP, T, P, nu0, dnu, cut, np.arange(n), plinth=True)
    S, a, g = (x[0] for x in oracle.line_params(L, SP, T, P))
    V = lambda d: sc.wofz((d + 1j * g) / a).real / (np.sqrt(np.pi) * a)
    d = nu0 + np.arange(n) * dnu - 10.0
    inside = np.abs(d) <= cut
    ref = np.where(inside, S * (V(d) - V(cut)), 0.0)
    assert k[16] == 0.0 and k[24] == 0.0  # |d| = cut exactly
    assert np.max(np.abs(k - ref)) <= 1e-13 * S * V(0.0)
    assert np.all(k[inside] >= 0.0) and np.all(k[~inside] == 0.0)


def test_plinth_lorentz_closed_form():
    L = _one(50.0, g=0.08)
    T, P, cut, nu0, dnu, n = 700.0, 3.0, 4.0, 44.0, 0.01, 1200
    k = oracle.opacity_ex(L, SP, T, P, nu0, dnu, cut, np.arange(n), profile=oracle.PROFILE_LORENTZ, plinth=True)
    S, _, g = (x[0] for x in oracle.line_params(L, SP, T, P))
    d = nu0 + np.arange(n) * dnu - 50.0
    ref = np.where(np.abs(d) <= cut, S * g / np.pi * (1 / (d * d + g * g) - 1 / (cut * cut + g * g)), 0.0)
    assert np.max(np.abs(k - ref)) <= 1e-14 * ref.max()


def _alpha_textbook(nu, T, M):
    return nu / C * np.sqrt(2 * R_GAS * T / M)


@pytest.mark.parametrize("mult", [3.0, 25.0])
def test_doppler_multiple_cut_bound(mult):
    """Cut = mult x Doppler half-width sqrt(ln 2) alpha; the included points are exactly those
    within that distance (alpha from the gas-constant form, independent of the oracle's k_B/amu)."""
    nu_l, T, P, nu0, dnu, n = 1000.0037, 1000.0, 1.0, 999.0, 0.0005, 4000
    L = _one(nu_l)
    c = mult * np.sqrt(np.log(2)) * _alpha_textbook(nu_l, T, 18.0)
    d = nu0 + np.arange(n) * dnu - nu_l
    assert np.min(np.abs(np.abs(d) - c)) > 1e-5 * c  # no grid point within the constants' spread
    k = oracle.opacity_ex(L, SP, T, P, nu0, dnu, mult, np.arange(n), cut_mode=oracle.CUT_DOPPLER)
    assert np.array_equal(k != 0.0, np.abs(d) <= c)
    cl = oracle.cut_lengths(L, SP, T, P, oracle.CUT_DOPPLER, mult)
    assert abs(cl[0] / c - 1) < 1e-6


@pytest.mark.parametrize("mult", [2.0, 40.0])
def test_lorentz_multiple_cut_bound(mult):
    nu_l, T, P, nu0, dnu, n = 300.0013, 600.0, 0.5, 295.0, 0.001, 10000
    L = _one(nu_l, g=0.07, n=0.7)
    gam = 0.07 * (296.0 / T) ** 0.7 * P
    c = mult * gam
    d = nu0 + np.arange(n) * dnu - nu_l
    assert np.min(np.abs(np.abs(d) - c)) > 1e-9 * c
    k = oracle.opacity_ex(L, SP, T, P, nu0, dnu, mult, np.arange(n), cut_mode=oracle.CUT_LORENTZ)
    assert np.array_equal(k != 0.0, np.abs(d) <= c)


def test_pure_profiles_closed_forms():
    L = _one(200.0, g=0.09)
    T, P, nu0, dnu, n = 1200.0, 2.0, 199.0, 0.002, 1000
    S, a, g = (x[0] for x in oracle.line_params(L, SP, T, P))
    d = nu0 + np.arange(n) * dnu - 200.0
    kd = oracle.opacity_ex(L, SP, T, P, nu0, dnu, np.inf, np.arange(n), profile=oracle.PROFILE_DOPPLER)
    a_tb = _alpha_textbook(200.0, T, 18.0)
    ref = S * np.exp(-(d / a_tb) ** 2) / (np.sqrt(np.pi) * a_tb)
    assert np.max(np.abs(kd - ref)) <= 2e-5 * ref.max()  # constants: CODATA k_B/amu vs the gas constant
    kl = oracle.opacity_ex(L, SP, T, P, nu0, dnu, np.inf, np.arange(n), profile=oracle.PROFILE_LORENTZ)
    refl = S * g / (np.pi * (d * d + g * g))
    assert np.max(np.abs(kl - refl)) <= 1e-14 * refl.max()
    # Voigt: between the two limits, and equal to scipy's voigt_profile (sigma = alpha / sqrt 2)
    kv = oracle.opacity_ex(L, SP, T, P, nu0, dnu, np.inf, np.arange(n))
    assert np.max(np.abs(kv - S * sc.voigt_profile(d, a / np.sqrt(2), g))) <= 1e-12 * kv.max()


def test_binned_gaussian_quadrature_and_unit_area():
    """Each point is the bin average of the Gaussian (mpmath quadrature over the bin); summed over
    a grid covering the line, times the spacing, it is the line strength (unit area per line)."""
    L = _one(500.0)
    T, P, nu0, dnu = 2500.0, 1.0, 499.9, 0.0007
    S, a, _ = (x[0] for x in oracle.line_params(L, SP, T, P))
    n = 290
    k = oracle.opacity_ex(L, SP, T, P, nu0, dnu, np.inf, np.arange(n), profile=oracle.PROFILE_BINNED_GAUSS)
    mpmath.mp.dps = 30
    for j in (0, 57, 142, 143, 200, 289):
        cj = mpmath.mpf(nu0) + j * mpmath.mpf(dnu) - 500
        f = lambda v: mpmath.exp(-(v / a) ** 2) / (mpmath.sqrt(mpmath.pi) * a)
        ref = S * mpmath.quad(f, [cj - dnu / 2, cj + dnu / 2]) / dnu
        assert abs(k[j] - float(ref)) <= 1e-12 * k.max() + 1e-14 * abs(float(ref)), (j, k[j], float(ref))
    wide = oracle.opacity_ex(L, SP, T, P, 499.0, dnu, np.inf, np.arange(3000), profile=oracle.PROFILE_BINNED_GAUSS)
    assert abs(wide.sum() * dnu / S - 1.0) < 1e-11


def test_binned_gaussian_plinth_and_tails():
    """Far tails (both bin edges on one side) keep their relative precision, and the plinth of the
    binned profile is its own value at the cut."""
    L = _one(800.0)
    T, P, nu0, dnu = 300.0, 1.0, 799.0, 0.001
    S, a, _ = (x[0] for x in oracle.line_params(L, SP, T, P))
    j = np.arange(2000)
    d = nu0 + j * dnu - 800.0
    k = oracle.opacity_ex(L, SP, T, P, nu0, dnu, np.inf, j, profile=oracle.PROFILE_BINNED_GAUSS)
    far = np.abs(d) > 8 * a
    ref = S * (sc.erfc((np.abs(d[far]) - dnu / 2) / a) - sc.erfc((np.abs(d[far]) + dnu / 2) / a)) / (2 * dnu)
    m = ref > 1e-290
    assert np.max(np.abs(k[far][m] / ref[m] - 1)) < 1e-10
    cut = 0.0305
    kp = oracle.opacity_ex(L, SP, T, P, nu0, dnu, cut, j, profile=oracle.PROFILE_BINNED_GAUSS, plinth=True)
    kc = oracle.opacity_ex(L, SP, T, P, nu0, dnu, cut, j, profile=oracle.PROFILE_BINNED_GAUSS)
    inside = np.abs(d) <= cut
    pl = S * (sc.erf((cut + dnu / 2) / a) - sc.erf((cut - dnu / 2) / a)) / (2 * dnu)
    assert np.max(np.abs((kc - kp)[inside] - pl)) <= 1e-12 * kc.max()


# --------------------------------------------------------------------- adjoint with options
NU0, DNU, NG = 95.0, 0.02, 2500


def _L(lines, T, P, g, cut, mode, plinth):
    k = oracle.opacity_ex(lines, SP, T, P, NU0, DNU, cut, np.arange(NG), cut_mode=mode, plinth=plinth)
    return float(np.dot(g, k))


CASES = [(4.0, oracle.CUT_FIXED, True), (120.0, oracle.CUT_DOPPLER, True), (30.0, oracle.CUT_LORENTZ, True),
         (120.0, oracle.CUT_DOPPLER, False)]


@pytest.mark.parametrize("cut,mode,plinth", CASES)
def test_adjoint_with_options_vs_central_differences(cut, mode, plinth):
    """Scalars and per-line gradients against central differences (h = 1e-4 relative) of
    L = g . k with the option. Without the plinth, a per-line cut still moves its bound with the
    parameters, and that indicator is not differentiated: those cases compare only where no grid
    point lies within the step of a bound (checked)."""
    rng = np.random.default_rng(21)
    L = {"nu": rng.uniform(100.0, 140.0, 10), "S_ref": 10 ** rng.uniform(-21, -19, 10),
         "E": rng.exponential(1500.0, 10), "gamma_ref": rng.uniform(0.02, 0.1, 10), "n": rng.uniform(0.4, 0.8, 10)}
    T, P = 800.0, 0.3
    g = np.random.default_rng(6).standard_normal(NG)
    G = oracle.gradient_ex(L, SP, T, P, NU0, DNU, NG, cut, g, cut_mode=mode, plinth=plinth)
    if not plinth:
        # no grid point within 1e-3 of any line's cut bound at the stepped parameters
        for TT in (T * (1 - 1e-4), T, T * (1 + 1e-4)):
            cl = oracle.cut_lengths(L, SP, TT, P, mode, cut)
            for s in (-1, 1):
                e = (L["nu"] + s * cl - NU0) / DNU
                assert np.min(np.abs(e - np.round(e))) > 1e-3
    h = 1e-4
    fd_T = (_L(L, T * (1 + h), P, g, cut, mode, plinth) - _L(L, T * (1 - h), P, g, cut, mode, plinth)) / (2 * h * T)
    assert abs(G["dT_part"].sum() - fd_T) <= 1e-6 * abs(fd_T) + 1e-9 * np.sum(np.abs(G["dT_part"]))
    if not plinth:
        return
    fd_P = (_L(L, T, P * np.exp(h), g, cut, mode, plinth) - _L(L, T, P * np.exp(-h), g, cut, mode, plinth)) / (2 * h)
    assert abs(G["dlnP_part"].sum() - fd_P) <= 1e-6 * abs(fd_P) + 1e-9 * np.sum(np.abs(G["dlnP_part"]))
    scale = {k: np.max(np.abs(G[k])) for k in ("dS_ref", "dgamma_ref", "dn")}
    for i in range(len(L["nu"])):
        for key, gkey in (("S_ref", "dS_ref"), ("gamma_ref", "dgamma_ref"), ("n", "dn")):
            hh = 1e-4 * L[key][i]
            Lp = {k: v.copy() for k, v in L.items()}
            Lm = {k: v.copy() for k, v in L.items()}
            Lp[key][i] += hh
            Lm[key][i] -= hh
            fd = (_L(Lp, T, P, g, cut, mode, plinth) - _L(Lm, T, P, g, cut, mode, plinth)) / (2 * hh)
            assert abs(G[gkey][i] - fd) <= 1e-5 * scale[gkey], (mode, key, i, G[gkey][i], fd)


def test_adjoint_with_plinth_invariants():
    rng = np.random.default_rng(8)
    L = _tiny(rng, 30, 100.0, 140.0)
    g = rng.standard_normal(NG)
    T, P = 1300.0, 2.0
    for mode, cut in ((oracle.CUT_FIXED, 4.0), (oracle.CUT_LORENTZ, 25.0)):
        G = oracle.gradient_ex(L, SP, T, P, NU0, DNU, NG, cut, g, cut_mode=mode, plinth=True)
        Lval = _L(L, T, P, g, cut, mode, True)
        assert abs(np.sum(L["S_ref"] * G["dS_ref"]) - Lval) <= 1e-12 * np.sum(np.abs(L["S_ref"] * G["dS_ref"]))
        assert abs(G["dlnP_part"].sum() - np.sum(L["gamma_ref"] * G["dgamma_ref"])) <= 1e-13 * np.sum(
            np.abs(G["dlnP_part"]))
