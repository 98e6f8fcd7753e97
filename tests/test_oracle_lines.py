"""Pins of the oracle's per-line quantities: strength S(T) (Sec. 2.2.2 eqs. S, S1), Doppler
width (eqs. gammaD/alphaD) and ExoMol Lorentz width (Sec. 2.2)."""
import mpmath
import numpy as np

import oracle

KB, C, H, AMU = 1.3806489e-16, 2.99792458e10, 6.62606957e-27, 1.660538921e-24


def _lines(N, rng):
    return {"nu": rng.uniform(1.0, 3e4, N), "S_ref": 10 ** rng.uniform(-26, -19, N),
            "E": rng.exponential(3000.0, N), "gamma_ref": rng.uniform(0.02, 0.1, N), "n": rng.uniform(0.4, 0.8, N)}


def test_strength_at_reference_temperature():
    rng = np.random.default_rng(11)
    L = _lines(2000, rng)
    sp = oracle.species(18.0, 296.0, 1.0, 0.05, 1.5)
    S, _, _ = oracle.line_params(L, sp, 296.0, 1.0)
    assert np.max(np.abs(S / L["S_ref"] - 1)) < 1e-13


def test_strength_matches_eq_S_form():
    # eq. (S) per molecule (no mass factor): S = A g' / (8 pi c nu^2 Q(T)) e^{-c2 E/T} (1 - e^{-c2 nu/T}),
    # evaluated in mpmath from synthetic A, g'; S_ref is that expression at T_ref.
    mpmath.mp.dps = 40
    rng = np.random.default_rng(5)
    c2 = mpmath.mpf(H) * mpmath.mpf(C) / mpmath.mpf(KB)
    sp = oracle.species(18.0, 296.0, 1.0, 0.05, 1.5)
    Q = lambda T: mpmath.mpf(0.05) * mpmath.mpf(T) ** mpmath.mpf(1.5)

    def S_eq(A, gp, nu, E, T):
        T = mpmath.mpf(T)
        return (A * gp / (8 * mpmath.pi * C * nu ** 2 * Q(T)) * mpmath.exp(-c2 * E / T)
                * (1 - mpmath.exp(-c2 * nu / T)))

    for _ in range(60):
        A, gp = 10 ** rng.uniform(-4, 2), float(rng.integers(1, 40))
        nu, E = float(10 ** rng.uniform(-3, 4.5)), float(rng.uniform(0, 3e4))
        sref = S_eq(mpmath.mpf(A), gp, mpmath.mpf(nu), mpmath.mpf(E), 296.0)
        L = {"nu": [nu], "S_ref": [float(sref)], "E": [E], "gamma_ref": [0.05], "n": [0.5]}
        for T in (100.0, 800.0, 3000.0):
            S, _, _ = oracle.line_params(L, sp, T, 1.0)
            ref = float(S_eq(mpmath.mpf(A), gp, mpmath.mpf(nu), mpmath.mpf(E), T))
            if ref > 1e-300:
                assert abs(S[0] / ref - 1) < 1e-12, (nu, E, T, S[0], ref)


def test_stimulated_emission_low_frequency_limit():
    # (1 - e^{-c2 nu/T}) / (1 - e^{-c2 nu/T_ref}) -> T_ref/T as nu -> 0
    sp = oracle.species(18.0, 296.0, 1.0, 0.05, 1.5)
    L = {"nu": [1e-13], "S_ref": [1e-20], "E": [0.0], "gamma_ref": [0.05], "n": [0.5]}
    for T in (100.0, 1500.0):
        S, _, _ = oracle.line_params(L, sp, T, 1.0)
        assert abs(S[0] / (1e-20 * (296.0 / T) ** 1.5 * (296.0 / T)) - 1) < 1e-11


def test_doppler_width_textbook_constant():
    # HWHM Gamma_D = sqrt(ln2) alpha = (nu/c) sqrt(2 ln2 R T / M) with the gas constant R
    R = 8.314462618e7  # erg / (mol K)
    nu = np.array([1.0, 1000.0, 3e4])
    for T, M in [(296.0, 18.0), (4000.0, 56.0)]:
        sp = oracle.species(M, 296.0, 1.0, 0.05, 1.5)
        L = {"nu": nu, "S_ref": np.ones(3), "E": np.zeros(3), "gamma_ref": np.ones(3), "n": np.ones(3)}
        _, a, _ = oracle.line_params(L, sp, T, 1.0)
        ref = nu / C * np.sqrt(2 * np.log(2) * R * T / M)
        assert np.max(np.abs(a * np.sqrt(np.log(2)) / ref - 1)) < 1e-6


def test_lorentz_width_scalings():
    rng = np.random.default_rng(2)
    L = _lines(100, rng)
    sp = oracle.species(18.0, 296.0, 1.0, 0.05, 1.5)
    _, _, g0 = oracle.line_params(L, sp, 296.0, 1.0)
    assert np.array_equal(g0, L["gamma_ref"])
    _, _, gP = oracle.line_params(L, sp, 296.0, 7.5)
    assert np.max(np.abs(gP / (7.5 * L["gamma_ref"]) - 1)) < 1e-15
    _, _, g1 = oracle.line_params(L, sp, 500.0, 1.0)
    _, _, g2 = oracle.line_params(L, sp, 1500.0, 1.0)
    assert np.max(np.abs(g1 / g2 - 3.0 ** L["n"])) < 1e-13


def test_strength_high_lower_state_energy_branch():
    """Lines with c2 E''/T_ref >= 700 (E'' above about 1.44e5 cm^-1 at 296 K) take the oracle's
    combined-exponent form, since exp(c2 E''/T_ref) alone would overflow. Pinned against eq. (S)
    per molecule evaluated in mpmath from synthetic A, g' (the input S_ref being that expression
    at T_ref, rounded to double), across the switch between the two forms."""
    mpmath.mp.dps = 50
    c2 = mpmath.mpf(H) * mpmath.mpf(C) / mpmath.mpf(KB)
    sp = oracle.species(18.0, 296.0, 1.0, 0.05, 1.5)
    Q = lambda T: mpmath.mpf(0.05) * mpmath.mpf(T) ** mpmath.mpf(1.5)

    def S_eq(Agp, nu, E, T):
        T = mpmath.mpf(T)
        return (Agp / (8 * mpmath.pi * C * nu ** 2 * Q(T)) * mpmath.exp(-c2 * E / T)
                * (1 - mpmath.exp(-c2 * nu / T)))

    E_switch = 700.0 * 296.0 / float(c2)
    energies = [E_switch * (1 - 1e-9), E_switch * (1 + 1e-9), 1.5e5, 1.8e5, 2.0e5]
    for E in energies:
        for nu in (0.5, 2000.0, 25000.0):
            # A g' chosen so that S_ref stays a normal double however small exp(-c2 E''/T_ref) is
            Agp = mpmath.mpf(10) ** (int(float(c2) * E / 296.0 / mpmath.log(10)) - 270) * nu ** 2
            sref = S_eq(Agp, mpmath.mpf(nu), mpmath.mpf(E), 296.0)
            assert 1e-300 < float(sref) < 1e300
            L = {"nu": [nu], "S_ref": [float(sref)], "E": [E], "gamma_ref": [0.05], "n": [0.5]}
            for T in (500.0, 3000.0, 10000.0):
                S, _, _ = oracle.line_params(L, sp, T, 1.0)
                ref = S_eq(Agp, mpmath.mpf(nu), mpmath.mpf(E), T) * (mpmath.mpf(float(sref)) / sref)
                assert abs(S[0] / float(ref) - 1) < 2e-13, (E, nu, T, S[0], float(ref))
