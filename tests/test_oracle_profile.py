"""Pins of the oracle's Voigt profile V = Re w((d + i gamma)/alpha)/(sqrt(pi) alpha):
Gaussian and Lorentz limits (the two profiles it convolves, Sec. 2.1), unit normalization,
and symmetry."""
import numpy as np

import oracle


def test_gaussian_limit():
    a = 0.013
    d = np.linspace(-0.1, 0.1, 401)
    V = oracle.voigt(d, a, 0.0)
    G = np.exp(-(d / a) ** 2) / (np.sqrt(np.pi) * a)
    assert np.max(np.abs(V - G)) <= 1e-14 * G.max()
    V2 = oracle.voigt(d, a, 1e-12 * a)
    assert np.max(np.abs(V2 - G)) <= 1e-10 * G.max()


def test_lorentz_limit():
    g = 0.07
    d = np.linspace(-3, 3, 601)
    L = g / (np.pi * (d * d + g * g))
    V = oracle.voigt(d, 1e-9 * g, g)
    assert np.max(np.abs(V / L - 1)) < 1e-12


def test_normalization_cut_span():
    # sum_j V_j dnu over |d| <= Lspan equals (2/pi) atan(Lspan/gamma) up to O(gamma alpha^2 / Lspan^3)
    a, g, Lspan, dnu = 0.05, 0.01, 100.0, 0.0025
    n = int(round(2 * Lspan / dnu)) + 1
    d = -Lspan + dnu * np.arange(n)
    V = oracle.voigt(d, a, g)
    s = (V.sum() - 0.5 * (V[0] + V[-1])) * dnu
    assert abs(s - 2 / np.pi * np.arctan(Lspan / g)) < 1e-8


def test_normalization_doppler_dominated():
    a, g, dnu = 0.3, 1e-4, 0.01
    d = dnu * np.arange(-20000, 20001)
    s = oracle.voigt(d, a, g).sum() * dnu
    assert abs(s - 2 / np.pi * np.arctan(200.0 / g)) < 1e-9


def test_symmetry_and_positivity():
    d = np.linspace(0, 50, 1001)
    for a, g in [(0.01, 0.05), (0.4, 0.001), (1e-6, 0.1)]:
        Vp, Vm = oracle.voigt(d, a, g), oracle.voigt(-d, a, g)
        assert np.array_equal(Vp, Vm)
        assert np.all(Vp > 0)
