"""Pins of the oracle's FP64 Faddeeva function w(z) = exp(-z^2) erfc(-iz) against
independent references: scipy's wofz (a different implementation), mpmath at 30 digits,
and closed forms on the axes and at infinity. The paper itself checks its Voigt code
against scipy.special.wofz over the a-u plane (Sec. 2.2.3, figure of fractional errors)."""
import mpmath
import numpy as np
import pytest
import scipy.special as sc

import oracle


def _sweep():
    r = np.logspace(-8, 12, 300)
    th = np.linspace(0.0, np.pi / 2, 120)
    R, TH = np.meshgrid(r, th)
    x = (R * np.cos(TH)).ravel()
    y = (R * np.sin(TH)).ravel()
    return np.concatenate([x, -x]), np.concatenate([y, y])


def test_vs_scipy_wofz_logpolar():
    x, y = _sweep()
    w = oracle.faddeeva(x, y)
    ws = sc.wofz(x + 1j * y)
    rel = np.abs(w - ws) / np.abs(ws)
    assert rel.max() < 1e-13, (rel.max(), x[rel.argmax()], y[rel.argmax()])
    # real part on its own wherever it is not exponentially small against |w|
    m = np.abs(ws.real) > 1e-3 * np.abs(ws)
    rr = np.abs(w.real - ws.real)[m] / np.abs(ws.real[m])
    assert rr.max() < 1e-12


def test_vs_mpmath():
    mpmath.mp.dps = 30
    rng = np.random.default_rng(7)
    pts = [(0.0, 0.0), (1e-3, 1e-3), (1.0, 1.0), (3.9, 0.01), (5.5, 1e-8), (6.3, 4.4 * 0.3), (8.0, 0.06),
           (12.0, 2.0), (100.0, 1e-6), (1e4, 3.0), (0.2, 30.0), (2.0, 5e-4)]
    pts += [(float(a), float(b)) for a, b in zip(rng.uniform(-15, 15, 60), 10 ** rng.uniform(-6, 1.5, 60))]
    for x, y in pts:
        z = mpmath.mpc(x, y)
        ref = complex(mpmath.exp(-z * z) * mpmath.erfc(-1j * z))
        w = complex(oracle.faddeeva([x], [y])[0])
        assert abs(w - ref) <= 1e-13 * abs(ref), (x, y, w, ref)


def test_origin_and_axes():
    assert oracle.faddeeva([0.0], [0.0])[0] == pytest.approx(1.0, abs=1e-15)
    y = np.logspace(-10, 8, 400)
    w = oracle.faddeeva(np.zeros_like(y), y)
    # w(iy) = erfcx(y), real
    assert np.max(np.abs(w.real - sc.erfcx(y)) / sc.erfcx(y)) < 1e-13
    assert np.max(np.abs(w.imag)) == 0.0
    x = np.linspace(-30, 30, 2001)
    w = oracle.faddeeva(x, np.zeros_like(x))
    # Re w(x) = exp(-x^2), Im w(x) = (2/sqrt(pi)) Dawson(x)
    assert np.max(np.abs(w.real - np.exp(-x * x))) < 1e-15
    assert np.max(np.abs(w.imag - 2 / np.sqrt(np.pi) * sc.dawsn(x))) < 1e-14


def test_asymptote_and_symmetry():
    z = np.array([1e8 + 1j, 3e9 + 5e3j, 1e7j + 1e7])
    w = oracle.faddeeva(z.real, z.imag)
    lead = 1j / (np.sqrt(np.pi) * z)
    assert np.max(np.abs(w / lead - 1)) < 1e-13
    x, y = np.linspace(0.1, 20, 50), np.linspace(0.0, 3, 50)
    assert np.array_equal(oracle.faddeeva(-x, y), np.conj(oracle.faddeeva(x, y)))


def test_derivative_relation():
    # w'(z) = -2 z w + 2i/sqrt(pi): check by central differences of the oracle itself
    rng = np.random.default_rng(3)
    for _ in range(40):
        x, y = rng.uniform(-9, 9), 10 ** rng.uniform(-2, 1)
        h = 1e-5
        dw = (oracle.faddeeva([x + h], [y])[0] - oracle.faddeeva([x - h], [y])[0]) / (2 * h)
        w = oracle.faddeeva([x], [y])[0]
        z = x + 1j * y
        assert abs(dw - (-2 * z * w + 2j / np.sqrt(np.pi))) < 1e-8 * max(1.0, abs(w))
