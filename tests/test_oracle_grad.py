"""Pins of the oracle's analytic FP64 adjoint: central finite differences of the oracle's
own forward (h = 1e-4 relative) and the exact invariants of the parameterisation."""
import numpy as np
import pytest

import oracle

SP = oracle.species(18.0, 296.0, 1.0, 0.05, 1.5)
NU0, DNU, NG, CUT = 95.0, 0.02, 2500, 4.0


def _lines(seed=0, N=30):
    rng = np.random.default_rng(seed)
    return {"nu": rng.uniform(100.0, 140.0, N), "S_ref": 10 ** rng.uniform(-21, -19, N),
            "E": rng.exponential(1500.0, N), "gamma_ref": rng.uniform(0.02, 0.1, N), "n": rng.uniform(0.4, 0.8, N)}


def _L(lines, T, P, g):
    k = oracle.opacity(lines, SP, T, P, NU0, DNU, CUT, np.arange(NG))
    return float(np.dot(g, k))


@pytest.mark.parametrize("T,P", [(800.0, 0.1), (2000.0, 3.0)])
def test_scalars_vs_central_differences(T, P):
    L = _lines(1)
    g = np.random.default_rng(4).standard_normal(NG)
    G = oracle.gradient(L, SP, T, P, NU0, DNU, NG, CUT, g)
    h = 1e-4 * T
    fd_T = (_L(L, T + h, P, g) - _L(L, T - h, P, g)) / (2 * h)
    assert abs(G["dT_part"].sum() - fd_T) <= 1e-6 * abs(fd_T)
    hp = 1e-4
    fd_P = (_L(L, T, P * np.exp(hp), g) - _L(L, T, P * np.exp(-hp), g)) / (2 * hp)
    assert abs(G["dlnP_part"].sum() - fd_P) <= 1e-6 * abs(fd_P)


def test_per_line_vs_central_differences():
    L = _lines(2, 12)
    T, P = 800.0, 0.1
    g = np.random.default_rng(6).standard_normal(NG)
    G = oracle.gradient(L, SP, T, P, NU0, DNU, NG, CUT, g)
    scale = {k: np.max(np.abs(G[k])) for k in ("dS_ref", "dgamma_ref", "dn")}
    for i in range(len(L["nu"])):
        for key, gkey in (("S_ref", "dS_ref"), ("gamma_ref", "dgamma_ref"), ("n", "dn")):
            h = 1e-4 * L[key][i]
            Lp = {k: v.copy() for k, v in L.items()}
            Lm = {k: v.copy() for k, v in L.items()}
            Lp[key][i] += h
            Lm[key][i] -= h
            fd = (_L(Lp, T, P, g) - _L(Lm, T, P, g)) / (2 * h)
            assert abs(G[gkey][i] - fd) <= 1e-6 * scale[gkey], (key, i, G[gkey][i], fd)


def test_invariants():
    L = _lines(3, 40)
    g = np.random.default_rng(8).standard_normal(NG)
    T, P = 1300.0, 2.0
    G = oracle.gradient(L, SP, T, P, NU0, DNU, NG, CUT, g)
    Lval = _L(L, T, P, g)
    # L is linear in S_ref
    assert abs(np.sum(L["S_ref"] * G["dS_ref"]) - Lval) <= 1e-12 * np.sum(np.abs(L["S_ref"] * G["dS_ref"]))
    # gamma depends on P only through P/P_ref
    assert abs(G["dlnP_part"].sum() - np.sum(L["gamma_ref"] * G["dgamma_ref"])) <= 1e-13 * np.sum(np.abs(G["dlnP_part"]))
    # d gamma / d n = gamma ln(T_ref/T)
    assert np.allclose(G["dn"], np.log(296.0 / T) * L["gamma_ref"] * G["dgamma_ref"], rtol=1e-13, atol=0)
    G0 = oracle.gradient(L, SP, 296.0, P, NU0, DNU, NG, CUT, g)
    assert np.all(G0["dn"] == 0.0)


# ---------------------------------------------------------------- profile derivatives
def _fd_derivs(d, a, g, h=1e-4):
    """Central differences of the oracle's profile in gamma and alpha (relative step h)."""
    hg, ha = h * np.maximum(g, 1e-300), h * a
    dg = (oracle.voigt(d, a, g + hg) - oracle.voigt(d, a, g - hg)) / (2 * hg)
    da = (oracle.voigt(d, a + ha, g) - oracle.voigt(d, a - ha, g)) / (2 * ha)
    return dg, da


@pytest.mark.parametrize("zabs", [12.0, 60.0, 1e3, 1e5, 1e7])
@pytest.mark.parametrize("phase", [0.0, 0.3, 1.2, 1.5])
def test_profile_derivatives_far_wing_vs_central_differences(zabs, phase):
    """Far from the centre the derivatives come from quadrature; central differences of the
    profile itself are well conditioned there (dV/dgamma ~ V/gamma), the closed form is not."""
    a = 0.01
    d = zabs * a * np.cos(phase)
    g = max(zabs * a * np.sin(phase), 1e-3 * a)
    dg, da = oracle.voigt_derivs(d, a, g)
    fg, fa = _fd_derivs(np.array([d]), np.array([a]), np.array([g]))
    assert abs(dg[0] - fg[0]) <= 1e-7 * abs(fg[0]), (dg, fg)
    # dV/dalpha is O(alpha^2/|z|^2) smaller than V/alpha: compare on the scale of V/alpha
    scale = oracle.voigt(d, a, g)[0] / a
    assert abs(da[0] - fa[0]) <= 1e-7 * scale, (da, fa, scale)


def test_profile_derivatives_quadrature_meets_closed_form():
    """On both sides of |z| = 10 the two forms agree (closed form still good to ~1e-13 there)."""
    a = 1.0
    for zabs in (9.999999, 10.000001, 14.0):
        for phase in np.linspace(0.0, np.pi / 2, 7):
            d, g = zabs * np.cos(phase), zabs * np.sin(phase)
            dg, da = oracle.voigt_derivs(d, a, g)
            x, y = d / a, g / a
            w = oracle.faddeeva(x, y)[0]
            K, L = w.real, w.imag
            Kx = -2.0 * (x * K - y * L)
            Ky = 2.0 * (x * L + y * K) - 2.0 / np.sqrt(np.pi)
            cg = Ky / (np.sqrt(np.pi) * a * a)
            ca = -(K + x * Kx + y * Ky) / (np.sqrt(np.pi) * a * a)
            scale = 1.0 / (np.pi * (d * d + g * g))  # size of the Lorentz wing's derivative
            assert abs(dg[0] - cg) <= 1e-11 * scale, (zabs, phase, dg[0], cg)
            assert abs(da[0] - ca) <= 1e-11 * scale, (zabs, phase, da[0], ca)


def test_profile_derivatives_lorentz_and_gauss_limits():
    """alpha -> 0: the Lorentzian's own derivative; gamma = 0 far out: dV/dgamma = 1/(pi delta^2)."""
    d = np.array([0.7, 3.0, 40.0])
    g = np.array([0.05, 0.2, 1.0])
    dg, _ = oracle.voigt_derivs(d, 1e-9, g)
    assert np.allclose(dg, (d * d - g * g) / (np.pi * (d * d + g * g) ** 2), rtol=1e-12, atol=0)
    dg0, da0 = oracle.voigt_derivs(d, 1e-3, 0.0)
    assert np.allclose(dg0, 1.0 / (np.pi * d * d), rtol=1e-5, atol=0)
    assert np.all(np.abs(da0) < 1e-300 + 1e-30)
