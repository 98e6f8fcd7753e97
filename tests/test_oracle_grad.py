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
