"""The synthetic input generator: counter-based uniforms, distributions, host selection."""
import numpy as np

import linegen


def _splitmix64_py(z):
    M = (1 << 64) - 1
    z = (z + 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def test_splitmix64_reference_value():
    # first output of SplitMix64 started from state 0 (published reference sequence)
    assert _splitmix64_py(0) == 0xE220A8397B1DCDAF


def test_uniforms_match_definition():
    seed, f = 12345, 3
    u = linegen.uniforms(seed, 1000, 64, f)
    M = (1 << 64) - 1
    for k in range(64):
        i = 1000 + k
        h = _splitmix64_py(seed ^ ((i * 0x9E3779B97F4A7C15) & M) ^ ((f * 0xD1B54A32D192ED03) & M))
        assert u[k] == (h >> 11) * 2.0 ** -53 + 2.0 ** -54
    assert np.all((u > 0) & (u < 1))


def test_distributions():
    w = linegen.workload("c2")
    L = linegen.generate(w.recipe(), w.seed, 200000)
    nu = L["nu"]
    assert nu.min() >= 0 and nu.max() < 30000
    # nu = 30000 u^2 -> P(nu < x) = sqrt(x/30000)
    assert abs(np.mean(nu < 7500.0) - 0.5) < 0.01
    assert abs(L["E"].mean() - 4000.0) < 60.0
    assert np.all((L["gamma_ref"] >= 0.02) & (L["gamma_ref"] < 0.1))
    assert np.all((L["n"] >= 0.4) & (L["n"] < 0.8))
    assert np.all(L["S_ref"] > 0) and np.all(L["S_ref"] <= 1e-19)


def test_select_consistent_with_generate():
    w = linegen.workload("c1")
    L = linegen.generate(w.recipe(), w.seed, w.N)
    idx, S = linegen.select(w.recipe(), w.seed, w.N, 700.0, 720.0)
    m = np.nonzero((L["nu"] >= 700.0) & (L["nu"] < 720.0))[0]
    assert np.array_equal(idx, m)
    for k in linegen.FIELDS:
        assert np.array_equal(S[k], L[k][m])


def test_generator_math_helpers():
    x = np.linspace(-700, 700, 20001)
    assert np.max(np.abs(linegen.math_helper("exp", x) / np.exp(x) - 1)) < 1e-15
    x = np.linspace(-0.9, 0.9, 20001)
    x = x[x != 0]
    assert np.max(np.abs(linegen.math_helper("expm1", x) / np.expm1(x) - 1)) < 1e-15
    x = 10 ** np.linspace(-300, 300, 20001)
    assert np.max(np.abs(linegen.math_helper("log", x) - np.log(x)) / np.maximum(1, np.abs(np.log(x)))) < 1e-15
