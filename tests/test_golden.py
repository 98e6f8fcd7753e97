"""Regression pins against stored values: the paper's printed constants, and the oracle's
own c1 opacity written by tests/golden/make_golden.py (guards against unintended changes
of the oracle)."""
import os
import re

import numpy as np

import linegen
import oracle

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_paper_constants_in_oracle_source():
    src = open(os.path.join(os.path.dirname(GOLD), "..", "oracle", "oracle.c")).read()
    vals = {}
    for line in open(os.path.join(GOLD, "paper_constants.txt")):
        if line.startswith("#") or not line.strip():
            continue
        key, val = line.split()[:2]
        vals[key] = float(val)
    kb = float(re.search(r"OR_KB = ([0-9.e+-]+);", src).group(1))
    c = float(re.search(r"OR_CLIGHT = ([0-9.e+-]+);", src).group(1))
    assert kb == vals["k_B_erg_per_K"] and c == vals["c_cm_per_s"]


def test_oracle_c1_regression():
    data = np.loadtxt(os.path.join(GOLD, "c1_oracle_k.txt"))
    pts, ref = data[:, 0].astype(np.int64), data[:, 1]
    w = linegen.workload("c1")
    L = linegen.generate(w.recipe(), w.seed, w.N)
    k = oracle.opacity(L, oracle.species(*w.species_tuple()), w.T[0], w.P[0], w.nu_start, w.dnu, w.cut, pts)
    assert np.max(np.abs(k - ref)) <= 1e-13 * ref.max()
