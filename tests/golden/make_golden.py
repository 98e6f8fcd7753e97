"""Writes tests/golden/c1_oracle_k.txt: the FP64 oracle's k at every 100th grid point of the
small workload (1e4 lines, 0-2000 cm^-1 at 0.1 cm^-1, cut 25 cm^-1, T = 1000 K, P = 1 atm).

Calls only oracle/ (and the seeded input generator). Rerun only when the oracle's arithmetic
changes for a reason stated in the commit message."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import linegen  # noqa: E402
import oracle  # noqa: E402


def main():
    w = linegen.workload("c1")
    L = linegen.generate(w.recipe(), w.seed, w.N)
    sp = oracle.species(*w.species_tuple())
    pts = np.arange(0, w.n_grid, 100)
    k = oracle.opacity(L, sp, w.T[0], w.P[0], w.nu_start, w.dnu, w.cut, pts)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_oracle_k.txt")
    with open(out, "w") as f:
        f.write("# FP64 oracle opacity k [cm^2/molecule], workload c1 (seed 1, 1e4 lines, scale reading),\n")
        f.write("# T=1000 K, P=1 atm, grid nu_j = 0 + 0.1 j, cut 25 cm^-1 (inclusive). Written by make_golden.py.\n")
        f.write("# j k_j\n")
        for j, v in zip(pts, k):
            f.write("%d %.17e\n" % (j, v))


if __name__ == "__main__":
    main()
