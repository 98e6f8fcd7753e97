"""The five workloads: synthetic line lists shaped like the paper's (input recipe).

The paper's timings (Sec. 3.5, Tables timing0-timing2) use the ExoMol BT2 water list, which
is not available here; the large list below is a synthetic stand-in with the same
wavenumber range and a density rising toward the infrared. All fields are drawn by
``linegen_core.h``; S_ref follows the "scale reading": the drawn log10 value s is the
line's temperature-independent intensity scale, so S_ref = 10^s e^{-c2 E''/T_ref}
(1 - e^{-c2 nu/T_ref}) and S(T) never exceeds 10^s_hi (a literal reading of independent
S_ref and E'' draws overflows FP32 at high T).
"""
from dataclasses import dataclass, field
from typing import Tuple

import numpy as np


@dataclass
class Workload:
    name: str
    N: int
    seed: int
    nu_law: int            # 0 uniform [nu_lo, nu_hi), 1 nu_hi*u^2
    nu_lo: float
    nu_hi: float
    s_lo: float
    s_hi: float
    e_law: int             # 0 exponential(mean e_par), 1 uniform [0, e_par)
    e_par: float
    g_lo: float
    g_hi: float
    n_lo: float = 0.4
    n_hi: float = 0.8
    mass_amu: float = 18.0
    T_ref: float = 296.0
    P_ref: float = 1.0
    q_a: float = 0.05
    q_b: float = 1.5
    T: Tuple[float, ...] = (1000.0,)
    P: Tuple[float, ...] = (1.0,)
    nu_start: float = 0.0
    nu_end: float = 2000.0
    dnu: float = 0.1
    cut: float = 25.0
    s_reading: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def n_grid(self):
        # half-open [nu_start, nu_end)
        return int(round((self.nu_end - self.nu_start) / self.dnu))

    def recipe(self, s_reading=None):
        from . import Recipe
        return Recipe(self.nu_law, self.e_law, self.s_reading if s_reading is None else s_reading, 0,
                      self.nu_lo, self.nu_hi, self.s_lo, self.s_hi, self.e_par, self.g_lo, self.g_hi,
                      self.n_lo, self.n_hi, self.T_ref)

    def species_tuple(self):
        return (self.mass_amu, self.T_ref, self.P_ref, self.q_a, self.q_b)


def _logspace(a, b, n):
    return tuple(float(v) for v in np.logspace(np.log10(a), np.log10(b), n))


CONFIGS = {
    # plain method, small
    "c1": Workload("c1_small_1e4", 10_000, 1, 0, 100.0, 2000.0, -26.0, -19.0, 0, 2000.0, 0.02, 0.1,
                   T=(1000.0,), P=(1.0,), nu_start=0.0, nu_end=2000.0, dnu=0.1, cut=25.0),
    # large molecular list (BT2-like stand-in), plain path; cut 25 (and 100), 0.01 (and 0.1) cm^-1
    "c2": Workload("c2_large_5e8", 500_000_000, 2, 1, 0.0, 30000.0, -26.0, -19.0, 0, 4000.0, 0.02, 0.1,
                   T=(1500.0,), P=(1.0,), nu_start=0.0, nu_end=30000.0, dnu=0.01, cut=25.0),
    # batched (T, P): 20 T log 100-3000 K x 15 P log 1e-6-1e2 atm, one list of 1e7 lines
    "c3": Workload("c3_batched_1e7", 10_000_000, 3, 1, 0.0, 10000.0, -26.0, -19.0, 0, 4000.0, 0.02, 0.1,
                   T=_logspace(100.0, 3000.0, 20), P=_logspace(1e-6, 1e2, 15), nu_start=0.0,
                   nu_end=10000.0, dnu=0.01, cut=100.0),
    # differentiation: the c3 list at 800 K, 0.1 atm
    "c4": Workload("c4_grad_1e7", 10_000_000, 3, 1, 0.0, 10000.0, -26.0, -19.0, 0, 4000.0, 0.02, 0.1,
                   T=(800.0,), P=(0.1,), nu_start=0.0, nu_end=10000.0, dnu=0.01, cut=100.0,
                   extra={"g_seed": 4}),
    # precision: atom-like uncut profiles
    "c5": Workload("c5_uncut_2e5", 200_000, 5, 0, 1000.0, 100000.0, -30.0, -14.0, 1, 100000.0, 0.01, 0.5,
                   mass_amu=56.0, T=(4000.0,), P=(10.0,), nu_start=1000.0, nu_end=100000.0, dnu=0.01,
                   cut=float("inf")),
}


def workload(name, **overrides):
    import dataclasses
    return dataclasses.replace(CONFIGS[name], **overrides)
