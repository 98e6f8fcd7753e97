"""Helpers shared by the GPU tests: move seeded line lists to the device, run the HIP path
through the C ABI, and compare with the FP64 oracle."""
import numpy as np

import linegen
import oracle

TOL_K = 1e-5  # max |k_gpu - k_oracle| <= TOL_K * max k_oracle over the compared points
TOL_G = 1e-4  # per-line gradients: max |gpu - oracle| <= TOL_G * max |oracle|; scalars: <= TOL_G * |oracle|


def to_device(L):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).cuda() for k, v in L.items()}


def prepare(L, sp_tuple):
    import paper_2101_02005_amd as hk
    d = to_device(L)
    return hk.hk_prepare_lines(d["nu"], d["S_ref"], d["E"], d["gamma_ref"], d["n"], hk.species(*sp_tuple))


def gpu_k(lines, T, P, nu_start, dnu, n, cut):
    import paper_2101_02005_amd as hk
    k = hk.hk_opacity(lines, T, P, hk.grid(nu_start, dnu, n), cut)
    return k.cpu().numpy().astype(np.float64)


def oracle_k(L, sp_tuple, T, P, nu_start, dnu, cut, pts):
    return oracle.opacity(L, oracle.species(*sp_tuple), T, P, nu_start, dnu, cut, pts)


def rel_err(k, ko):
    m = ko.max()
    return float(np.max(np.abs(k - ko)) / m) if m > 0 else float(np.max(np.abs(k)))


def workload_lines(name, **kw):
    w = linegen.workload(name, **kw)
    return w, linegen.generate(w.recipe(), w.seed, w.N)


def _lines(nu, S=1e-20, E=500.0, g=0.05, n=0.5):
    """A small hand-made line list (constant fields unless arrays are given)."""
    nu = np.atleast_1d(np.asarray(nu, dtype=np.float64))
    N = nu.size
    f = lambda v: np.full(N, v, dtype=np.float64) if np.isscalar(v) else np.asarray(v, dtype=np.float64)
    return {"nu": nu, "S_ref": f(S), "E": f(E), "gamma_ref": f(g), "n": f(n)}


def upstream(n, seed):
    """Seeded dL/dk ~ N(0, 1) in float32 (the upstream gradient of the differentiation workload)."""
    return np.random.default_rng(seed).standard_normal(n).astype(np.float32)


def vec_err(a, ao):
    m = np.max(np.abs(ao))
    return float(np.max(np.abs(a - ao)) / m) if m > 0 else float(np.max(np.abs(a)))
