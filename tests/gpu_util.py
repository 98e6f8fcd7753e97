"""Helpers shared by the GPU tests: move seeded line lists to the device, run the HIP path
through the C ABI, and compare with the FP64 oracle."""
import numpy as np

import linegen
import oracle

TOL_K = 1e-5  # max |k_gpu - k_oracle| <= TOL_K * max k_oracle over the compared points


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
