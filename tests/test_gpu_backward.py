"""GPU parity of the adjoint (hk_opacity_backward, HkOpacityFn) against the FP64 oracle
gradient and FP64 central differences of the oracle's forward sum, through the C ABI.

Tolerance: per-line gradients max |gpu - oracle| <= 1e-4 max |oracle|; dL/dT and dL/dlnP
within 1e-4 of the oracle value."""
import math

import numpy as np
import pytest

import linegen
import oracle
from gpu_util import TOL_G, _lines, prepare, to_device, upstream, vec_err

pytestmark = pytest.mark.gpu

SP = (18.0, 296.0, 1.0, 0.05, 1.5)


def _gpu_backward(lines, T, P, nu0, dnu, n, cut, g):
    import torch

    import paper_2101_02005_amd as hk
    gd = torch.from_numpy(g).cuda()
    out2, dS, dg, dn = hk.hk_opacity_backward(lines, T, P, hk.grid(nu0, dnu, n), cut, gd)
    torch.cuda.synchronize()
    return out2.cpu().numpy(), dS.cpu().numpy(), dg.cpu().numpy().astype(np.float64), dn.cpu().numpy().astype(np.float64)


def _oracle_grad(L, T, P, nu0, dnu, n, cut, g, sel=None):
    return oracle.gradient(L, oracle.species(*SP), T, P, nu0, dnu, n, cut, g.astype(np.float64), sel=sel)


def _check(L, T, P, nu0, dnu, n, cut, g, label):
    lines = prepare(L, SP)
    out2, dS, dg, dn = _gpu_backward(lines, T, P, nu0, dnu, n, cut, g)
    lines.release()
    go = _oracle_grad(L, T, P, nu0, dnu, n, cut, g)
    dT, dlnP = go["dT_part"].sum(), go["dlnP_part"].sum()
    errs = {"dS_ref": vec_err(dS, go["dS_ref"]), "dgamma_ref": vec_err(dg, go["dgamma_ref"]),
            "dn": vec_err(dn, go["dn"]),
            "dT": abs(out2[0] - dT) / abs(dT) if dT != 0 else abs(out2[0]),
            "dlnP": abs(out2[1] - dlnP) / abs(dlnP) if dlnP != 0 else abs(out2[1])}
    print(label, {k: "%.2e" % v for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL_G, (label, k, v)
    return out2, go


def _c4_subset(N):
    w = linegen.workload("c4")
    assert tuple(w.species_tuple()) == SP
    return w, linegen.generate(w.recipe(), w.seed, N)


def test_c4_subset_vs_oracle_gradient():
    """1e4 lines of the differentiation list on its full grid (0-10000 cm^-1 at 0.01, cut 100)."""
    w, L = _c4_subset(10_000)
    g = upstream(w.n_grid, w.extra["g_seed"])
    _check(L, w.T[0], w.P[0], w.nu_start, w.dnu, w.n_grid, w.cut, g, "c4 subset 1e4")


def test_c4_subset_vs_central_differences():
    """dL/dT and dL/dlnP against FP64 central differences (h = 1e-4 relative) of the oracle's
    L = sum_j g_j k_j on the same 1e4-line subset; per-line dL/dgamma_ref and dL/dn of a few
    lines against central differences of their own line functional."""
    w, L = _c4_subset(10_000)
    g = upstream(w.n_grid, w.extra["g_seed"])
    T, P = w.T[0], w.P[0]
    lines = prepare(L, SP)
    out2, dS, dg, dn = _gpu_backward(lines, T, P, w.nu_start, w.dnu, w.n_grid, w.cut, g)
    lines.release()
    sp = oracle.species(*SP)
    g64 = g.astype(np.float64)

    def Lsum(T_, P_, LL=L):
        return float(np.sum(oracle.line_functional(LL, sp, T_, P_, w.nu_start, w.dnu, w.n_grid, w.cut, g64)))

    h = 1e-4
    fdT = (Lsum(T * (1 + h), P) - Lsum(T * (1 - h), P)) / (2 * h * T)
    fdP = (Lsum(T, P * math.exp(h)) - Lsum(T, P * math.exp(-h))) / (2 * h)
    eT, eP = abs(out2[0] - fdT) / abs(fdT), abs(out2[1] - fdP) / abs(fdP)
    print("central differences: dT %.3e (rel err %.2e), dlnP %.3e (rel err %.2e)" % (fdT, eT, fdP, eP))
    assert eT <= TOL_G and eP <= TOL_G
    # per-line parameters of 12 lines with the largest |dL/dgamma_ref|
    idx = np.argsort(-np.abs(dg))[:12]
    sub = {k: v[idx].copy() for k, v in L.items()}
    for field, gpu in (("gamma_ref", dg[idx]), ("n", dn[idx]), ("S_ref", dS[idx])):
        fd = np.empty(idx.size)
        for q in range(idx.size):
            x0 = sub[field][q]
            step = h * abs(x0)
            vals = []
            for sgn in (1, -1):
                s2 = {k: v[q:q + 1].copy() for k, v in sub.items()}
                s2[field][0] = x0 + sgn * step
                vals.append(oracle.line_functional(s2, sp, T, P, w.nu_start, w.dnu, w.n_grid, w.cut, g64)[0])
            fd[q] = (vals[0] - vals[1]) / (2 * step)
        e = vec_err(gpu, fd)
        print("central differences per line, %s: rel err %.2e" % (field, e))
        assert e <= TOL_G, field


BWD_EDGE = [
    # (name, lines, T, P, nu_start, dnu, n, cut)
    ("one line on a grid point", _lines([50.0]), 1000.0, 1.0, 0.0, 0.1, 1000, 25.0),
    ("line beyond the grid end within the cut", _lines([102.3]), 800.0, 0.5, 0.0, 0.1, 1000, 25.0),
    ("no cut", _lines(np.linspace(3.0, 180.0, 37)), 1500.0, 2.0, 0.0, 0.05, 4000, np.inf),
    ("narrow Doppler lines, unsampled peaks", _lines(np.linspace(5.0, 60.0, 300) + 0.0013, g=0.03),
     100.0, 1e-6, 0.0, 0.01, 7000, 10.0),
    ("zero pressure (pure Gaussian)", _lines(np.linspace(500.0, 520.0, 50)), 1000.0, 0.0, 490.0, 0.001, 30000, 3.0),
    ("very broad Lorentz lines", _lines(np.linspace(100.0, 300.0, 100)), 100.0, 100.0, 0.0, 0.01, 40000, 100.0),
    ("ragged chunks, cut shorter than a wave", _lines(np.linspace(10.0, 11.0, 77)), 300.0, 1.0, 9.0, 0.005, 600, 0.2),
    ("high-E lines at low T", _lines(np.linspace(1000.0, 1010.0, 40), E=np.linspace(0, 20000, 40), S=1e-22),
     150.0, 1.0, 990.0, 0.01, 3000, 25.0),
]


@pytest.mark.parametrize("case", BWD_EDGE, ids=[c[0] for c in BWD_EDGE])
def test_backward_edge_cases(case):
    name, L, T, P, nu0, dnu, n, cut = case
    g = upstream(n, 11)
    if P == 0.0:
        lines = prepare(L, SP)
        out2, dS, dg, dn = _gpu_backward(lines, T, P, nu0, dnu, n, cut, g)
        lines.release()
        go = _oracle_grad(L, T, P, nu0, dnu, n, cut, g)
        assert vec_err(dS, go["dS_ref"]) <= TOL_G
        assert abs(out2[0] - go["dT_part"].sum()) <= TOL_G * abs(go["dT_part"].sum())
        assert out2[1] == 0.0 and np.all(dn == 0.0)  # gamma = 0: no pressure or n dependence
    else:
        _check(L, T, P, nu0, dnu, n, cut, g, name)


def test_backward_lines_outside_grid_get_zero():
    L = _lines([5000.0, 6000.0])
    g = upstream(1000, 3)
    lines = prepare(L, SP)
    out2, dS, dg, dn = _gpu_backward(lines, 800.0, 1.0, 0.0, 0.1, 1000, 25.0, g)
    lines.release()
    assert np.all(out2 == 0) and np.all(dS == 0) and np.all(dg == 0) and np.all(dn == 0)


def test_autograd_function_matches_abi_and_is_deterministic():
    import torch

    import paper_2101_02005_amd as hk
    w, L = _c4_subset(20_000)
    d = to_device(L)
    g = torch.from_numpy(upstream(w.n_grid, w.extra["g_seed"])).cuda()
    grd = hk.grid(w.nu_start, w.dnu, w.n_grid)
    lines = prepare(L, SP)
    T = torch.tensor(w.T[0], dtype=torch.float64, requires_grad=True)
    lnP = torch.tensor(math.log(w.P[0]), dtype=torch.float64, requires_grad=True)
    S = d["S_ref"].clone().requires_grad_(True)
    gr = d["gamma_ref"].clone().requires_grad_(True)
    nx = d["n"].clone().requires_grad_(True)
    k = hk.opacity(lines, T, lnP, grd, w.cut, S_ref=S, gamma_ref=gr, n_exp=nx)
    Pv = math.exp(math.log(w.P[0]))  # the pressure the function sees
    k_plain = hk.hk_opacity(lines, w.T[0], Pv, grd, w.cut)
    assert torch.equal(k, k_plain)
    (k.double() * g.double()).sum().backward()
    out2, dS, dg, dn = hk.hk_opacity_backward(lines, w.T[0], Pv, grd, w.cut, g)
    out2b, dSb, dgb, dnb = hk.hk_opacity_backward(lines, w.T[0], Pv, grd, w.cut, g)
    torch.cuda.synchronize()
    assert torch.equal(out2, out2b) and torch.equal(dS, dSb) and torch.equal(dg, dgb) and torch.equal(dn, dnb)
    assert T.grad.item() == out2[0].item() and lnP.grad.item() == out2[1].item()
    assert torch.equal(S.grad, dS) and torch.equal(gr.grad, dg.double()) and torch.equal(nx.grad, dn.double())
    # identities of the chain rule: L = sum S_ref dL/dS_ref, dL/dlnP = sum gamma_ref dL/dgamma_ref
    Lk = float((k.detach().double() * g.double()).sum())
    LS = float((S.detach() * S.grad).sum())
    assert abs(LS - Lk) <= 1e-4 * abs(Lk)
    assert abs(float((gr.detach() * gr.grad).sum()) - out2[1].item()) <= 1e-4 * abs(out2[1].item())
    lines.release()


def test_override_changes_gradient_like_oracle():
    """Per-line overrides (S_ref, gamma_ref, n) reach both passes."""
    import torch

    import paper_2101_02005_amd as hk
    w, L = _c4_subset(2_000)
    g = upstream(200_000, 5)
    nu0, dnu, n, cut = 0.0, 0.05, 200_000, 50.0
    L2 = {k: v.copy() for k, v in L.items()}
    rng = np.random.default_rng(9)
    L2["S_ref"] *= rng.uniform(0.5, 2.0, L2["S_ref"].size)
    L2["gamma_ref"] *= rng.uniform(0.5, 2.0, L2["gamma_ref"].size)
    L2["n"] = rng.uniform(0.3, 0.9, L2["n"].size)
    lines = prepare(L, SP)
    d2 = to_device(L2)
    ovr = (d2["S_ref"], d2["gamma_ref"], d2["n"])
    out2, dS, dg, dn = hk.hk_opacity_backward(lines, 900.0, 0.3, hk.grid(nu0, dnu, n), cut,
                                              torch.from_numpy(g).cuda(), ovr=ovr)
    torch.cuda.synchronize()
    lines.release()
    go = _oracle_grad(L2, 900.0, 0.3, nu0, dnu, n, cut, g)
    assert vec_err(dS.cpu().numpy(), go["dS_ref"]) <= TOL_G
    assert vec_err(dg.cpu().numpy().astype(np.float64), go["dgamma_ref"]) <= TOL_G
    assert vec_err(dn.cpu().numpy().astype(np.float64), go["dn"]) <= TOL_G
    assert abs(out2[0].item() - go["dT_part"].sum()) <= TOL_G * abs(go["dT_part"].sum())


def test_c4_full_list_sampled_lines_and_identities():
    """The full differentiation list (1e7 lines, 0-10000 cm^-1 at 0.01, cut 100): per-line
    gradients of 300 sampled lines against the oracle, and the chain-rule identities
    sum S_ref dL/dS_ref = L = sum_j g_j k_j and dL/dlnP = sum gamma_ref dL/dgamma_ref."""
    import torch

    import paper_2101_02005_amd as hk
    w = linegen.workload("c4")
    dev = [torch.empty(w.N, dtype=torch.float64, device="cuda") for _ in range(5)]
    linegen.generate_device(w.recipe(), w.seed, w.N, [t.data_ptr() for t in dev],
                            stream=torch.cuda.current_stream().cuda_stream)
    lines = hk.hk_prepare_lines(*dev, hk.species(*w.species_tuple()))
    grd = hk.grid(w.nu_start, w.dnu, w.n_grid)
    g = upstream(w.n_grid, w.extra["g_seed"])
    gd = torch.from_numpy(g).cuda()
    out2, dS, dg, dn = hk.hk_opacity_backward(lines, w.T[0], w.P[0], grd, w.cut, gd)
    k = hk.hk_opacity(lines, w.T[0], w.P[0], grd, w.cut)
    torch.cuda.synchronize()
    Lk = float((k.double() * gd.double()).sum())
    LS = float((dev[1] * dS).sum())
    lnP = float((dev[3] * dg.double()).sum())
    print("L %.6e  sum S dL/dS %.6e  dL/dlnP %.6e  sum g dL/dg %.6e  dL/dT %.6e" % (Lk, LS, out2[1].item(), lnP,
                                                                                 out2[0].item()))
    assert abs(LS - Lk) <= 1e-4 * abs(Lk)
    assert abs(lnP - out2[1].item()) <= 1e-4 * abs(out2[1].item())
    rng = np.random.default_rng(44)
    sel = np.sort(rng.choice(w.N, 300, replace=False))
    L = {kk: t.cpu().numpy()[sel] for kk, t in zip(linegen.FIELDS, dev)}
    lines.release()
    go = _oracle_grad(L, w.T[0], w.P[0], w.nu_start, w.dnu, w.n_grid, w.cut, g)
    for name, gpu in (("dS_ref", dS.cpu().numpy()[sel]), ("dgamma_ref", dg.cpu().numpy()[sel].astype(np.float64)),
                      ("dn", dn.cpu().numpy()[sel].astype(np.float64))):
        e = vec_err(gpu, go[name])
        print("c4 full list, 300 sampled lines, %s: rel err %.2e" % (name, e))
        assert e <= TOL_G, name
