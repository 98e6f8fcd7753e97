"""GPU parity of HITRAN-style lists against the FP64 oracle, through the C ABI: air and self
broadening (eq. gammaL without the natural term) and the pressure shift of line centres
(Table binary2), which makes each call bin the list again by the shifted centres."""
import numpy as np
import pytest

import oracle
from gpu_util import TOL_K, to_device

pytestmark = pytest.mark.gpu

SP = (18.0, 296.0, 1.0, 0.05, 1.5)


def _hitran_list(N, seed, lo=100.0, hi=2000.0, dmax=0.02):
    """Seeded synthetic list with the c1 distributions plus self widths and shifts (the shift
    range reorders close lines at high pressure)."""
    rng = np.random.default_rng(seed)
    s = rng.uniform(-26.0, -19.0, N)
    nu = rng.uniform(lo, hi, N)
    E = rng.exponential(2000.0, N)
    c2 = 1.438776855773617
    Sref = 10 ** s * np.exp(-c2 * E / 296.0) * (-np.expm1(-c2 * nu / 296.0))
    return {"nu": nu, "S_ref": Sref, "E": E, "gamma_air": rng.uniform(0.02, 0.1, N),
            "gamma_self": rng.uniform(0.1, 0.5, N), "n": rng.uniform(0.4, 0.8, N),
            "delta": rng.uniform(-dmax, 0.5 * dmax, N)}


def _prepare(L):
    import paper_2101_02005_amd as hk
    d = to_device(L)
    return hk.hk_prepare_lines_hitran(d["nu"], d["S_ref"], d["E"], d["gamma_air"], d["gamma_self"], d["n"],
                                      d["delta"], hk.species(*SP))


GRIDS = {"c1": (0.0, 0.1, 20_000), "fine": (1000.0, 0.001, 20_000)}


@pytest.mark.parametrize("grid", sorted(GRIDS))
@pytest.mark.parametrize("P,P_self", [(1.0, 0.0), (30.0, 3.0), (5.0, 5.0), (0.0, 0.0)])
@pytest.mark.parametrize("profile,cut_mode,cutoff,plinth", [(0, 0, 25.0, 0), (0, 2, 200.0, 1), (1, 0, 10.0, 1),
                                                            (3, 1, 30.0, 0)])
def test_hitran_vs_oracle(profile, cut_mode, cutoff, plinth, P, P_self, grid):
    import paper_2101_02005_amd as hk
    L = _hitran_list(10_000, 41)
    lines = _prepare(L)
    g = GRIDS[grid]
    T = 1000.0
    opts = hk.options(profile=profile, cut_mode=cut_mode, plinth=plinth)
    k = hk.hk_opacity_hitran(lines, T, P, P_self, hk.grid(*g), cutoff, opts=opts).cpu().numpy().astype(np.float64)
    lines.release()
    pts = np.arange(g[2])
    sp = oracle.species(*SP)
    ko = oracle.opacity_hitran(L, sp, T, P, P_self, g[0], g[1], cutoff, pts, cut_mode=cut_mode, profile=profile,
                               plinth=plinth)
    scale = ko.max() if not plinth else oracle.opacity_hitran(L, sp, T, P, P_self, g[0], g[1], cutoff, pts,
                                                              cut_mode=cut_mode, profile=profile, plinth=0).max()
    if scale <= 0:  # P = 0 with a Lorentzian: nothing anywhere
        assert np.all(k == 0.0) and np.all(ko == 0.0)
        return
    e = float(np.max(np.abs(k - ko)) / scale)
    print("hitran profile %d cut %d plinth %d P=%g P_self=%g grid %s: %.3e" % (profile, cut_mode, plinth, P, P_self,
                                                                                grid, e))
    assert e <= TOL_K


def test_no_shift_equal_widths_match_plain_handle():
    """delta = 0 and gamma_self = gamma_air: the same k as the ExoMol-form handle's options path."""
    import paper_2101_02005_amd as hk
    L = _hitran_list(10_000, 42)
    L["delta"][:] = 0.0
    L["gamma_self"] = L["gamma_air"].copy()
    lines = _prepare(L)
    d = to_device({"nu": L["nu"], "S_ref": L["S_ref"], "E": L["E"], "g": L["gamma_air"], "n": L["n"]})
    plain = hk.hk_prepare_lines(d["nu"], d["S_ref"], d["E"], d["g"], d["n"], hk.species(*SP))
    g = hk.grid(0.0, 0.05, 40_000)
    opts = hk.options(plinth=1)
    a = hk.hk_opacity_hitran(lines, 700.0, 2.0, 0.7, g, 25.0, opts=opts).double()
    b = hk.hk_opacity(plain, 700.0, 2.0, g, 25.0, opts=opts).double()
    assert (a - b).abs().max().item() <= 1e-6 * b.abs().max().item()
    lines.release()
    plain.release()


def test_shift_reorders_and_large_list_windows():
    """3e5 lines over 100 cm^-1 with shifts up to 0.5 cm^-1 at 50 atm (centres reorder across many
    bins), on a 1e6-point grid: sampled windows against the oracle."""
    import paper_2101_02005_amd as hk
    L = _hitran_list(300_000, 43, 1000.0, 1100.0, dmax=0.01)
    lines = _prepare(L)
    g = (990.0, 0.000125, 1_000_000)
    k = hk.hk_opacity_hitran(lines, 1500.0, 50.0, 10.0, hk.grid(*g), 5.0).cpu().numpy().astype(np.float64)
    lines.release()
    sp = oracle.species(*SP)
    rng = np.random.default_rng(44)
    for s0 in [0, int(np.argmax(k)) - 16, g[2] - 32] + list(rng.integers(0, g[2] - 32, 6)):
        s0 = min(max(int(s0), 0), g[2] - 32)
        pts = np.arange(s0, s0 + 32)
        ko = oracle.opacity_hitran(L, sp, 1500.0, 50.0, 10.0, g[0], g[1], 5.0, pts)
        if ko.max() == 0.0:  # no line within the cut of the window: exactly zero
            assert np.all(k[pts] == 0.0), s0
            continue
        e = float(np.max(np.abs(k[pts] - ko)) / ko.max())
        assert e <= TOL_K, (s0, e)


def test_hitran_invalid_arguments():
    import paper_2101_02005_amd as hk
    L = _hitran_list(1000, 45)
    lines = _prepare(L)
    g = hk.grid(0.0, 0.1, 1000)
    with pytest.raises(hk.HkError) as ei:
        hk.hk_opacity_hitran(lines, 500.0, 1.0, 2.0, g, 25.0)  # P_self > P
    assert ei.value.status == hk.HK_EINVAL
    with pytest.raises(hk.HkError):
        hk.hk_opacity_hitran(lines, 500.0, 1.0, 0.5, g, 25.0, opts=hk.options(direct=1))
    lines.release()
    d = to_device({k: L[k] for k in ("nu", "S_ref", "E", "gamma_air", "n")})
    plain = hk.hk_prepare_lines(d["nu"], d["S_ref"], d["E"], d["gamma_air"], d["n"], hk.species(*SP))
    with pytest.raises(hk.HkError) as ei:
        hk.hk_opacity_hitran(plain, 500.0, 1.0, 0.5, g, 25.0)  # not a HITRAN-style handle
    assert ei.value.status == hk.HK_EINVAL
    plain.release()
    bad = dict(L)
    bad["gamma_self"] = L["gamma_self"].copy()
    bad["gamma_self"][17] = -0.1
    with pytest.raises(hk.HkError) as ei:
        _prepare(bad)
    assert ei.value.status == hk.HK_EINVAL
