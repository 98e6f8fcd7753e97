"""GPU parity of the options path against the FP64 oracle, through the C ABI: the four line
profiles of Sec. 2.1 (Voigt, Lorentz, Doppler, binned Gaussian), plinth removal (Sec. 2.1.1)
and cutting lengths that are multiples of each line's Doppler or Lorentz half-width (Sec. 2.4.3
step 4); per-line cut bounds exact against the oracle's cutting lengths; the batched form with
options against plain calls; the direct-evaluation mode of the default path; the evaluation
classes of the default path (each one exercised, with a stress case where lines evaluated at
Chebyshev nodes dominate k); and the work-item overflow flag."""
import os

import numpy as np
import pytest

import linegen
import oracle
from gpu_util import TOL_K, _lines, prepare, rel_err, workload_lines

pytestmark = pytest.mark.gpu

SP = (18.0, 296.0, 1.0, 0.05, 1.5)
PROFILES = {"voigt": 0, "lorentz": 1, "doppler": 2, "binned": 3}
# cutoff per cut mode: a length in cm^-1, or the multiple of the Doppler / Lorentz half-width
CUTS = {"fixed": (0, 25.0), "doppler": (1, 500.0), "doppler_near": (1, 4.0), "lorentz": (2, 100.0)}
# the same for the per-line records: lengths at which every profile's plinth is far from zero
CUTS_REC = {"fixed": (0, 0.01), "doppler": (1, 3.0), "lorentz": (2, 20.0)}
GRIDS = {"c1": (0.0, 0.1, 20_000), "fine": (1000.0, 0.001, 20_000)}


class _env:
    """Temporarily set environment variables read by the library on each call."""

    def __init__(self, **kv):
        self.kv = {k: str(v) for k, v in kv.items()}

    def __enter__(self):
        self.old = {k: os.environ.get(k) for k in self.kv}
        os.environ.update(self.kv)

    def __exit__(self, *exc):
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _oracle_ex(L, T, P, g, cutoff, cut_mode, profile, plinth, pts):
    return oracle.opacity_ex(L, oracle.species(*SP), T, P, g[0], g[1], cutoff, pts, cut_mode=cut_mode,
                             profile=profile, plinth=plinth)


@pytest.mark.parametrize("grid", sorted(GRIDS))
@pytest.mark.parametrize("plinth", [0, 1])
@pytest.mark.parametrize("cut", sorted(CUTS))
@pytest.mark.parametrize("profile", sorted(PROFILES))
def test_profiles_cut_modes_plinth_c1(profile, cut, plinth, grid):
    import paper_2101_02005_amd as hk
    w, L = workload_lines("c1")
    lines = prepare(L, SP)
    mode, cutoff = CUTS[cut]
    g = GRIDS[grid]
    opts = hk.options(profile=PROFILES[profile], cut_mode=mode, plinth=plinth)
    k = hk.hk_opacity(lines, 1000.0, 1.0, hk.grid(*g), cutoff, opts=opts).cpu().numpy().astype(np.float64)
    lines.release()
    pts = np.arange(g[2])
    ko = _oracle_ex(L, 1000.0, 1.0, g, cutoff, mode, PROFILES[profile], plinth, pts)
    # the scale: max k without plinth removal (the removal can cancel a line's values to nearly
    # zero, e.g. a binned Gaussian cut inside its own bin; the error is relative to the terms)
    scale = ko.max() if not plinth else _oracle_ex(L, 1000.0, 1.0, g, cutoff, mode, PROFILES[profile], 0, pts).max()
    e = float(np.max(np.abs(k - ko)) / scale)
    print("%s cut=%s plinth=%d grid=%s: max |k - k_orc| / max k_orc(no plinth) = %.3e" % (profile, cut, plinth, grid,
                                                                                          e))
    assert np.all(np.isfinite(k))
    assert e <= TOL_K
    # no line reaches a point outside the union of its cut: exact zero there
    assert np.all(k[ko == 0.0] == 0.0) or plinth


def _bounds_ok(nu, c, nu_start, dnu, n, jlo, jhi):
    """Per line: [jlo, jhi] is exactly the set of grid points with |nu_start + j dnu - nu| <= c."""
    def inside(j):
        jj = np.clip(j, 0, n - 1)
        v = np.abs((nu_start + jj.astype(np.float64) * dnu) - nu) <= c
        return v & (j >= 0) & (j <= n - 1)
    nonempty = jlo <= jhi
    ok = np.ones(nu.size, dtype=bool)
    ok &= ~nonempty | (inside(jlo) & inside(jhi) & ~inside(jlo - 1) & ~inside(jhi + 1))
    # empty ranges: no grid point within the cut (the nearest candidates fail the predicate)
    j0 = np.floor((nu - nu_start) / dnu).astype(np.int64)
    for d in (-1, 0, 1, 2):
        ok &= nonempty | ~inside(j0 + d)
    for j in (0, n - 1):  # lines beyond either end of the grid
        ok &= nonempty | ~inside(np.full(nu.size, j, dtype=np.int64))
    return ok


@pytest.mark.parametrize("cut", ["doppler", "lorentz", "fixed"])
@pytest.mark.parametrize("profile", sorted(PROFILES))
def test_grid_records_exact(profile, cut):
    """Per-line cut bounds equal the oracle's predicate on its own cutting lengths; plinth values
    S(T) f(cut) within FP32 rounding of the oracle's."""
    import paper_2101_02005_amd as hk
    from scipy import special
    w, L = workload_lines("c1", N=20_000)
    lines = prepare(L, SP)
    mode, cutoff = CUTS_REC[cut]
    T, P = 700.0, 3.0
    g = GRIDS["fine"]
    opts = hk.options(profile=PROFILES[profile], cut_mode=mode, plinth=1)
    lo, hi, pl = (x.cpu().numpy() for x in hk.hk_debug_grid_records(lines, T, P, hk.grid(*g), cutoff, opts))
    lines.release()
    sp = oracle.species(*SP)
    c = oracle.cut_lengths(L, sp, T, P, mode, cutoff)
    assert np.all(_bounds_ok(L["nu"], c, g[0], g[1], g[2], lo.astype(np.int64), hi.astype(np.int64)))
    S, a, gam = oracle.line_params(L, sp, T, P)
    if profile == "voigt":
        f = oracle.voigt(c, a, gam)
    elif profile == "lorentz":
        f = gam / (np.pi * (c * c + gam * gam))
    elif profile == "doppler":
        f = np.exp(-(c / a) ** 2) / (np.sqrt(np.pi) * a)
    else:
        f = (special.erfc((c - 0.5 * g[1]) / a) - special.erfc((c + 0.5 * g[1]) / a)) / (2 * g[1])
    expect = np.where(lo <= hi, S * f, 0.0)
    scale = np.maximum(np.abs(expect), 1e-300)
    big = np.abs(expect) > 1e-37  # FP32 normal range
    if not (profile in ("doppler", "binned") and cut == "lorentz"):  # there the Gaussian is 0 at the cut
        assert big.sum() > 0.5 * (lo <= hi).sum()  # most lines with points carry a plinth worth checking
    if big.any():
        assert np.max(np.abs(pl[big] - expect[big]) / scale[big]) < 2e-6
    assert np.all(np.abs(pl[~big]) <= 2e-37)


def test_options_batched_matches_plain_and_oracle():
    import torch

    import paper_2101_02005_amd as hk
    w, L = workload_lines("c3", N=300_000)
    lines = prepare(L, w.species_tuple())
    T = [300.0, 1200.0, 2500.0]
    P = [0.01, 1.0, 20.0]
    grids = [hk.grid(0.0, 0.01, 300_000), hk.grid(500.0, 0.005, 100_000), hk.grid(0.0, 0.05, 200_000)]
    opts = hk.options(profile=0, cut_mode=2, plinth=1)
    cutoff = 200.0
    with _env(HK_SLOTS=2):
        kb = hk.hk_opacity_batched(lines, T, P, grids, cutoff, opts=opts).clone()
        off = 0
        for t, pr, g in zip(T, P, grids):
            # within FP32 accumulation tolerance (the batch may split work items differently)
            kp = hk.hk_opacity(lines, t, pr, g, cutoff, opts=opts).double()
            ref = kb[off:off + g.n].double()
            assert (kp - ref).abs().max().item() <= 1e-6 * ref.abs().max().item(), (t, pr)
            off += g.n
    lines.release()
    kb = kb.cpu().numpy().astype(np.float64)
    off = 0
    rng = np.random.default_rng(7)
    for t, pr, g in zip(T, P, grids):
        kp = kb[off:off + g.n]
        for s0 in sorted(set([0, int(np.argmax(kp)) - 8, g.n - 16] + list(rng.integers(0, g.n - 16, 3)))):
            s0 = min(max(s0, 0), g.n - 16)
            pts = np.arange(s0, s0 + 16)
            ko = oracle.opacity_ex(L, oracle.species(*w.species_tuple()), t, pr, g.nu_start, g.dnu, cutoff, pts,
                                   cut_mode=2, profile=0, plinth=True)
            m = np.abs(ko).max()
            assert np.max(np.abs(kp[pts] - ko)) <= TOL_K * m, (t, pr, s0)
        off += g.n


def test_direct_mode_c1_and_counters():
    """Every (line, point) pair evaluated (no Chebyshev-node classes): parity at every point, and
    the kernels' counters show direct and core evaluations only."""
    import paper_2101_02005_amd as hk
    w, L = workload_lines("c1")
    lines = prepare(L, SP)
    with _env(HK_TIMING=1):
        k = hk.hk_opacity(lines, 1000.0, 1.0, hk.grid(0.0, 0.1, 20_000), 25.0,
                          opts=hk.options(direct=1)).cpu().numpy().astype(np.float64)
        tm = hk.hk_get_timings()
    lines.release()
    ko = oracle.opacity(L, oracle.species(*SP), 1000.0, 1.0, 0.0, 0.1, 25.0, np.arange(20_000))
    assert rel_err(k, ko) <= TOL_K
    cls = dict(zip(hk.CLASS_NAMES, list(tm.class_evals)))
    print("direct mode classes:", cls)
    assert cls["direct"] > 0 and cls["core"] > 0
    assert all(cls[c] == 0 for c in ("far", "very_far", "middle", "masked", "tile_far", "tile_far8"))


def _gap_list():
    """Strong lines on both sides of a line-free gap: inside the gap, k is made of lines evaluated
    at the Chebyshev nodes of spans and tiles (middle, far, very far, masked, tile-far)."""
    rng = np.random.default_rng(11)
    nu = np.concatenate([rng.uniform(1000.0, 1180.0, 12_000), rng.uniform(1220.0, 1400.0, 12_000)])
    S = 10 ** rng.uniform(-20.0, -19.0, nu.size)
    g = rng.uniform(0.02, 0.1, nu.size)
    n = rng.uniform(0.4, 0.8, nu.size)
    E = rng.exponential(2000.0, nu.size)
    return _lines(nu, S=S, E=E, g=g, n=n)


@pytest.mark.parametrize("slots", [1, 2, 4, 8])
def test_interpolation_stress_every_class(slots):
    import paper_2101_02005_amd as hk
    L = _gap_list()
    lines = prepare(L, SP)
    T, P, cut = 1000.0, 1.0, 100.0
    g = (1000.0, 0.01, 40_000)
    with _env(HK_TIMING=1, HK_SLOTS=slots):
        k = hk.hk_opacity(lines, T, P, hk.grid(*g), cut).cpu().numpy().astype(np.float64)
        tm = hk.hk_get_timings()
    lines.release()
    cls = dict(zip(hk.CLASS_NAMES, list(tm.class_evals)))
    print("P=%d classes:" % slots, cls)
    for c in ("direct", "far", "very_far", "middle", "tile_far", "tile_far8", "core"):
        assert cls[c] > 0, c
    if slots <= 2:
        assert cls["masked"] > 0
    sp = oracle.species(*SP)
    # the gap (18000-22000: lines only from its sides) and windows on the line-dense sides
    for a, b in ((18_000, 22_000), (17_000, 18_000), (22_000, 23_000), (0, 500), (39_500, 40_000)):
        pts = np.arange(a, b)
        ko = oracle.opacity(L, sp, T, P, g[0], g[1], cut, pts)
        e = rel_err(k[pts], ko)
        print("P=%d window [%d, %d): %.3e" % (slots, a, b, e))
        assert e <= TOL_K


@pytest.mark.parametrize("options", [None, "plinth"])
def test_items_overflow_is_flagged(options):
    """A work item beyond the workspace's partial rows (forced by a tiny cap from the host) gives
    HK_EDEVICE on a timed call and NaN over its span, never a silently wrong k."""
    import torch

    import paper_2101_02005_amd as hk
    w, L = workload_lines("c1")
    lines = prepare(L, SP)
    opts = None if options is None else hk.options(plinth=1)
    k = torch.zeros(20_000, dtype=torch.float32, device="cuda")
    with _env(HK_TIMING=1, HK_CHUNK=256, HK_DEBUG_ITEMS_CAP=1, HK_SLOTS=2):
        with pytest.raises(hk.HkError) as ei:
            hk.hk_opacity(lines, 1000.0, 1.0, hk.grid(0.0, 0.1, 20_000), 25.0, k=k, opts=opts)
        assert ei.value.status == hk.HK_EDEVICE
    torch.cuda.synchronize()
    assert torch.isnan(k).any()
    # and without the cap the same call succeeds
    with _env(HK_TIMING=1, HK_CHUNK=256, HK_SLOTS=2):
        k = hk.hk_opacity(lines, 1000.0, 1.0, hk.grid(0.0, 0.1, 20_000), 25.0, opts=opts)
        assert hk.hk_get_timings().status == 0
    assert torch.isfinite(k).all()
    lines.release()


def test_side_stream_workspace_kept():
    """Calls on a side stream with library-allocated workspace: torch must not reuse that memory
    for allocations on its current stream before the side stream's work is done."""
    import torch

    import paper_2101_02005_amd as hk
    w, L = workload_lines("c1")
    lines = prepare(L, SP)
    ref = hk.hk_opacity(lines, 1000.0, 1.0, hk.grid(0.0, 0.1, 20_000), 25.0).clone()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    outs = []
    for _ in range(3):
        outs.append(hk.hk_opacity(lines, 1000.0, 1.0, hk.grid(0.0, 0.1, 20_000), 25.0, stream=side))
        junk = torch.full((1 << 22,), 7.0, device="cuda")  # allocations on the current stream meanwhile
        del junk
    side.synchronize()
    for o in outs:
        assert torch.equal(o, ref)
    lines.release()
