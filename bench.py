"""Benchmark of the line-by-line opacity hot path on one MI355X.

Workload (one step): the large synthetic molecular list -- 5e8 lines over 0-30000 cm^-1 with a
density rising toward the infrared (a stand-in for the ExoMol BT2 water list the paper times),
T = 1500 K, P = 1 atm, grid 0-30000 cm^-1 at 0.01 cm^-1 (3e6 points), cutting length 25 cm^-1.
A step is the whole hot path on device-resident inputs: binning (hk_prepare_lines), per-line
strength/widths, tile work list, Voigt evaluation + accumulation, combine, release.

Prints one JSON line: lines/s (whole job); (line, point) pairs within the cut per second; the
FP32 roofline of the wing kernel on one evaluation per pair (8 flops each), measured with the
kernel evaluating every pair outside the line cores (direct mode), over its duration from the
library's HIP events on the launch stream; the default (interpolating) wing pass beside it, with
the evaluations it makes (at grid points, or at Chebyshev nodes of a span or tile for lines far
from it) and its speed-up over direct evaluation; the batched 300-(T, P) form against 300 plain
calls, the adjoint, and the FP64 oracle timed on a bounded sample on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "lines/s + Voigt evals/s at 0.01 cm^-1; %FP32 VALU peak; batched vs plain"
PEAK_FP32_TFLOPS = 157.3     # MI355X vector FP32 (256 CU x 2.4 GHz x 256 flop/clk)
FLOPS_PER_EVAL = 8           # FP32 work per wing evaluation made (at a grid point or a Chebyshev node):
                             # offset FMA, D^2+gamma^2 FMA, reciprocal, amplitude multiply, accumulate
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "wing_pass_c2_5e8_cut25_traffic.txt")
TRAFFIC_FILE_DIRECT = os.path.join(ROOT, "profiles", "wing_direct_c2_5e8_cut25_traffic.txt")
SQ_FILE = os.path.join(ROOT, "profiles", "voigt_kernels_c2_5e8_cut25_sq.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2101_02005_amd", "csrc", "hk_kernels.hip")


def _profile_kv(path, lines, cut, dnu):
    """Key: value lines of a committed profile summary, or None when it is absent, was taken on
    another workload or on a different kernel source."""
    import hashlib
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for ln in f:
            if ":" in ln and not ln.startswith("#"):
                k, v = ln.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        with open(KERNEL_SRC, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        if kv.get("kernel_src_sha256") != sha:
            return None
        if (float(kv["lines"]), float(kv["cut"]), float(kv["dnu"])) != (float(lines), float(cut), float(dnu)):
            return None
    except (KeyError, ValueError, OSError):
        return None
    return kv


def direct_counter_flops(lines, cut, dnu, tile_width):
    """FP32 flops the direct-mode wing kernel executes per pair by the SQ counters (2 FMA + ADD +
    MUL + TRANS, from the committed counter runs), or None when stale."""
    kv = _profile_kv(SQ_FILE, lines, cut, dnu)
    try:
        if kv is None or int(kv["tile_width_direct"]) != int(tile_width):
            return None
        return float(kv["counter_fp32_flops_per_direct_pair"])
    except (KeyError, ValueError):
        return None


def wing_traffic(lines, cut, dnu, tile_width, direct=False):
    """HBM bytes of one launch of the wing kernel evaluating every pair (direct) or of one wing
    pass (k_wing + k_far + k_combine_far) from the committed FETCH_SIZE / WRITE_SIZE counter runs,
    scaled by the same counters on a plain copy; None when absent, taken on another workload or
    span width, or taken on a different kernel source."""
    kv = _profile_kv(TRAFFIC_FILE_DIRECT if direct else TRAFFIC_FILE, lines, cut, dnu)
    try:
        if kv is None or int(kv["tile_width"]) != int(tile_width):
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lines", type=float, default=5e8, help="line count of the large list")
    ap.add_argument("--cut", type=float, default=25.0)
    ap.add_argument("--dnu", type=float, default=0.01)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extras", default="cut100,dnu0.1,batched,backward,options,stream,hitran",
                    help="comma list of cut100, dnu0.1, batched, backward, options, stream, hitran; or none")
    ap.add_argument("--batched-lines", type=float, default=1e7, help="line count of the batched/backward list")
    ap.add_argument("--copy-calibration", type=float, default=0,
                    help="bytes of a plain device copy run after the steps (HBM counter calibration)")
    return ap.parse_args()


PEAK_HBM_GBS = 8000.0
BIN_BYTES_PER_LINE = 88      # read 5 FP64 fields; write them sorted, the permutation and the bin keys
PREP_BYTES_PER_LINE = 72     # strengths/widths: read 40 B, write 8 B; grid records: read 8 B, write 16 B


def hbm_phases(N, bin_ms, prep_ms):
    """Algorithmic HBM rates of the bandwidth-bound phases (binning once per list, per-T prep)."""
    out = {}
    for name, bpl, ms in (("bin", BIN_BYTES_PER_LINE, bin_ms), ("prep", PREP_BYTES_PER_LINE, prep_ms)):
        gbs = N * bpl / (ms * 1e-3) / 1e9
        out[name] = {"bytes_per_line": bpl, "ms": ms, "achieved_GBs": gbs, "peak_GBs": PEAK_HBM_GBS,
                     "frac": gbs / PEAK_HBM_GBS}
    return out


def count_evals(hk, lines, grd, cut):
    """Exact (line, point) pairs with |nu_j - nu_i| <= cut, from the library's cut bounds."""
    import torch
    lo, hi = hk.hk_debug_cut_bounds(lines, grd, cut)
    c = (hi.to(torch.int64) - lo.to(torch.int64) + 1).clamp_(min=0).sum().item()
    del lo, hi
    return int(c)


def cpu_baseline(w, n_total_evals):
    """The FP64 oracle on a bounded sample of the same workload: 2000 grid points at
    5000-5020 cm^-1 with every line within the cut of them."""
    import numpy as np

    import linegen
    import oracle
    nu_a, npts = 5000.0, 2000
    j0 = int(round((nu_a - w.nu_start) / w.dnu))
    pts = np.arange(j0, j0 + npts)
    lo = w.nu_start + j0 * w.dnu - w.cut - 1.0
    hi = w.nu_start + (j0 + npts) * w.dnu + w.cut + 1.0
    t0 = time.perf_counter()
    _, L = linegen.select(w.recipe(), w.seed, w.N, lo, hi, cap=1 << 23)
    t_sel = time.perf_counter() - t0
    sp = oracle.species(*w.species_tuple())
    evals = 0
    nuj = w.nu_start + pts * w.dnu
    srt = np.sort(L["nu"])
    for v in nuj:
        evals += int(np.searchsorted(srt, v + w.cut, "right") - np.searchsorted(srt, v - w.cut, "left"))
    t0 = time.perf_counter()
    oracle.opacity(L, sp, w.T[0], w.P[0], w.nu_start, w.dnu, w.cut, pts)
    t = time.perf_counter() - t0
    eps = evals / t
    return {"value": w.N * eps / n_total_evals, "unit": "lines/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d grid points at %.0f-%.0f cm^-1, %d lines within the cut, %.3g evals in %.2f s "
                      "(%.3g evals/s; line selection %.1f s not timed); scaled to the whole job by its %.4g evals"
                      % (npts, nu_a, nu_a + npts * w.dnu, len(L["nu"]), evals, t, eps, t_sel, n_total_evals),
            "evals_per_s": eps}


def _device_list(w, N):
    import torch

    import linegen
    dev = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in range(5)]
    linegen.generate_device(w.recipe(), w.seed, N, [t.data_ptr() for t in dev],
                            stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return dev


def _oracle_windows(w, N, T, P, grd, k_host, starts, width=16):
    """Max |k - k_oracle| / max k_oracle over oracle windows (lines selected around each window)."""
    import numpy as np

    import linegen
    import oracle
    sp = oracle.species(*w.species_tuple())
    worst = 0.0
    for s0 in starts:
        s0 = int(min(max(s0, 0), grd.n - width))
        lo = grd.nu_start + s0 * grd.dnu - w.cut - 0.5
        hi = grd.nu_start + (s0 + width) * grd.dnu + w.cut + 0.5
        _, L = linegen.select(w.recipe(), w.seed, N, max(lo, 0.0), hi, cap=1 << 24)
        pts = np.arange(s0, s0 + width)
        ko = oracle.opacity(L, sp, T, P, grd.nu_start, grd.dnu, w.cut, pts)
        if ko.max() > 0:
            worst = max(worst, float(np.max(np.abs(k_host[pts].astype(np.float64) - ko)) / ko.max()))
    return worst


def _median(xs):
    import statistics
    return float(statistics.median(xs))


class _env:
    """Temporarily set (or unset, with None) environment variables the library reads per call."""

    def __init__(self, **kv):
        self.kv = kv

    def __enter__(self):
        self.old = {k: os.environ.get(k) for k in self.kv}
        for k, v in self.kv.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = str(v)

    def __exit__(self, *exc):
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def bench_batched(hk, n_lines, repeats=5):
    """300 (T, P) pairs of the batched workload: one hk_opacity_batched call (graph replay) against
    300 hk_opacity calls on the same device-resident list; each the median of `repeats` timings,
    with per-call timing off (no host synchronization inside either leg)."""
    import numpy as np
    import torch

    import linegen
    w = linegen.workload("c3", N=int(n_lines))
    dev = _device_list(w, w.N)
    lines = hk.hk_prepare_lines(*dev, hk.species(*w.species_tuple()))
    del dev
    T = [t for t in w.T for _ in w.P]
    P = [p for _ in w.T for p in w.P]
    n_pairs = len(T)
    grd = hk.grid(w.nu_start, w.dnu, w.n_grid)
    kb = torch.empty(n_pairs * w.n_grid, dtype=torch.float32, device="cuda")
    kp = torch.empty_like(kb)
    wsb = hk._lib._workspace(hk.hk_workspace_size(lines, 1, [grd] * n_pairs, w.cut, n_temps=len(w.T)))
    wsp = hk._lib._workspace(hk.hk_workspace_size(lines, 0, [grd], w.cut))
    with _env(HK_TIMING=None):
        # the first batched call tunes and records the graph (untimed)
        hk.hk_opacity_batched(lines, T, P, [grd] * n_pairs, w.cut, k=kb, ws=wsb)
        torch.cuda.synchronize()
        print("bench: batched graph recorded", file=sys.stderr, flush=True)
        tb = []
        for _ in range(repeats):
            t0 = time.perf_counter()
            hk.hk_opacity_batched(lines, T, P, [grd] * n_pairs, w.cut, k=kb, ws=wsb)
            torch.cuda.synchronize()
            tb.append(time.perf_counter() - t0)
        print("bench: batched %.3f s (median of %d)" % (_median(tb), repeats), file=sys.stderr, flush=True)
        hk.hk_opacity(lines, T[0], P[0], grd, w.cut, k=kp[:w.n_grid], ws=wsp)  # tunes the plain call
        torch.cuda.synchronize()
        tp = []
        for _ in range(repeats):
            t0 = time.perf_counter()
            for p in range(n_pairs):
                hk.hk_opacity(lines, T[p], P[p], grd, w.cut, k=kp[p * w.n_grid:(p + 1) * w.n_grid], ws=wsp)
            torch.cuda.synchronize()
            tp.append(time.perf_counter() - t0)
        print("bench: 300 plain calls %.3f s (median of %d)" % (_median(tp), repeats), file=sys.stderr, flush=True)
    t_b, t_p = _median(tb), _median(tp)
    kb2, kp2 = kb.view(n_pairs, -1), kp.view(n_pairs, -1)
    diff = ((kb2 - kp2).abs().amax(dim=1).double() / kp2.amax(dim=1).double().clamp_min(1e-300)).max().item()
    pairs_one = count_evals(hk, lines, grd, w.cut)
    lines.release()
    # oracle windows for two extreme pairs (lowest T and P, highest T and P)
    orc = {}
    for p in (0, n_pairs - 1):
        kh = kb2[p].cpu().numpy()
        starts = [int(np.argmax(kh)) - 8, w.n_grid // 3, w.n_grid - 16]
        orc["T=%g,P=%g" % (T[p], P[p])] = _oracle_windows(w, w.N, T[p], P[p], grd, kh, starts)
    del kb, kp, kb2, kp2, wsb, wsp
    torch.cuda.empty_cache()
    return {"workload": "%d lines (nu = 10000 u^2), %d T x %d P = %d pairs, grid %g-%g cm^-1 at %g (%d points), "
                        "cut %g" % (w.N, len(w.T), len(w.P), n_pairs, w.nu_start, w.nu_end, w.dnu, w.n_grid, w.cut),
            "batched_s": t_b, "plain_300_s": t_p, "speedup": t_p / t_b, "repeats": repeats,
            "batched_s_all": tb, "plain_300_s_all": tp,
            "pairs_per_s_batched": pairs_one * n_pairs / t_b, "lines_pairs_per_s_batched": w.N * n_pairs / t_b,
            "max_rel_diff_batched_vs_plain": diff, "oracle_window_max_rel_err": orc}


ADJ_FLOPS_PER_EVAL = 16  # the adjoint's FP32 work per evaluation made: the profile (8) plus the
                         # two derivative polynomials and three dL/dk-weighted accumulations


def bench_backward(hk, n_lines, repeats=5):
    """The adjoint at the differentiation workload (T = 800 K, P = 0.1 atm, cut 100)."""
    import torch

    import linegen
    w = linegen.workload("c4", N=int(n_lines))
    dev = _device_list(w, w.N)
    lines = hk.hk_prepare_lines(*dev, hk.species(*w.species_tuple()))
    del dev
    grd = hk.grid(w.nu_start, w.dnu, w.n_grid)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(w.extra["g_seed"])
    g = torch.randn(w.n_grid, generator=gen, device="cuda", dtype=torch.float32)
    ws = hk._lib._workspace(hk.hk_workspace_size(lines, 2, [grd], w.cut))
    hk.hk_opacity_backward(lines, w.T[0], w.P[0], grd, w.cut, g, ws=ws)  # warm
    torch.cuda.synchronize()
    tb, tk = [], []
    for _ in range(repeats):
        t0 = time.perf_counter()
        out2, dS, dg, dn = hk.hk_opacity_backward(lines, w.T[0], w.P[0], grd, w.cut, g, ws=ws)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
        tm = hk.hk_get_timings()
        tk.append(tm.backward_ms)
    evals = int(tm.backward_evals)  # direct points and 16 per far unit (each stands for its points)
    wsf = hk._lib._workspace(hk.hk_workspace_size(lines, 0, [grd], w.cut))
    kf = torch.empty(w.n_grid, dtype=torch.float32, device="cuda")
    hk.hk_opacity(lines, w.T[0], w.P[0], grd, w.cut, k=kf, ws=wsf)
    torch.cuda.synchronize()
    tf = []
    for _ in range(repeats):
        t1 = time.perf_counter()
        hk.hk_opacity(lines, w.T[0], w.P[0], grd, w.cut, k=kf, ws=wsf)
        torch.cuda.synchronize()
        tf.append(time.perf_counter() - t1)
    ne = count_evals(hk, lines, grd, w.cut)
    lines.release()
    t, kms = _median(tb), _median(tk)
    ach = ADJ_FLOPS_PER_EVAL * evals / (kms * 1e-3) / 1e12
    return {"workload": "%d lines, grid %g-%g cm^-1 at %g (%d points), cut %g, T=%g K, P=%g atm, dL/dk ~ N(0,1)"
                        % (w.N, w.nu_start, w.nu_end, w.dnu, w.n_grid, w.cut, w.T[0], w.P[0]),
            "backward_s": t, "backward_kernel_ms": kms, "forward_s": _median(tf), "backward_over_forward": t / _median(tf),
            "pairs": ne, "pairs_per_s_backward": ne / t, "evals_made": evals,
            "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                         "frac": ach / PEAK_FP32_TFLOPS, "flops_per_eval": ADJ_FLOPS_PER_EVAL,
                         "kernel": "adjoint (k_adj_nodes + k_adj_lines + k_adjoint + k_reduce2), on the "
                                   "evaluations made (direct points, 16 nodes per far unit)"},
            "dL_dT": out2[0].item(), "dL_dlnP": out2[1].item()}


def bench_direct(hk, dev, sp, w, grd, n_pairs, repeats=3):
    """The default path with every (line, point) pair outside the line cores evaluated by the wing
    kernel (no Chebyshev-node classes, no tile-far pass): the FP32 roofline on the unit of one
    evaluation per pair, 8 flops each."""
    import torch
    ln = hk.hk_prepare_lines(*dev, sp)
    opts = hk.options(direct=1)
    need = hk.hk_workspace_size_ex(ln, 0, [w.T[0]], [w.P[0]], [grd], w.cut, opts)
    ws = hk._lib._workspace(need)
    k = torch.empty(grd.n, dtype=torch.float32, device="cuda")
    with _env(HK_TIMING=1):
        hk.hk_opacity(ln, w.T[0], w.P[0], grd, w.cut, k=k, ws=ws, opts=opts)  # tunes (autotuner) and warms
        torch.cuda.synchronize()
        tw, tc, tot = [], [], []
        for _ in range(repeats):
            t0 = time.perf_counter()
            hk.hk_opacity(ln, w.T[0], w.P[0], grd, w.cut, k=k, ws=ws, opts=opts)
            torch.cuda.synchronize()
            tot.append(time.perf_counter() - t0)
            tm = hk.hk_get_timings()
            tw.append(tm.voigt_ms)
            tc.append(tm.core_ms)
    ln.release()
    cls = dict(zip(hk.CLASS_NAMES, list(tm.class_evals)))
    wing_pairs = n_pairs - tm.core_evals
    t_w = _median(tw)
    ach = FLOPS_PER_EVAL * wing_pairs / (t_w * 1e-3) / 1e12
    del ws, k
    torch.cuda.empty_cache()
    return {"k_wing_ms": t_w, "k_core_ms": _median(tc), "opacity_s": _median(tot), "tile_width": tm.tile_width,
            "wing_pairs": wing_pairs, "core_pairs": tm.core_evals, "evals_made": cls["direct"],
            "achieved_TFLOPs": ach, "frac": ach / PEAK_FP32_TFLOPS, "k_wing_ms_all": tw}


def bench_options(hk, n_lines, repeats=3):
    """The options path (every (line, point) pair inside each line's own cut evaluated directly)
    on the differentiation list: each line profile, plinth removal and the width-multiple cuts."""
    import torch

    import linegen
    w = linegen.workload("c4", N=int(n_lines))
    dev = _device_list(w, w.N)
    lines = hk.hk_prepare_lines(*dev, hk.species(*w.species_tuple()))
    nu = dev[0]
    del dev
    grd = hk.grid(w.nu_start, w.dnu, w.n_grid)
    T, P = w.T[0], w.P[0]
    alpha = hk.hk_debug_line_params(lines, T, P)[1]
    cases = [("voigt_plinth", dict(profile=0, plinth=1), w.cut),
             ("lorentz", dict(profile=1), w.cut), ("doppler", dict(profile=2), w.cut),
             ("binned_gauss", dict(profile=3), w.cut), ("voigt_lorentz_cut_plinth", dict(cut_mode=2, plinth=1), 500.0),
             ("voigt_doppler_cut", dict(cut_mode=1), 1000.0)]
    out = {"workload": "%d lines (nu = 10000 u^2), grid %g-%g cm^-1 at %g (%d points), T=%g K, P=%g atm"
                       % (w.N, w.nu_start, w.nu_end, w.dnu, w.n_grid, T, P)}
    k = torch.empty(w.n_grid, dtype=torch.float32, device="cuda")
    for name, kw, cut in cases:
        opts = hk.options(**kw)
        need = hk.hk_workspace_size_ex(lines, 0, [T], [P], [grd], cut, opts)
        ws = hk._lib._workspace(need)
        with _env(HK_TIMING=1):
            hk.hk_opacity(lines, T, P, grd, cut, k=k, ws=ws, opts=opts)  # tunes and warms
            torch.cuda.synchronize()
            tt, td, tc = [], [], []
            for _ in range(repeats):
                t0 = time.perf_counter()
                hk.hk_opacity(lines, T, P, grd, cut, k=k, ws=ws, opts=opts)
                torch.cuda.synchronize()
                tt.append(time.perf_counter() - t0)
                tm = hk.hk_get_timings()
                td.append(tm.voigt_ms)
                tc.append(tm.core_ms if tm.core_ms > 0 else 0.0)
        made = tm.class_evals[0]  # lines staged per span x span points (points outside a cut included)
        lo, hi, _ = hk.hk_debug_grid_records(lines, T, P, grd, cut, opts)
        lo, hi = lo.to(torch.int64), hi.to(torch.int64)
        pairs = int((hi - lo + 1).clamp_(min=0).sum().item())
        prof = kw.get("profile", 0)
        if prof in (2, 3):
            # a Gaussian (or its bin average) is below e^-81 of its peak beyond 9 alpha + a bin
            # from the centre: the pairs that carry a value are those within that reach
            cen = (nu - w.nu_start) / w.dnu
            reach = (9.0 * alpha + w.dnu) / w.dnu
            glo = torch.maximum(lo, torch.ceil(cen - reach).to(torch.int64))
            ghi = torch.minimum(hi, torch.floor(cen + reach).to(torch.int64))
            work = int((ghi - glo + 1).clamp_(min=0).sum().item())
            del glo, ghi, cen, reach
        else:
            work = pairs - tm.core_evals if prof == 0 else pairs
        del lo, hi
        t_d = _median(td)
        ach = FLOPS_PER_EVAL * work / (t_d * 1e-3) / 1e12
        out[name] = {"cut": cut, "opacity_s": _median(tt), "k_direct_ms": t_d, "k_core_ms": _median(tc),
                     "pairs": pairs, "core_pairs": tm.core_evals if prof == 0 else 0,
                     "pairs_evaluated": work, "pairs_per_s": pairs / _median(tt), "span_evals_made": made,
                     "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                                  "frac": ach / PEAK_FP32_TFLOPS, "flops_per_pair": FLOPS_PER_EVAL,
                                  "kernel": "k_direct (pairs_evaluated: outside the Voigt cores; Gaussians "
                                            "within 9 alpha + a bin)"}}
        del ws
        print("bench: options %s done" % name, file=sys.stderr, flush=True)
    lines.release()
    del k, nu, alpha
    torch.cuda.empty_cache()
    return out


def bench_stream(hk, n_lines, chunk):
    """The streamed form: the large list's first n_lines lines in pinned host memory, processed in
    chunks whose host-to-device copies overlap the binning and evaluation; against the same
    lines resident on the device (one prepare + one opacity)."""
    import torch

    import linegen
    w = linegen.workload("c2", N=int(n_lines))
    dev = _device_list(w, w.N)
    host = [torch.empty(w.N, dtype=torch.float64, pin_memory=True) for _ in range(5)]
    for h, d in zip(host, dev):
        h.copy_(d)
    torch.cuda.synchronize()
    sp = hk.species(*w.species_tuple())
    grd = hk.grid(w.nu_start, w.dnu, w.n_grid)
    k = torch.empty(w.n_grid, dtype=torch.float32, device="cuda")
    with _env(HK_TIMING=None):
        for _ in range(2):  # the first pass tunes the list size's key; the second is timed
            t0 = time.perf_counter()
            ln = hk.hk_prepare_lines(*dev, sp)
            hk.hk_opacity(ln, w.T[0], w.P[0], grd, w.cut, k=k)
            torch.cuda.synchronize()
            ln.release()
            t_res = time.perf_counter() - t0
        del dev
        torch.cuda.empty_cache()
        hk.hk_opacity_stream(*host, sp, w.T[0], w.P[0], grd, w.cut, int(chunk), k=k)  # warms the block cache
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hk.hk_opacity_stream(*host, sp, w.T[0], w.P[0], grd, w.cut, int(chunk), k=k)
        torch.cuda.synchronize()
        t_str = time.perf_counter() - t0
        # the copies alone, from the same pinned memory
        buf = torch.empty(w.N, dtype=torch.float64, device="cuda")
        t0 = time.perf_counter()
        for h in host:
            buf.copy_(h, non_blocking=True)
        torch.cuda.synchronize()
        t_copy = time.perf_counter() - t0
    del host, buf, k
    torch.cuda.empty_cache()
    return {"workload": "first %d lines of the large list in pinned host memory, chunks of %d, grid %g-%g cm^-1 at "
                        "%g, cut %g" % (w.N, chunk, w.nu_start, w.nu_end, w.dnu, w.cut),
            "streamed_s": t_str, "lines_per_s_streamed": w.N / t_str, "device_resident_s": t_res,
            "h2d_copy_s": t_copy, "h2d_GBs": 40.0 * w.N / t_copy / 1e9,
            "overlap": (t_copy + t_res) / t_str}


def bench_hitran(hk, n_lines, repeats=3):
    """HITRAN-style widths and pressure shifts: each call bins the list again by its shifted
    centres, then evaluates every pair directly."""
    import numpy as np
    import torch
    rng = np.random.default_rng(61)
    N = int(n_lines)
    nu = 10000.0 * rng.uniform(0.0, 1.0, N) ** 2 + 1e-3
    E = rng.exponential(4000.0, N)
    c2 = 1.438776855773617
    S = 10 ** rng.uniform(-26.0, -19.0, N) * np.exp(-c2 * E / 296.0) * (-np.expm1(-c2 * nu / 296.0))
    cols = [nu, S, E, rng.uniform(0.02, 0.1, N), rng.uniform(0.1, 0.5, N), rng.uniform(0.4, 0.8, N),
            rng.uniform(-0.02, 0.01, N)]
    dev = [torch.from_numpy(c).cuda() for c in cols]
    lines = hk.hk_prepare_lines_hitran(*dev, hk.species(18.0))
    del dev
    grd = hk.grid(0.0, 0.01, 1_000_000)
    k = torch.empty(grd.n, dtype=torch.float32, device="cuda")
    hk.hk_opacity_hitran(lines, 800.0, 1.0, 0.1, grd, 25.0, k=k)
    torch.cuda.synchronize()
    tt = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        hk.hk_opacity_hitran(lines, 800.0, 1.0, 0.1, grd, 25.0, k=k)
        torch.cuda.synchronize()
        tt.append(time.perf_counter() - t0)
    lines.release()
    del k
    torch.cuda.empty_cache()
    return {"workload": "%d lines (nu = 10000 u^2), gamma_air, gamma_self, delta_air synthetic; grid 0-10000 cm^-1 "
                        "at 0.01; cut 25; T=800 K, P=1 atm, P_self=0.1 atm" % N,
            "opacity_s": _median(tt), "lines_per_s": N / _median(tt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported" % args.gpus)
        sys.exit(2)
    os.environ.setdefault("HK_TIMING", "1")
    os.environ.setdefault("HK_AUTOTUNE", "1")  # span width timed on the first call of each tuning key
    import torch

    import linegen
    import paper_2101_02005_amd as hk

    torch.cuda.set_device(0)
    w = linegen.workload("c2", N=int(args.lines), cut=args.cut, dnu=args.dnu)
    N = w.N
    print("bench: generating %d lines on the device" % N, file=sys.stderr, flush=True)
    dev = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in range(5)]
    linegen.generate_device(w.recipe(), w.seed, N, [t.data_ptr() for t in dev],
                            stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    sp = hk.species(*w.species_tuple())
    grd = hk.grid(w.nu_start, w.dnu, w.n_grid)
    k = torch.empty(w.n_grid, dtype=torch.float32, device="cuda")

    # exact (line, point) pair count (outside the timed region)
    lines = hk.hk_prepare_lines(*dev, sp)
    n_pairs = count_evals(hk, lines, grd, w.cut)
    ws_bytes = hk.hk_workspace_size(lines, 0, [grd], w.cut)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device="cuda")
    lines.release()
    print("bench: %.4g (line, point) pairs per step, workspace %.2f GB" % (n_pairs, ws_bytes / 1e9),
          file=sys.stderr, flush=True)

    def step():
        ln = hk.hk_prepare_lines(*dev, sp)
        t_bin = hk.hk_get_timings().bin_ms
        hk.hk_opacity(ln, w.T[0], w.P[0], grd, w.cut, k=k, ws=ws)
        tm = hk.hk_get_timings()
        ln.release()
        return t_bin, tm

    for i in range(args.warmup):
        step()
        print("bench: warmup %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per, host = [], []
    for i in range(args.steps):
        ts = time.perf_counter()
        per.append(step())
        host.append(time.perf_counter() - ts)
        print("bench: step %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    med = lambda f: _median([f(t) for _, t in per])  # noqa: E731
    kv_ms, far_ms, core_ms = med(lambda t: t.voigt_ms), med(lambda t: t.far_ms), med(lambda t: t.core_ms)
    interp_ms = kv_ms + far_ms  # the wing pass: k_wing, then the tile-far pass
    tm = per[-1][1]
    cls = dict(zip(hk.CLASS_NAMES, list(tm.class_evals)))
    wing_pairs = n_pairs - tm.core_evals
    made = tm.wing_evals  # evaluations the wing pass made (grid points and Chebyshev nodes)
    del ws
    torch.cuda.empty_cache()

    # the same kernel evaluating every pair: the roofline on one evaluation per pair
    print("bench: direct-evaluation leg", file=sys.stderr, flush=True)
    direct = bench_direct(hk, dev, sp, w, grd, n_pairs)
    rf_traffic = wing_traffic(N, w.cut, w.dnu, direct["tile_width"], direct=True)
    cflops = direct_counter_flops(N, w.cut, w.dnu, direct["tile_width"])
    c_ach = (cflops * direct["wing_pairs"] / (direct["k_wing_ms"] * 1e-3) / 1e12) if cflops else None
    out = {
        "metric": METRIC, "value": N / dt, "unit": "lines/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "median_ms_per_step": _median(host) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c2 large molecular list: %.3g lines, nu = 30000 u^2, grid %g-%g cm^-1 at %g "
                               "(%d points), cut %g cm^-1, T=%g K, P=%g atm (synthetic stand-in for ExoMol BT2)"
                               % (N, w.nu_start, w.nu_end, w.dnu, w.n_grid, w.cut, w.T[0], w.P[0]),
                   "lines": N, "grid_points": w.n_grid, "dnu": w.dnu, "cut": w.cut},
        "pairs": n_pairs, "core_pairs": tm.core_evals,
        "pairs_per_s": n_pairs / dt,
        "pairs_per_s_voigt_passes": n_pairs / ((interp_ms + core_ms) * 1e-3),
        "roofline": {"bound": "alu", "achieved": direct["achieved_TFLOPs"], "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": direct["frac"], "traffic": rf_traffic,
                     "kernel": "k_wing<%d> evaluating every (line, point) pair outside the line cores (direct mode)"
                               % (direct["tile_width"] // 64),
                     "flops_per_pair": FLOPS_PER_EVAL, "pairs_per_launch": direct["wing_pairs"],
                     "avg_launch_ms": direct["k_wing_ms"],
                     # the flops the kernel executes per pair by the SQ counters (series terms, Kahan
                     # flushes), and the FP32 fraction on them, next to the nominal 8 per pair
                     "counter_flops_per_pair": cflops, "counter_achieved": c_ach,
                     "counter_frac": (c_ach / PEAK_FP32_TFLOPS) if c_ach else None},
        "interpolated": {
            "kernel": "wing pass: k_wing<%d> + k_far + k_combine_far (lines far from a span or tile at its "
                      "Chebyshev nodes)" % (tm.tile_width // 64),
            "k_wing_ms": kv_ms, "k_far_ms": far_ms, "wing_pass_ms": interp_ms, "wing_pairs": wing_pairs,
            "evals_made": made, "evals_made_per_s": made / (interp_ms * 1e-3),
            "wing_pairs_per_s": wing_pairs / (interp_ms * 1e-3),
            "speedup_vs_direct": direct["k_wing_ms"] / interp_ms,
            "traffic": wing_traffic(N, w.cut, w.dnu, tm.tile_width),
            "frac_fp32_on_evals_made": FLOPS_PER_EVAL * made / (interp_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
            "class_evals": cls},
        "direct": direct,
        "phases_ms": {"bin": _median([b for b, _ in per]), "prep": med(lambda t: t.prep_ms),
                      "worklist": med(lambda t: t.worklist_ms), "voigt_wing": kv_ms, "tile_far": far_ms,
                      "voigt_core": core_ms, "combine": med(lambda t: t.combine_ms)},
        "hbm": hbm_phases(N, _median([b for b, _ in per]), med(lambda t: t.prep_ms)),
        "tuning": {"tile_width": tm.tile_width, "lines_per_batch": tm.lines_per_batch,
                   "chunk_lines": tm.chunk_lines, "items_bound": tm.n_items},
        "paper_context": "HELIOS-K 2.0: BT2 water (~4.5e8 lines, data read from RAM) 45 s at 0.01 cm^-1 / cut 25 "
                         "(~1e7 lines/s) and 12.5 s at 0.1 cm^-1 on an RTX 2080 Ti",
    }
    if args.copy_calibration > 0:
        nf = int(args.copy_calibration) // 4
        src = torch.ones(nf, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"bytes_read": 4 * nf, "bytes_written": 4 * nf}
        del src, dst
    extras = {}
    for ex in [e for e in args.extras.split(",") if e and e != "none" and e in ("cut100", "dnu0.1")]:
        cut, dnu = (100.0, w.dnu) if ex == "cut100" else (w.cut, 0.1)
        g2 = hk.grid(w.nu_start, dnu, int(round((w.nu_end - w.nu_start) / dnu)))
        ln = hk.hk_prepare_lines(*dev, sp)
        ne = count_evals(hk, ln, g2, cut)
        kk = torch.empty(g2.n, dtype=torch.float32, device="cuda")
        hk.hk_opacity(ln, w.T[0], w.P[0], g2, cut, k=kk)  # tunes and warms
        torch.cuda.synchronize()
        te = []
        for _ in range(3):
            t1 = time.perf_counter()
            hk.hk_opacity(ln, w.T[0], w.P[0], g2, cut, k=kk)
            torch.cuda.synchronize()
            te.append(time.perf_counter() - t1)
        t2 = hk.hk_get_timings()
        tv, tc = t2.voigt_ms + t2.far_ms, t2.core_ms
        ln.release()
        extras[ex] = {"dnu": dnu, "cut": cut, "pairs": ne, "core_pairs": t2.core_evals, "opacity_s": _median(te),
                      "tile_width": t2.tile_width, "lines_per_batch": t2.lines_per_batch,
                      "wing_pass_ms": tv, "tile_far_ms": t2.far_ms, "voigt_core_ms": tc,
                      "pairs_per_s_voigt_passes": ne / ((tv + tc) * 1e-3),
                      "evals_made": t2.wing_evals,
                      "frac_fp32_on_evals_made": FLOPS_PER_EVAL * t2.wing_evals / (tv * 1e-3) / 1e12 / PEAK_FP32_TFLOPS}
        print("bench: extra %s done" % ex, file=sys.stderr, flush=True)
    out["extra"] = extras
    del dev
    torch.cuda.empty_cache()
    wanted = args.extras.split(",")
    if "batched" in wanted:
        out["batched"] = bench_batched(hk, args.batched_lines)
        print("bench: batched done", file=sys.stderr, flush=True)
    if "backward" in wanted:
        out["backward"] = bench_backward(hk, args.batched_lines)
        print("bench: backward done", file=sys.stderr, flush=True)
    if "options" in wanted:
        out["options"] = bench_options(hk, args.batched_lines)
    if "stream" in wanted:
        out["stream"] = bench_stream(hk, 2e8, 5e7)
        print("bench: stream done", file=sys.stderr, flush=True)
    if "hitran" in wanted:
        out["hitran"] = bench_hitran(hk, args.batched_lines)
        print("bench: hitran done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, n_pairs)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
