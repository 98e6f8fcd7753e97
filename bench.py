"""Benchmark of the line-by-line opacity hot path on one MI355X.

Workload (one step): the large synthetic molecular list -- 5e8 lines over 0-30000 cm^-1 with a
density rising toward the infrared (a stand-in for the ExoMol BT2 water list the paper times),
T = 1500 K, P = 1 atm, grid 0-30000 cm^-1 at 0.01 cm^-1 (3e6 points), cutting length 25 cm^-1.
A step is the whole hot path on device-resident inputs: binning (hk_prepare_lines), per-line
strength/widths, tile work list, Voigt evaluation + accumulation, combine, release.

Prints one JSON line: lines/s (whole job), Voigt evaluations/s, the FP32 roofline of the Voigt
kernel (algorithmic flops from an exact evaluation count, duration from the library's HIP events
on the launch stream) and the FP64 oracle timed on a bounded sample on the host cores.
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
FLOPS_PER_EVAL = 8           # algorithmic FP32 work per wing evaluation


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lines", type=float, default=5e8, help="line count of the large list")
    ap.add_argument("--cut", type=float, default=25.0)
    ap.add_argument("--dnu", type=float, default=0.01)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extras", default="cut100,dnu0.1", help="comma list: cut100, dnu0.1, or none")
    return ap.parse_args()


def count_evals(hk, lines, grd, cut):
    """Exact (line, point) pairs with |nu_j - nu_i| <= cut, from the library's cut bounds."""
    import torch
    lo, hi = hk.hk_debug_cut_bounds(lines, grd, cut)
    c = (hi.to(torch.int64) - lo.to(torch.int64) + 1).clamp_(min=0).sum().item()
    del lo, hi
    return int(c)


def cpu_baseline(w, n_total_evals):
    """The FP64 oracle on a bounded sample of the same workload: 200 grid points at
    5000-5002 cm^-1 with every line within the cut of them."""
    import numpy as np

    import linegen
    import oracle
    nu_a, npts = 5000.0, 200
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


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported" % args.gpus)
        sys.exit(2)
    os.environ.setdefault("HK_TIMING", "1")
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

    # exact evaluation count (outside the timed region)
    lines = hk.hk_prepare_lines(*dev, sp)
    n_evals = count_evals(hk, lines, grd, w.cut)
    ws_bytes = hk.hk_workspace_size(lines, 0, [grd], w.cut)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device="cuda")
    lines.release()
    print("bench: %.4g Voigt evaluations per step, workspace %.2f GB" % (n_evals, ws_bytes / 1e9),
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
    per = []
    for i in range(args.steps):
        per.append(step())
        print("bench: step %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    voigt_ms = sum(t.voigt_ms for _, t in per) / len(per)
    tm = per[-1][1]
    achieved = FLOPS_PER_EVAL * n_evals / (voigt_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": N / dt, "unit": "lines/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c2 large molecular list: %.3g lines, nu = 30000 u^2, grid %g-%g cm^-1 at %g "
                               "(%d points), cut %g cm^-1, T=%g K, P=%g atm (synthetic stand-in for ExoMol BT2)"
                               % (N, w.nu_start, w.nu_end, w.dnu, w.n_grid, w.cut, w.T[0], w.P[0]),
                   "lines": N, "grid_points": w.n_grid, "dnu": w.dnu, "cut": w.cut},
        "evals_per_s": n_evals / dt,
        "voigt_evals_per_s": n_evals / (voigt_ms * 1e-3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "k_voigt", "flops_per_eval": FLOPS_PER_EVAL, "evals_per_launch": n_evals,
                     "avg_launch_ms": voigt_ms},
        "phases_ms": {"bin": sum(b for b, _ in per) / len(per), "prep": tm.prep_ms, "worklist": tm.worklist_ms,
                      "voigt": voigt_ms, "combine": tm.combine_ms},
        "tuning": {"tile_width": tm.tile_width, "lines_per_batch": tm.lines_per_batch,
                   "chunk_lines": tm.chunk_lines, "items_bound": tm.n_items},
        "paper_context": "HELIOS-K 2.0: BT2 water (~4.5e8 lines, data read from RAM) 45 s at 0.01 cm^-1 / cut 25 "
                         "(~1e7 lines/s) and 12.5 s at 0.1 cm^-1 on an RTX 2080 Ti",
    }
    extras = {}
    for ex in [e for e in args.extras.split(",") if e and e != "none"]:
        cut, dnu = (100.0, w.dnu) if ex == "cut100" else (w.cut, 0.1)
        g2 = hk.grid(w.nu_start, dnu, int(round((w.nu_end - w.nu_start) / dnu)))
        ln = hk.hk_prepare_lines(*dev, sp)
        ne = count_evals(hk, ln, g2, cut)
        kk = torch.empty(g2.n, dtype=torch.float32, device="cuda")
        hk.hk_opacity(ln, w.T[0], w.P[0], g2, cut, k=kk)  # warm
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        hk.hk_opacity(ln, w.T[0], w.P[0], g2, cut, k=kk)
        torch.cuda.synchronize()
        te = time.perf_counter() - t1
        tv = hk.hk_get_timings().voigt_ms
        ln.release()
        extras[ex] = {"dnu": dnu, "cut": cut, "evals": ne, "opacity_s": te, "voigt_ms": tv,
                      "voigt_evals_per_s": ne / (tv * 1e-3), "frac_fp32": FLOPS_PER_EVAL * ne / (tv * 1e-3) / 1e12
                      / PEAK_FP32_TFLOPS}
        print("bench: extra %s done" % ex, file=sys.stderr, flush=True)
    out["extra"] = extras
    del dev
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, n_evals)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
