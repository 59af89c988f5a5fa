#!/usr/bin/env python3
"""MGFWA hot-path benchmark on one MI355X: prints one JSON line.

A step is one full MGFWA generation (explosion sparks, their fitness, ranking
and multi-guiding sparks, their fitness, selection, amplitude update, loser-out)
over the whole population, with every input already resident in HBM.  The
default workload is the 64-128-128-10 ReLU cross-entropy network (D = 26,122)
on 4096 Gaussian-mixture samples, 8 fireworks x 256 sparks + 4 guiding sparks.

value     = candidate evaluations per second over the timed steps
roofline  = the explosion-spark fitness kernel (the dominant kernel): algorithmic
            matmul FLOP per launch / its average duration from HIP events
cpu_baseline = the CPU oracle on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "spark-evals/sec & MFMA % peak, BF16 vs FP32 fitness; gen latency p50/p99"
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}   # MI355X dense matrix peaks
WORKLOAD_TAG = {
    "mlp8-16-1": "mgfwa-mlp8-16-1-tanh-mse-teacher256",
    "mlp64-128-128-10": "mgfwa-mlp64-128-128-10-relu-ce-gmm4096",
    "mlp784-256-10": "mgfwa-mlp784-256-10-relu-ce-prototypes8192",
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="mlp64-128-128-10", choices=sorted(WORKLOAD_TAG))
    ap.add_argument("--precision", default=None, choices=["fp32", "bf16"])
    ap.add_argument("--cpu-baseline", type=int, default=1, help="1: time the oracle (rank 0)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU time budget of the oracle sample")
    ap.add_argument("--precision-study", action="store_true",
                    help="also run the 784-256-10 workload in BF16 and FP32 and compare")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--calib-copy-mib", type=int, default=256,
                    help="size of a plain device copy run once before the timed region; its "
                         "FETCH_SIZE / WRITE_SIZE readings scale the fitness kernel's counters")
    return ap.parse_args()


def calibration_copy(mib):
    """A plain device-to-device copy of known size (read mib MiB, write mib MiB)."""
    import torch

    if mib <= 0:
        return
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def run_gpu(wl, precision, steps, warmup, seed):
    import torch

    from paper_2501_03944_amd import mgfwa as M

    g = M.MGFWA.from_workload(wl, precision=precision, seed=seed,
                              max_generations=max(wl.generations, warmup + 2 * steps + 1))
    C = g.BN * (wl.n_sparks + wl.n_guiding)
    g.step(warmup)
    torch.cuda.synchronize()
    # timed region: per-phase HIP events on the library's stream
    g.set_timing(True)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(g.stream)
    g.step(steps)
    end.record(g.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end)
    tinfo = g.timing()
    g.set_timing(False)
    # the same number of generations replayed as one HIP graph each
    gs, ge = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    gs.record(g.stream)
    g.step(steps)
    ge.record(g.stream)
    torch.cuda.synchronize()
    graph_ms = gs.elapsed_time(ge)
    x, best, gen = g.best()
    g.close()
    return dict(C=C, ms=ms, wall=wall, timing=tinfo, graph_ms=graph_ms, best=best, gen=gen)


def cpu_baseline(wl, seconds, seed):
    """Oracle on a bounded sample: initial fireworks, then generation-1 explosion
    sparks and their binary64 fitness, in chunks until the time budget is spent."""
    import numpy as np

    from oracle import oracle as O

    p = O.Problem.from_workload(wl)
    cfg = O.make_config(N=wl.n_fireworks, lam=wl.n_sparks, G=wl.n_guiding, lb=wl.lb, ub=wl.ub,
                        T=wl.generations, seed=seed)
    D = wl.dim
    a0 = np.float32(cfg.ub) - np.float32(cfg.lb)
    t0 = time.perf_counter()
    F = np.stack([O.init_row(cfg, D, f, 0) for f in range(wl.n_fireworks)])
    evals = 0
    chunk = 16
    rows_total = wl.n_fireworks * wl.n_sparks
    while evals < rows_total:
        rows = range(evals, min(evals + chunk, rows_total))
        S = np.stack([O.explosion_row(cfg, F[r // wl.n_sparks], a0, r, 1) for r in rows])
        p.loss_rows(S)
        evals += len(rows)
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=evals / dt, unit="spark-evals/s", cores=threads, kind="oracle",
                sample=f"{evals} generation-1 explosion sparks of the same workload (plus the "
                       f"initial fireworks), binary64 fitness, {dt:.1f} s")


def precision_study(steps, seed):
    from paper_2501_03944_amd import inputs

    wl = inputs.workload("mlp784-256-10")
    out = {}
    for prec in ("bf16", "fp32"):
        r = run_gpu(wl, prec, steps, 1, seed)
        out[prec] = dict(spark_evals_per_s=r["C"] * steps / (r["ms"] / 1e3),
                         ms_per_step=r["ms"] / steps,
                         fit_kernel_tflops=wl.flops_per_eval() * wl.n_fireworks * wl.n_sparks
                         / (r["timing"]["fit_kernel_ms"] / steps / 1e3) / 1e12)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the hot path is measured on one GPU's share).", file=sys.stderr)
        sys.exit(2)
    from paper_2501_03944_amd import inputs

    wl = inputs.workload(args.workload)
    precision = args.precision or "fp32"
    calibration_copy(args.calib_copy_mib)
    r = run_gpu(wl, precision, args.steps, args.warmup, args.seed)
    K = args.steps
    value = r["C"] * K / (r["ms"] / 1e3)
    t = r["timing"]
    rows = wl.n_fireworks * wl.n_sparks
    flops = wl.flops_per_eval() * rows
    fit_ms = t["fit_kernel_ms"] / K
    achieved = flops / (fit_ms / 1e3) / 1e12
    peak = PEAK_TFLOPS[precision]
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "spark-evals/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": r["ms"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if precision == "fp32" else "bf16",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TAG[args.workload], "fireworks": wl.n_fireworks,
                   "sparks": wl.n_sparks, "guiding": wl.n_guiding, "samples": wl.n_samples,
                   "D": wl.dim, "precision": precision, "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "k_fit (explosion-spark fitness)",
                     "flop_per_launch": flops, "avg_launch_ms": fit_ms},
        "mfma_pct_peak": 100.0 * achieved / peak,
        "gen_latency_ms": {"p50": t["gen_ms_p50"], "p99": t["gen_ms_p99"],
                           "mean": t["gen_ms_mean"]},
        "phase_ms_per_step": {k: v / K for k, v in t["phase_ms"].items()},
        "graph_ms_per_step": r["graph_ms"] / K,
        "best_fitness": r["best"],
        "generations_run": r["gen"],
    }
    if args.precision_study:
        line["precision_study"] = precision_study(max(2, min(K, 5)), args.seed)
    if args.cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds, args.seed)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
