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
# the paper's testbed (Table 2): input optimisation of a fixed MLP
WORKLOAD_TAG.update({f"net{i}": f"mgfwa-testbed-net{i}-input-optimisation" for i in range(1, 13)})


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
    ap.add_argument("--precision-study", type=int, default=1,
                    help="1: also run the 784-256-10 workload in BF16 and FP32 and compare")
    ap.add_argument("--batch-study", type=int, default=1,
                    help="1: also run 64 mixed-shape BF16 jobs as one batched graph per generation")
    ap.add_argument("--serving-study", type=int, default=1,
                    help="1: also run a Poisson stream of mixed jobs through the serving loop")
    ap.add_argument("--serve-seconds", type=float, default=8.0, help="arrival window of that study")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: autotune the fitness launches before timing (mgfwa_autotune)")
    ap.add_argument("--testbed-study", type=int, default=1,
                    help="1: the paper's testbed (Table 2 nets, input optimisation), per net")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--calib-copy-mib", type=int, default=256,
                    help="size of a plain device copy run once before the timed region; its "
                         "FETCH_SIZE / WRITE_SIZE readings scale the fitness kernel's counters")
    return ap.parse_args()


PROFILE_FOR = {   # (workload, precision) -> committed rocprofv3 traffic summary of its dominant kernel
    ("mlp64-128-128-10", "fp32"): "k_fit_mlp64-128-128-10_fp32_traffic.json",
    ("mlp64-128-128-10", "bf16"): "k_fit_mlp64-128-128-10_bf16_traffic.json",
    ("mlp784-256-10", "bf16"): "k_fit_wide_mlp784-256-10_bf16_traffic.json",
    ("mlp784-256-10", "fp32"): "k_fit_wide_mlp784-256-10_fp32_traffic.json",
    ("net12", "fp32"): "k_net_layer_net12_fp32_traffic.json",   # the fitness step's launches
}


def measured_traffic(workload, precision):
    """HBM bytes per launch of the dominant kernel from the committed FETCH_SIZE /
    WRITE_SIZE summary, or None when there is none or the kernel's sources changed
    since the counters were taken."""
    import hashlib

    name = PROFILE_FOR.get((workload, precision))
    path = os.path.join(ROOT, "profiles", name) if name else None
    if not path or not os.path.exists(path):
        return None, None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in sorted(rec["sources"]):
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None, name + " (stale: kernel sources changed)"
    return rec["hbm_bytes_per_launch"], name


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


def run_gpu(wl, precision, steps, warmup, seed, autotune=True):
    import torch

    from paper_2501_03944_amd import mgfwa as M

    g = M.MGFWA.from_workload(wl, precision=precision, seed=seed,
                              max_generations=max(wl.generations, warmup + 2 * steps + 1))
    C = g.BN * (wl.n_sparks + wl.n_guiding)
    if autotune:
        g.autotune(3)     # the kernel variant / tile shape of each launch size
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


def topk_agreement(y_run, y_ref, lam, G, sigma):
    """Guiding-group decisions (top and bottom k members of each group of m sparks)
    taken on y_run against those taken on y_ref, both [fireworks, lam] numpy."""
    import numpy as np

    m = lam // G
    k = max(1, int(sigma * m))
    same_sets = overlap = groups = 0
    for f in range(y_run.shape[0]):
        for g in range(G):
            a, b = y_run[f, g * m:(g + 1) * m], y_ref[f, g * m:(g + 1) * m]
            oa, ob = np.argsort(a, kind="stable"), np.argsort(b, kind="stable")
            ta, tb = set(oa[:k]), set(ob[:k])
            ba, bb = set(oa[-k:]), set(ob[-k:])
            overlap += len(ta & tb) + len(ba & bb)
            same_sets += (ta == tb) and (ba == bb)
            groups += 1
    best_same = float(np.mean(np.argmin(y_run, axis=1) == np.argmin(y_ref, axis=1)))
    return dict(member_agreement=overlap / (2.0 * k * groups),
                groups_identical=same_sets / groups, best_spark_agreement=best_same, k=k, m=m)


def precision_study(steps, seed, gens=3):
    """784-256-10 in BF16 and FP32: throughput of each, and for the sparks of the
    first generations of the BF16 run, the BF16 fitness against the FP32 fitness
    of the same sparks (relative error, guiding top/bottom-k and best-spark
    agreement)."""
    import numpy as np
    import torch

    from paper_2501_03944_amd import inputs
    from paper_2501_03944_amd import mgfwa as M

    wl = inputs.workload("mlp784-256-10")
    out = {}
    for prec in ("bf16", "fp32"):
        r = run_gpu(wl, prec, steps, 1, seed)
        out[prec] = dict(spark_evals_per_s=r["C"] * steps / (r["ms"] / 1e3),
                         ms_per_step=r["ms"] / steps,
                         fit_kernel_tflops=wl.flops_per_eval() * wl.n_fireworks * wl.n_sparks
                         / (r["timing"]["fit_kernel_ms"] / steps / 1e3) / 1e12)
    g16 = M.MGFWA.from_workload(wl, precision="bf16", seed=seed)
    g32 = M.MGFWA.from_workload(wl, precision="fp32", seed=seed)
    lam, N = wl.n_sparks, wl.n_fireworks
    rel, agree = [], []
    for _ in range(gens):
        g16.step(1)
        st = g16.state()
        y16 = st["Yc"][:, :lam].float().cpu().numpy()
        y32 = g32.evaluate(st["SE"]).view(N, lam).cpu().numpy()
        rel.append(np.abs(y16 - y32) / np.maximum(np.abs(y32), 1e-30))
        agree.append(topk_agreement(y16, y32, lam, wl.n_guiding, 0.2))
    torch.cuda.synchronize()
    g16.close()
    g32.close()
    rel = np.concatenate([r.ravel() for r in rel])
    out["bf16_vs_fp32"] = dict(
        generations=gens, sparks=int(rel.size),
        rel_err_max=float(rel.max()), rel_err_median=float(np.median(rel)),
        topk_member_agreement=float(np.mean([a["member_agreement"] for a in agree])),
        topk_groups_identical=float(np.mean([a["groups_identical"] for a in agree])),
        best_spark_agreement=float(np.mean([a["best_spark_agreement"] for a in agree])),
        k=agree[0]["k"], group_size=agree[0]["m"])
    out["bf16_speedup"] = out["bf16"]["spark_evals_per_s"] / out["fp32"]["spark_evals_per_s"]
    return out


def batch_study(steps, seed, n_jobs=64):
    """64 independent jobs of uneven shape (D log-uniform in [1k, 50k], 2-3 layers of
    width 32-256, 64-512 sparks, 1024-4096 samples), BF16 fitness with autotuned
    launch shapes: one HIP graph launch per generation for all jobs, against the
    same jobs' own per-job graphs launched one after another."""
    import torch

    from paper_2501_03944_amd import inputs
    from paper_2501_03944_amd import mgfwa as M

    wls = inputs.mixed_jobs(n_jobs=n_jobs)
    gens = 2 * steps + 4
    jobs = [M.MGFWA.from_workload(wl, precision="bf16", seed=seed + i, max_generations=gens)
            for i, wl in enumerate(wls)]
    t0 = time.perf_counter()
    for g in jobs:
        g.autotune(3)
    tune_s = time.perf_counter() - t0
    C = sum(g.BN * (wl.n_sparks + wl.n_guiding) for g, wl in zip(jobs, wls))
    flops = sum(wl.flops_per_eval() * g.BN * (wl.n_sparks + wl.n_guiding)
                for g, wl in zip(jobs, wls))
    stream = torch.cuda.current_stream()
    b = M.Batch(jobs, stream=stream)
    b.step(1)
    for g in jobs:
        g.step(1)
    torch.cuda.synchronize()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    batched_ms = timed(lambda: b.step(steps))

    def one_by_one():
        for _ in range(steps):
            for g in jobs:
                g.step(1)

    sequential_ms = timed(one_by_one)
    b.close()
    for g in jobs:
        g.close()
    dims = [wl.dim for wl in wls]
    return dict(jobs=n_jobs, candidates_per_generation=C, D_min=min(dims), D_max=max(dims),
                autotune_s=tune_s, batched_ms_per_generation=batched_ms,
                sequential_ms_per_generation=sequential_ms,
                spark_evals_per_s=C / (batched_ms / 1e3),
                fitness_tflops_whole_step=flops / (batched_ms / 1e3) / 1e12,
                speedup_vs_sequential=sequential_ms / batched_ms)


# serving mix: (workload, share of arrivals, precision, generation budget, target loss)
SERVE_MIX = (("mlp8-16-1", 0.70, "fp32", 100, 40.0),
             ("mlp64-128-128-10", 0.25, "fp32", 30, None),
             ("mlp784-256-10", 0.05, "bf16", 10, None))


def serving_study(seconds, seed, rate=20.0, arena_gib=64, n_streams=4):
    """Poisson arrivals (rate jobs/s over `seconds`) of the SERVE_MIX shapes into the
    continuous-batching server; per-generation device latency p50/p99, throughput,
    and the offered load implied by the single-job generation times."""
    import numpy as np
    import torch

    from paper_2501_03944_amd import inputs
    from paper_2501_03944_amd import mgfwa as M

    rng = np.random.default_rng(1234 + seed)
    t, arrivals = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > seconds:
            break
        arrivals.append(t)
    shares = np.array([m[1] for m in SERVE_MIX])
    kinds = rng.choice(len(SERVE_MIX), size=len(arrivals), p=shares / shares.sum())
    wls = []
    for name, _, _, _, _ in SERVE_MIX:
        wl = inputs.workload(name)
        # device copies once; every job of the kind shares them
        wl.x = torch.from_numpy(wl.x).cuda()
        wl.y = None if wl.y is None else torch.from_numpy(wl.y).cuda()
        wl.labels = None if wl.labels is None else torch.from_numpy(wl.labels).cuda()
        wls.append(wl)
    torch.cuda.synchronize()
    srv = M.Server(arena_gib << 30, n_streams=n_streams)
    t0 = time.perf_counter()
    i, ids = 0, []
    while True:
        now = time.perf_counter() - t0
        while i < len(arrivals) and arrivals[i] <= now:
            name, _, prec, gens, target = SERVE_MIX[kinds[i]]
            ids.append(srv.submit_workload(wls[kinds[i]], sync=False, precision=prec,
                                           max_generations=gens, target_loss=target,
                                           seed=seed + i))
            i += 1
        srv.tick()
        if i == len(arrivals):
            st = srv.stats()
            if st["queued"] == 0 and st["running"] == 0:
                break
    wall = time.perf_counter() - t0
    st = srv.stats()
    infos = [srv.job(j)[0] for j in ids]
    srv.close()
    waits = [x["admit_ms"] - x["submit_ms"] for x in infos]
    turn = [x["finish_ms"] - x["submit_ms"] for x in infos]
    counts = {SERVE_MIX[k][0]: int((kinds == k).sum()) for k in range(len(SERVE_MIX))}
    # offered matrix work: every arrived job run to its full generation budget
    offered = sum(counts[m[0]] * m[3] * wl.n_fireworks * (wl.n_sparks + wl.n_guiding)
                  * wl.flops_per_eval() for m, wl in zip(SERVE_MIX, wls)) / seconds
    return dict(arrival_rate_jobs_per_s=rate, arrival_window_s=seconds, jobs=len(ids),
                mix={m[0]: dict(share=m[1], precision=m[2], generations=m[3],
                                target_loss=m[4], arrived=counts[m[0]]) for m in SERVE_MIX},
                done=st["done"], failed=st["failed"], generations=st["generations"],
                gen_latency_ms={"p50": st["gen_ms_p50"], "p99": st["gen_ms_p99"]},
                spark_evals_per_s=st["spark_evals_per_s"], wall_s=wall,
                admission_wait_ms={"p50": float(np.percentile(waits, 50)),
                                   "p99": float(np.percentile(waits, 99))},
                turnaround_ms={"p50": float(np.percentile(turn, 50)),
                               "p99": float(np.percentile(turn, 99))},
                offered_tflops_at_full_budgets=offered / 1e12,
                arena_gib=arena_gib, arena_peak_gib=st["arena_peak"] / 2**30, streams=n_streams)


def testbed_study(steps, seed, warmup=3):
    """The paper's own testbed (Sec. 4.1, eq. (1), Table 2): minimise the output
    of each fixed random MLP over its input, 8 fireworks x 512 sparks + 8 guiding
    sparks per generation.  Per net: generation time, candidate evaluations per
    second, the fitness kernels' time and FP32 MFMA rate (after autotuning their
    tile shapes), and the best output after the timed generations."""
    import torch

    from paper_2501_03944_amd import inputs
    from paper_2501_03944_amd import mgfwa as M

    out = {}
    for net_id in sorted(inputs.TESTBED_NETS):
        wl = inputs.testbed_net(net_id)
        g = M.MGFWA.from_workload(wl, seed=seed, max_generations=warmup + steps + 1)
        g.autotune(3)
        kernels = (g.fit_plan(0)["net_kernel"], g.fit_plan(1)["net_kernel"])
        g.step(warmup)
        torch.cuda.synchronize()
        g.set_timing(True)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(g.stream)
        g.step(steps)
        b.record(g.stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        t = g.timing()
        g.set_timing(False)
        x, best, gen = g.best()
        g.close()
        rows = wl.n_fireworks * wl.n_sparks
        fit_ms = t["fit_kernel_ms"] / steps
        tflops = wl.flops_per_eval() * rows / (fit_ms / 1e3) / 1e12
        out[f"net{net_id}"] = {
            "d": wl.dim, "widths": f"{wl.widths[0]}-{wl.widths[1]}x{len(wl.widths) - 2}-1",
            "act": wl.acts[0], "params": wl.n_params,
            "ms_per_generation": ms,
            "spark_evals_per_s": g.BN * (wl.n_sparks + wl.n_guiding) / (ms / 1e3),
            "fit_kernel_ms": fit_ms, "fit_kernel_tflops": tflops,
            "fit_mfma_pct_fp32_peak": 100.0 * tflops / PEAK_TFLOPS["fp32"],
            "best_output": best, "generations": gen,
            "tuned_kernel": {"explosion": kernels[0], "guiding": kernels[1]}}
    return {"fireworks": 8, "sparks": 512, "guiding": 8, "steps": steps, "nets": out}


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
    r = run_gpu(wl, precision, args.steps, args.warmup, args.seed, bool(args.autotune))
    K = args.steps
    value = r["C"] * K / (r["ms"] / 1e3)
    t = r["timing"]
    rows = wl.n_fireworks * wl.n_sparks
    flops = wl.flops_per_eval() * rows
    fit_ms = t["fit_kernel_ms"] / K
    achieved = flops / (fit_ms / 1e3) / 1e12
    peak = PEAK_TFLOPS[precision]
    traffic, traffic_src = measured_traffic(args.workload, precision)
    # algorithmic bytes of one launch: every spark's weights once (the wide kernel
    # reads them packed in its own precision), the samples once
    es = 4 if precision == "fp32" else 2
    wide = args.workload == "mlp784-256-10"
    testbed = getattr(wl, "net", None) is not None
    if testbed:   # every spark (the network input) once, the fixed parameters once
        alg_bytes = rows * wl.dim * 4 + wl.n_params * 4
    else:
        alg_bytes = rows * wl.dim * (es if wide else 4) + wl.n_samples * wl.widths[0] * es
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
                   "sparks": wl.n_sparks, "guiding": wl.n_guiding,
                   "samples": 0 if testbed else wl.n_samples,
                   "D": wl.dim, "precision": precision, "autotuned": bool(args.autotune),
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic, "traffic_source": traffic_src,
                     "algorithmic_bytes": alg_bytes,
                     "kernel": ("k_net_input (explosion-spark fitness, fixed network)" if testbed
                                else "k_fit (explosion-spark fitness)"),
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
    if args.serving_study:
        line["serving_study"] = serving_study(args.serve_seconds, args.seed)
    if args.batch_study:
        line["batch_study"] = batch_study(max(2, min(K, 10)), args.seed)
    if args.testbed_study:
        line["testbed_study"] = testbed_study(max(2, min(K, 20)), args.seed)
    if args.cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds, args.seed)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
