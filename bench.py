#!/usr/bin/env python3
"""MGFWA hot-path benchmark on one MI355X: prints one JSON line.

A step is one full MGFWA generation (explosion sparks, their fitness, ranking
and multi-guiding sparks, their fitness, selection, amplitude update, loser-out)
over the whole population, with every input already resident in HBM.  The
default workload is the 784-256-10 ReLU cross-entropy network (D = 203,530) on
8192 sparse prototype samples, 16 fireworks x 256 sparks + 4 guiding sparks,
with FP32 fitness; the same workload with BF16 fitness (FP32 accumulation, FP32
re-check of each firework's selection winner) is reported beside it.

value     = candidate evaluations per second over the timed steps
roofline  = the explosion-spark fitness kernel (the dominant kernel): algorithmic
            matmul FLOP per launch / its average duration from HIP events
bf16      = the same workload with BF16 fitness: throughput, its own roofline,
            and its error and top-k agreement against the oracle's binary64
            fitness of sampled guiding groups (computed in the CPU-baseline leg)
cpu_baseline = the CPU oracle on a bounded sample of the same workload, on all
            host threads and on one
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
    ap.add_argument("--workload", default="mlp784-256-10", choices=sorted(WORKLOAD_TAG))
    ap.add_argument("--precision", default=None, choices=["fp32", "bf16"])
    ap.add_argument("--cpu-baseline", type=int, default=1,
                    help="1: time the oracle on sampled guiding groups (all threads and one)")
    ap.add_argument("--bf16", type=int, default=1,
                    help="1: also run the workload with BF16 fitness (its own roofline, its "
                         "error and top-k agreement against the oracle)")
    ap.add_argument("--gmm-study", type=int, default=1,
                    help="1: also run the 64-128-128-10 workload in FP32")
    ap.add_argument("--latency-study", type=int, default=1,
                    help="1: per-generation latency of the 8-16-1 workload (graph replays)")
    ap.add_argument("--batch-study", type=int, default=1,
                    help="1: also run 64 mixed-shape BF16 jobs as one batched graph per generation")
    ap.add_argument("--serving-study", type=int, default=1,
                    help="1: also run a Poisson stream of mixed jobs through the serving loop")
    ap.add_argument("--serve-seconds", type=float, default=3.0, help="arrival window of that study")
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
    se_written = g.sparks_materialised
    g.close()
    return dict(C=C, ms=ms, wall=wall, timing=tinfo, graph_ms=graph_ms, best=best, gen=gen,
                se_written=se_written)


_T0 = time.perf_counter()


def log(msg):
    """Progress of the run on stderr (the JSON line alone goes to stdout)."""
    print(f"bench [{time.perf_counter() - _T0:6.1f} s] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# guiding groups (firework, group) whose sparks are scored by the oracle: one per
# quarter of the population, a different group index each
SAMPLE_GROUPS = ((0, 0), (5, 1), (10, 2), (15, 3))


def sample_generation(wl, seed, gens=3):
    """The explosion sparks of generation gens+1 of an FP32 run (the library's
    ask writes them to the workspace), with their fitness from the library's FP32
    and BF16 kernels; host copies of the rows of SAMPLE_GROUPS for the oracle."""
    import numpy as np
    import torch

    from paper_2501_03944_amd import mgfwa as M

    lam, G = wl.n_sparks, wl.n_guiding
    m = lam // G
    g32 = M.MGFWA.from_workload(wl, precision="fp32", seed=seed)
    g32.step(gens)
    W = g32.ask()
    y32 = g32.evaluate(W)
    g16 = M.MGFWA.from_workload(wl, precision="bf16", seed=seed)
    y16 = g16.evaluate(W)
    torch.cuda.synchronize()
    groups = [(f, g) for f, g in SAMPLE_GROUPS if f < wl.n_fireworks and g < G]
    idx = np.concatenate([np.arange(f * lam + g * m, f * lam + (g + 1) * m) for f, g in groups])
    rows = W[torch.from_numpy(idx).to(W.device)][:, :wl.dim].cpu().numpy()
    out = dict(t=gens + 1, groups=groups, idx=idx, rows=rows, m=m,
               y32=y32.cpu().numpy().reshape(-1, lam), y16=y16.cpu().numpy().reshape(-1, lam))
    g16.close()
    g32.close()
    return out


def cpu_baseline(wl, sample, one_core_rows=4):
    """The oracle on a bounded sample: the binary64 fitness of the sampled guiding
    groups' sparks on all host threads, and of a few of them on one thread.  The
    values also measure the GPU paths' error (returned beside the timing)."""
    import numpy as np

    from oracle import oracle as O

    p = O.Problem.from_workload(wl)
    rows = sample["rows"]
    nthreads = O.threads(0)
    t0 = time.perf_counter()
    y64 = p.loss_rows(rows)
    dt = time.perf_counter() - t0
    n1 = min(one_core_rows, len(rows))
    O.threads(1)
    t1 = time.perf_counter()
    y1 = p.loss_rows(rows[:n1])
    dt1 = time.perf_counter() - t1
    O.threads(nthreads)
    assert np.array_equal(y1, y64[:n1]), "oracle fitness depends on its thread count"
    what = (f"{len(rows)} explosion sparks of generation {sample['t']} of the same workload "
            f"({len(sample['groups'])} guiding groups of {sample['m']}), binary64 fitness")
    rec = dict(value=len(rows) / dt, unit="spark-evals/s", cores=nthreads, kind="oracle",
               sample=f"{what}, {dt:.1f} s", cpu_model=cpu_model(), host_cpus=os.cpu_count(),
               one_core=dict(value=n1 / dt1, unit="spark-evals/s", cores=1,
                             sample=f"the first {n1} of those sparks, {dt1:.1f} s"))
    return rec, y64


def group_agreement(y_run, y_ref, m, k):
    """Guiding-group decisions taken on y_run against those taken on y_ref (both
    [groups, m]): top-k and bottom-k members, whole sets, and the group's best."""
    import numpy as np

    overlap = same = best = 0
    for a, b in zip(y_run, y_ref):
        oa, ob = np.argsort(a, kind="stable"), np.argsort(b, kind="stable")
        ta, tb, ba, bb = set(oa[:k]), set(ob[:k]), set(oa[-k:]), set(ob[-k:])
        overlap += len(ta & tb) + len(ba & bb)
        same += (ta == tb) and (ba == bb)
        best += oa[0] == ob[0]
    n = len(y_run)
    return dict(topk_member_agreement=overlap / (2.0 * k * n), topk_groups_identical=same / n,
                group_best_agreement=best / n, groups=n, k=k, m=m)


def error_stats(y_run, y_ref):
    import numpy as np

    y_run, y_ref = np.asarray(y_run, np.float64).ravel(), np.asarray(y_ref, np.float64).ravel()
    rel = np.abs(y_run - y_ref) / np.maximum(np.abs(y_ref), 1e-30)
    return dict(sparks=int(rel.size), rel_err_max=float(rel.max()),
                rel_err_median=float(np.median(rel)))


def vs_reference(y_run, y_ref, m, sigma=0.2):
    """Error and guiding-group agreement of y_run ([groups, m]) against y_ref."""
    k = max(1, int(sigma * m))
    return dict(**error_stats(y_run, y_ref), **group_agreement(y_run, y_ref, m, k))


def sampled_groups(y, sample, lam):
    """[groups, m] fitness of the sampled guiding groups from a [fireworks, lam] array."""
    import numpy as np

    m = sample["m"]
    return np.stack([y[f, g * m:(g + 1) * m] for f, g in sample["groups"]])


def kernel_roofline(wl, precision, fit_ms, workload_name):
    """Roofline record of the explosion-spark fitness kernel from its average
    launch duration (HIP events on the library's stream)."""
    rows = wl.n_fireworks * wl.n_sparks
    flops = wl.flops_per_eval() * rows
    achieved = flops / (fit_ms / 1e3) / 1e12
    peak = PEAK_TFLOPS[precision]
    traffic, traffic_src = measured_traffic(workload_name, precision)
    es = 4 if precision == "fp32" else 2
    wide = workload_name == "mlp784-256-10"
    testbed = getattr(wl, "net", None) is not None
    if testbed:   # every spark (the network input) once, the fixed parameters once
        alg_bytes = rows * wl.dim * 4 + wl.n_params * 4
        kernel = "k_net_input / k_net_layer (explosion-spark fitness, fixed network)"
    else:         # every spark's weights once (the wide kernel reads them packed in its
        # own precision), the samples once
        alg_bytes = rows * wl.dim * (es if wide else 4) + wl.n_samples * wl.widths[0] * es
        kernel = ("k_fit_wide_pipe" if precision == "bf16" else "k_fit_wide32") if wide else "k_fit"
        kernel += " (explosion-spark fitness)"
    return {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic, "traffic_source": traffic_src,
            "algorithmic_bytes": alg_bytes, "kernel": kernel, "flop_per_launch": flops,
            "avg_launch_ms": fit_ms}


def phase_hbm(wl, precision, timing, steps, se_written, wide):
    """HBM rate of the state-path phases from their algorithmic bytes per
    generation: explosion (writes every spark once in the layout the fitness reads,
    plus the FP32 rows when they are stored; reads each firework row), guiding
    (writes the guiding sparks; reads each firework row, and the 2k member rows of
    every group when they are stored rather than regenerated), selection (at most
    one candidate row read and one firework row written per firework, plus the
    best row)."""
    BN, lam, G, D = wl.n_fireworks, wl.n_sparks, wl.n_guiding, wl.dim
    k = max(1, int(0.2 * (lam // G)))
    es = (4 if precision == "fp32" else 2) if wide else 4
    expl = BN * lam * D * es + (BN * lam * D * 4 if wide and se_written else 0) + BN * D * 4
    guide = BN * G * D * 4 + BN * D * 4 + (0 if not se_written else BN * G * 2 * k * D * 4)
    select = 2 * BN * D * 4 + D * 4
    out = {}
    for name, phase, nbytes in (("explosion", "explosion", expl), ("guiding", "guiding", guide),
                                ("selection", "selection", select)):
        ms = timing["phase_ms"][phase] / steps
        out[name] = dict(bytes=nbytes, ms=ms, GB_s=nbytes / (ms / 1e3) / 1e9,
                         frac_of_8TB_s=nbytes / (ms / 1e3) / 8e12)
    return out


def batch_study(steps, seed, n_jobs=64):
    """64 independent jobs of uneven shape (D log-uniform in [1k, 50k], 2-3 layers of
    width 32-256, 64-512 sparks, 1024-4096 samples), BF16 fitness with autotuned
    launch shapes: one HIP graph launch per generation for all jobs, against the
    same jobs' own per-job graphs, each on its job's stream."""
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
    stream = torch.cuda.Stream()   # the library never takes the null stream
    stream.wait_stream(torch.cuda.current_stream())
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
        # each job on its own stream (how jobs run without a batch), bracketed
        # by the timing stream on both sides
        for g in jobs:
            g.stream.wait_stream(stream)
        for _ in range(steps):
            for g in jobs:
                g.step(1)
        for g in jobs:
            stream.wait_stream(g.stream)

    own_ms = timed(one_by_one)
    b.close()
    for g in jobs:
        g.close()
    dims = [wl.dim for wl in wls]
    return dict(jobs=n_jobs, candidates_per_generation=C, D_min=min(dims), D_max=max(dims),
                autotune_s=tune_s, batched_ms_per_generation=batched_ms,
                own_streams_ms_per_generation=own_ms,
                spark_evals_per_s=C / (batched_ms / 1e3),
                fitness_tflops_whole_step=flops / (batched_ms / 1e3) / 1e12,
                speedup_vs_own_streams=own_ms / batched_ms)


# serving mix: (workload, share of arrivals, precision, generation budget, target loss).
# Every job runs to its target loss or 300 generations.  The targets are losses the
# shape's MGFWA runs reach at about 60 % of that budget (8-16-1: twice the noise
# variance of its targets; the two cross-entropy shapes: 1.0, from ln 10 = 2.3 at
# chance level and thousands at the random start).
SERVE_MIX = (("mlp8-16-1", 0.70, "fp32", 300, 0.02),
             ("mlp64-128-128-10", 0.25, "fp32", 300, 1.0),
             ("mlp784-256-10", 0.05, "bf16", 300, 1.0))


def alone_gen_ms(wl, precision, seed, gens=8):
    """Device time of one generation of one job of this shape running alone."""
    import torch

    from paper_2501_03944_amd import mgfwa as M

    g = M.MGFWA.from_workload(wl, precision=precision, seed=seed, max_generations=300)
    g.step(2)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(g.stream)
    g.step(gens)
    b.record(g.stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / gens
    g.close()
    return ms


def serving_study(seconds, seed, rate=20.0, arena_gib=64, n_streams=4):
    """Poisson arrivals (rate jobs/s over `seconds`) of the SERVE_MIX shapes into the
    continuous-batching server; per-generation device latency p50/p99, throughput,
    admission wait, and the offered load against one GPU's capacity from the
    single-job generation times."""
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
    wls, gen_ms = [], []
    for name, _, prec, _, _ in SERVE_MIX:
        wl = inputs.workload(name)
        gen_ms.append(alone_gen_ms(wl, prec, seed))
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
    gens_run = {m[0]: [x["generations"] for x, k in zip(infos, kinds) if k == j]
                for j, m in enumerate(SERVE_MIX)}
    stopped = {m[0]: sum(1 for x, k in zip(infos, kinds) if k == j and x["generations"] < m[3])
               for j, m in enumerate(SERVE_MIX)}
    # offered load in GPU-seconds per second: every arrived job at its full budget
    # (and at the generations it actually ran), each generation at its alone time
    offered_full = sum(counts[m[0]] * m[3] * ms for m, ms in zip(SERVE_MIX, gen_ms)) / 1e3 / seconds
    offered_run = sum(sum(gens_run[m[0]]) * ms for m, ms in zip(SERVE_MIX, gen_ms)) / 1e3 / seconds
    offered = sum(counts[m[0]] * m[3] * wl.n_fireworks * (wl.n_sparks + wl.n_guiding)
                  * wl.flops_per_eval() for m, wl in zip(SERVE_MIX, wls)) / seconds
    return dict(arrival_rate_jobs_per_s=rate, arrival_window_s=seconds, jobs=len(ids),
                mix={m[0]: dict(share=m[1], precision=m[2], generation_budget=m[3],
                                target_loss=m[4], arrived=counts[m[0]],
                                stopped_at_target=stopped[m[0]],
                                mean_generations=float(np.mean(gens_run[m[0]]))
                                if gens_run[m[0]] else 0.0,
                                alone_ms_per_generation=ms)
                     for m, ms in zip(SERVE_MIX, gen_ms)},
                done=st["done"], failed=st["failed"], generations=st["generations"],
                gen_latency_ms={"p50": st["gen_ms_p50"], "p99": st["gen_ms_p99"]},
                spark_evals_per_s=st["spark_evals_per_s"], wall_s=wall,
                admission_wait_ms={"p50": float(np.percentile(waits, 50)),
                                   "p99": float(np.percentile(waits, 99))},
                turnaround_ms={"p50": float(np.percentile(turn, 50)),
                               "p99": float(np.percentile(turn, 99))},
                offered_load_gpu_s_per_s={"at_full_budgets": offered_full,
                                          "at_generations_run": offered_run},
                served_gpu_s_per_s=offered_run * seconds / wall,
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


def latency_study(seed, gens=100, warmup=5):
    """Per-generation latency of the 8-16-1 workload (4 fireworks x 32 sparks): each
    generation one HIP graph replay, bracketed by its own events."""
    import numpy as np
    import torch

    from paper_2501_03944_amd import inputs
    from paper_2501_03944_amd import mgfwa as M

    wl = inputs.workload("mlp8-16-1")
    g = M.MGFWA.from_workload(wl, seed=seed, max_generations=gens + warmup)
    g.step(warmup)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(gens)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(g.stream)
        g.step(1)
        b.record(g.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    _, best, gen = g.best()
    g.close()
    C = wl.n_fireworks * (wl.n_sparks + wl.n_guiding)
    return dict(workload=WORKLOAD_TAG["mlp8-16-1"], generations=gens,
                gen_latency_ms={"p50": float(np.percentile(ms, 50)),
                                "p99": float(np.percentile(ms, 99)), "mean": float(ms.mean())},
                host_ms_per_generation=wall / gens * 1e3,
                spark_evals_per_s=C * gens / wall, best_fitness=best)


def workload_record(name, precision, steps, warmup, seed, autotune):
    """Throughput and fitness-kernel roofline of one workload at one precision."""
    from paper_2501_03944_amd import inputs

    wl = inputs.workload(name)
    r = run_gpu(wl, precision, steps, warmup, seed, autotune)
    t = r["timing"]
    rec = dict(workload=WORKLOAD_TAG[name], precision=precision,
               value=r["C"] * steps / (r["ms"] / 1e3), unit="spark-evals/s",
               ms_per_step=r["ms"] / steps,
               roofline=kernel_roofline(wl, precision, t["fit_kernel_ms"] / steps, name),
               gen_latency_ms={"p50": t["gen_ms_p50"], "p99": t["gen_ms_p99"]},
               phase_ms_per_step={k: v / steps for k, v in t["phase_ms"].items()},
               graph_ms_per_step=r["graph_ms"] / steps, best_fitness=r["best"])
    if precision == "bf16":
        rec["check_fit_ms_per_step"] = t["check_fit_ms"] / steps
    return rec, r, wl


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the hot path is measured on one GPU's share).", file=sys.stderr)
        sys.exit(2)
    from paper_2501_03944_amd import inputs

    wl = inputs.workload(args.workload)
    precision = args.precision or "fp32"
    testbed = getattr(wl, "net", None) is not None
    calibration_copy(args.calib_copy_mib)
    r = run_gpu(wl, precision, args.steps, args.warmup, args.seed, bool(args.autotune))
    log(f"{args.workload} {precision}: {r['ms'] / args.steps:.3f} ms per generation")
    K = args.steps
    t = r["timing"]
    wide = args.workload == "mlp784-256-10"
    line = {
        "metric": METRIC,
        "value": r["C"] * K / (r["ms"] / 1e3),
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
        "roofline": kernel_roofline(wl, precision, t["fit_kernel_ms"] / K, args.workload),
        "gen_latency_ms": {"p50": t["gen_ms_p50"], "p99": t["gen_ms_p99"],
                           "mean": t["gen_ms_mean"]},
        "phase_ms_per_step": {k: v / K for k, v in t["phase_ms"].items()},
        "state_path_hbm": None if testbed else phase_hbm(wl, precision, t, K, r["se_written"], wide),
        "graph_ms_per_step": r["graph_ms"] / K,
        "best_fitness": r["best"],
        "generations_run": r["gen"],
    }
    line["mfma_pct_peak"] = 100.0 * line["roofline"]["frac"]
    bf16 = None
    if args.bf16 and precision == "fp32" and not testbed:
        bf16, rb, _ = workload_record(args.workload, "bf16", K, args.warmup, args.seed,
                                      bool(args.autotune))
        bf16["dtype"] = "bf16"
        bf16["state_path_hbm"] = phase_hbm(wl, "bf16", rb["timing"], K, rb["se_written"], wide)
        bf16["speedup_vs_fp32"] = bf16["value"] / line["value"]
        line["bf16"] = bf16
        log(f"{args.workload} bf16: {bf16['ms_per_step']:.3f} ms per generation")
    sample = None
    if not testbed and (bf16 is not None or args.cpu_baseline):
        sample = sample_generation(wl, args.seed)
        log("sampled generation taken")
        if bf16 is not None:   # every explosion spark of the sampled generation: BF16 vs FP32
            m = sample["m"]
            y16 = sample["y16"].reshape(-1, m)
            y32 = sample["y32"].reshape(-1, m)
            bf16["vs_fp32_gpu"] = dict(generation=sample["t"], **vs_reference(y16, y32, m))
    if args.gmm_study and args.workload != "mlp64-128-128-10":
        line["gmm_study"], _, _ = workload_record("mlp64-128-128-10", "fp32", K, args.warmup,
                                                  args.seed, bool(args.autotune))
        log("64-128-128-10 study done")
    if args.latency_study:
        line["latency_study"] = latency_study(args.seed)
        log("latency study done")
    if args.serving_study:
        line["serving_study"] = serving_study(args.serve_seconds, args.seed)
        log("serving study done")
    if args.batch_study:
        line["batch_study"] = batch_study(max(2, min(K, 10)), args.seed)
        log("batch study done")
    if args.testbed_study:
        line["testbed_study"] = testbed_study(max(2, min(K, 20)), args.seed)
        log("testbed study done")
    if args.cpu_baseline and sample is not None:
        rec, y64 = cpu_baseline(wl, sample)
        line["cpu_baseline"] = rec
        log("cpu baseline done")
        y64 = y64.reshape(-1, sample["m"])
        line["fp32_vs_oracle"] = dict(generation=sample["t"], **vs_reference(
            sampled_groups(sample["y32"], sample, wl.n_sparks), y64, sample["m"]))
        if bf16 is not None:
            bf16["vs_oracle"] = dict(generation=sample["t"], **vs_reference(
                sampled_groups(sample["y16"], sample, wl.n_sparks), y64, sample["m"]))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
