"""Benchmark: general CQK solve, n = 1e8, FP64, on one MI355X.

One step = one whole solve (cqk_solve_f64: the sampled-bracket estimate, the
Newton passes with compaction of resolved indices, then the x-writing pass)
over inputs already resident in HBM, with the compaction threshold theta
tuned on the instance first (cqk_tune_theta_f64; --theta fixes it instead).
Prints one JSON line: the metric (elements/s = n / ms per solve), the
roofline of the first Newton pass and of the x-writing pass (algorithmic
bytes per launch over the average launch time from HIP events stamped by the
dispatches in the timed region, against 8 TB/s, and the measured HBM traffic
per launch when the committed counter summary matches the kernel source),
each pass of one solve (indices read, bytes, µs, GB/s), the same solve on
seeds 1-3 of both n = 1e8
generators, the n = 1e5 latency case (seeds 1-20, median over seeds of the
best run), the oracle's CPU rate (best of 3 on a 1e7 sample, best of 10 at
1e5), and "extras": the other workloads (correlated CQK, simplex and l1 at
n = 1e8 with dense and sparse output, warm starts from a previous solution,
batched and differentiable batched projections) on the same GPU, each
checked for its status.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n N]
                    [--no-cpu-baseline] [--no-extras] [--calibrate-copy]
                    [--oracle-full] [--theta T]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gen_kernels_cqk_uniform_1e8.traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2603_15910_amd", "csrc", "cqk_general.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cpu_desc():
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    return os.cpu_count(), model


def _oracle_best(n, seed, reps):
    """Best of reps single-threaded oracle solves (exact breakpoint sort)."""
    from oracle import cqk_oracle as O
    from paper_2603_15910_amd import workloads as W
    inst = W.cqk_uniform(n, seed)
    best = None
    for _ in range(reps):
        t0 = time.perf_counter()
        res = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
        dt = time.perf_counter() - t0
        assert res.status == O.OK
        best = dt if best is None else min(best, dt)
    return best


def cpu_baseline(n_sample: int, reps: int = 3, full: bool = False):
    """The oracle (exact breakpoint-sort solver, numpy, one thread) on a
    bounded sample of the same workload, best of reps; also the C1 size
    (n = 1e5, best of 10) and, with full, the whole workload (n = 1e8, best
    of 3)."""
    ncpu, model = host_cpu_desc()
    dt = _oracle_best(n_sample, 1, reps)
    out = {"value": n_sample / dt, "unit": "elements/s", "cores": 1, "kind": "oracle",
           "sample": f"cqk_uniform n={n_sample} seed=1 ({n_sample / 1e8:g} of the workload), "
                     f"exact breakpoint-sort solve (numpy, 1 thread), best of {reps}: "
                     f"{dt:.2f} s on {model} ({ncpu} logical CPUs)"}
    dt5 = _oracle_best(100_000, 1, 10)
    out["c1_n1e5_best_of_10_s"] = dt5
    if full:
        dt8 = _oracle_best(100_000_000, 1, 3)
        out["n1e8_best_of_3_s"] = dt8
        out["n1e8_elements_per_s"] = 1e8 / dt8
    return out


def measured_traffic(kernel_sha, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    if it was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_sha:
        return None
    return rec.get("bytes_per_launch", {}).get(kernel)


def timed(fn, reps, sync):
    out = []
    for _ in range(reps):
        sync()
        t0 = time.perf_counter()
        fn()
        sync()
        out.append((time.perf_counter() - t0) * 1e3)
    return statistics.median(out)


def graph_replay_ms(torch, fn, reps):
    """Captures fn (queue-only, no host sync) in a graph and times replays
    with events on the replay stream."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps

def pass_table(ctx, in_bytes=40.0):
    """Per grid pass of the last timed, traced general solve: indices read
    (n_k), survivors written, algorithmic bytes, kernel µs and GB/s."""
    ms = ctx.pass_ms()
    recs = [t for t in ctx.trace() if t["kind"] in (0, 1, 2, 8, 9)]
    rows = []
    for k, t in enumerate(recs):
        per_in = in_bytes if t["source"] == 0 else 32.0
        # n_out: survivors written for both sides of the evaluation (the
        # sample's record: survivors it predicts, nothing written)
        nbytes = per_in * t["n_in"] + (32.0 * t["n_out"] if t["kind"] in (1, 2) else 0.0)
        us = ms[k] * 1e3 if k < len(ms) else None
        rows.append({"kind": {0: "lambda0", 1: "evaluate", 2: "breakpoint",
                              8: "sample", 9: "sample2"}[t["kind"]],
                     "source": "original" if t["source"] == 0 else "compacted",
                     "n_in": t["n_in"], "n_out": t["n_out"], "adopted": bool(t["compacted"]),
                     "bytes": nbytes, "us": us,
                     "gbs": nbytes / (us * 1e-6) / 1e9 if us else None,
                     "frac_of_peak": nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS if us else None})
    # passes queued after the loop stopped: no trace record, no bytes
    tail = [m * 1e3 for m in ms[len(recs):]]
    return rows, tail


def c1_latency(ctx, dev, torch, seeds=range(1, 21), runs=20):
    """C1: general CQK, n = 1e5, FP64, lambda_0 = 0, no compaction, seeds
    1-20.  Per seed the minimum over runs, then the median over seeds, of the
    whole call (wall clock, one host wait) and of its kernels alone (events).
    The 4 MB working set is cache-resident: a latency figure, not an HBM one."""
    from paper_2603_15910_amd import workloads as W
    sync = torch.cuda.synchronize
    wall, kern, iters, per_it = [], [], [], []
    for seed in seeds:
        inst = W.cqk_uniform(100_000, seed)
        t = [torch.from_numpy(inst[k]).to(dev) for k in "dablu"]
        x = torch.empty_like(t[0])
        r = inst["r"]
        best_w = best_k = None
        info = None
        for _ in range(runs):
            sync()
            t0 = time.perf_counter()
            _, info = ctx.solve(*t, r, out=x, compaction="off")
            w = (time.perf_counter() - t0) * 1e3
            best_w = w if best_w is None else min(best_w, w)
        for _ in range(runs):
            _, inf = ctx.solve(*t, r, out=x, compaction="off", timing=True)
            k = inf["pass_ms"] + inf["finalize_ms"]
            best_k = k if best_k is None else min(best_k, k)
        assert info["status"] == 0, info
        wall.append(best_w)
        kern.append(best_k)
        iters.append(info["iterations"])
        per_it.append(best_w / max(1, info["iterations"]))
    return {"workload": "cqk_uniform n=100000 fp64, lambda0=0, compaction=off, seeds 1-20",
            "ms_median_of_min": statistics.median(wall),
            "kernel_ms_median_of_min": statistics.median(kern),
            "iterations_median": statistics.median(iters),
            "ms_per_iteration_median": statistics.median(per_it),
            "elements_per_s": 1e5 / (statistics.median(wall) * 1e-3),
            "runs_per_seed": runs}


def c2_seeds(ctx, dev, torch, gen, seeds=(1, 2, 3), reps=5):
    """C2 on seeds 1-3: ms per solve (median of reps), iterations."""
    from paper_2603_15910_amd import workloads as W
    sync = torch.cuda.synchronize
    out = []
    for seed in seeds:
        inst = getattr(W, gen)(100_000_000, seed)
        t = [torch.from_numpy(inst[k]).to(dev) for k in "dablu"]
        r = inst["r"]
        del inst
        x = torch.empty_like(t[0])
        ctx.solve(*t, r, out=x)
        ms = timed(lambda: ctx.solve(*t, r, out=x), reps, sync)
        _, info = ctx.solve(*t, r, out=x)
        assert info["status"] == 0, info
        out.append({"seed": seed, "ms": ms, "elements_per_s": 1e8 / (ms * 1e-3),
                    "iterations": info["iterations"]})
        del t, x
        torch.cuda.empty_cache()
    return out


EXTRA_SECTIONS = ("correlated", "simplex", "warm", "batched", "differentiable", "spg")


def extras(ctx, dev, torch, sections=EXTRA_SECTIONS, row_loop=True):
    import paper_2603_15910_amd as cqk
    from paper_2603_15910_amd import workloads as W
    sync = torch.cuda.synchronize
    ex = {}
    default_sched = ctx.batch_schedule()

    # general CQK, correlated variant (n = 1e8, FP64)
    if "correlated" in sections:
        ex.update(extra_correlated(ctx, dev, torch))
    if "simplex" in sections:
        ex.update(extra_simplex(ctx, dev, torch))
    if "warm" in sections:
        ex.update(extra_warm(ctx, dev, torch))
    if "batched" in sections:
        ex.update(extra_batched(ctx, dev, torch, row_loop))
    if "differentiable" in sections:
        ex.update(extra_differentiable(ctx, dev, torch))
    if "spg" in sections:
        ex.update(extra_spg(ctx, dev, torch))
    ctx.set_batch_schedule(**default_sched)
    ctx.set_batch_schedule(**default_sched, backward=True)
    return ex


def copy_ceiling(torch):
    """Read + write GB/s of a 1 GiB device-to-device copy, best of 5."""
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        t = e0.elapsed_time(e1)
        best = t if best is None else min(best, t)
    del src, dst
    return 2.0 * (1 << 30) / (best * 1e-3) / 1e9


def extra_correlated(ctx, dev, torch):
    from paper_2603_15910_amd import workloads as W
    sync = torch.cuda.synchronize
    ex = {}
    inst = W.cqk_correlated(100_000_000, 1)
    t = [torch.from_numpy(inst[k]).to(dev) for k in "dablu"]
    r = inst["r"]
    del inst
    x = torch.empty_like(t[0])
    ctx.solve(*t, r, out=x)
    ms = timed(lambda: ctx.solve(*t, r, out=x), 5, sync)
    _, info = ctx.solve(*t, r, out=x, timing=True, trace=True)
    ex["cqk_correlated_1e8_f64"] = {
        "ms": ms, "elements_per_s": 1e8 / (ms * 1e-3), "iterations": info["iterations"],
        "status": info["status_name"],
        "pass_gbs": info["pass_bytes"] / (info["pass_ms"] * 1e-3) / 1e9,
        "finalize_gbs": info["finalize_bytes"] / (info["finalize_ms"] * 1e-3) / 1e9}
    # the eq. (CQKlambda0) start instead of lambda_0 = 0
    ctx.solve(*t, r, out=x, lambda0="formula")
    ms = timed(lambda: ctx.solve(*t, r, out=x, lambda0="formula"), 5, sync)
    _, info = ctx.solve(*t, r, out=x, lambda0="formula", timing=True)
    ex["cqk_correlated_1e8_f64_formula_start"] = {
        "ms": ms, "elements_per_s": 1e8 / (ms * 1e-3), "iterations": info["iterations"],
        "status": info["status_name"],
        "pass_gbs": info["pass_bytes"] / (info["pass_ms"] * 1e-3) / 1e9}
    del t, x
    torch.cuda.empty_cache()
    # FP32 arrays (FP64 arithmetic), both generators, lambda_0 = 0
    for gen in ("uniform", "correlated"):
        inst = W.cqk_uniform(100_000_000, 1) if gen == "uniform" else \
            W.cqk_correlated(100_000_000, 1)
        t = [torch.from_numpy(inst[k].astype(np.float32)).to(dev) for k in "dablu"]
        r = float(inst["r"])
        del inst
        x = torch.empty_like(t[0])
        ctx.solve(*t, r, out=x)
        ms = timed(lambda: ctx.solve(*t, r, out=x), 5, sync)
        _, info = ctx.solve(*t, r, out=x)
        ex[f"cqk_{gen}_1e8_f32in"] = {
            "ms": ms, "elements_per_s": 1e8 / (ms * 1e-3), "iterations": info["iterations"],
            "status": info["status_name"]}
        del t, x
        torch.cuda.empty_cache()
    return ex


def extra_simplex(ctx, dev, torch):
    from paper_2603_15910_amd import workloads as W
    sync = torch.cuda.synchronize
    ex = {}
    # simplex and l1 projections, n = 1e8, FP32 inputs
    n = 100_000_000
    for dist in ("normal", "uniform"):
        y = torch.from_numpy(W.simplex_input(n, 1, dist, np.float32)).to(dev)
        xs = torch.empty_like(y)
        for start in ("condat", "zero"):
            for accum in ("f64", "f32"):
                kw = dict(lambda0=start, accum=accum)
                ctx.project_simplex(y, 1.0, out=xs, **kw)
                ms = timed(lambda: ctx.project_simplex(y, 1.0, out=xs, **kw), 5, sync)
                _, info = ctx.project_simplex(y, 1.0, out=xs, timing=True, trace=True, **kw)
                ex[f"simplex_{dist}_1e8_f32in_{accum}acc_{start}"] = {
                    "ms": ms, "elements_per_s": n / (ms * 1e-3), "iterations": info["iterations"],
                    "n_after_init": info["n_after_init"], "status": info["status_name"],
                    "gbs_total": (info["pass_bytes"] + info["finalize_bytes"]) / (ms * 1e-3) / 1e9}
        # the same projection returned as its support (no dense x written)
        out = (torch.empty(1 << 20, dtype=torch.int64, device=dev),
               torch.empty(1 << 20, dtype=torch.float32, device=dev))
        for kind, fn in (("simplex", ctx.project_simplex_sparse), ("l1", ctx.project_l1_sparse)):
            fn(y, 1.0, out=out)
            ms = timed(lambda: fn(y, 1.0, out=out), 5, sync)
            _, _, info = fn(y, 1.0, out=out, timing=True)
            ex[f"{kind}_{dist}_1e8_f32in_f64acc_condat_sparse"] = {
                "ms": ms, "elements_per_s": n / (ms * 1e-3), "iterations": info["iterations"],
                "nnz": info["nnz"], "status": info["status_name"],
                "output_ms": info["finalize_ms"]}
        del out
        # l1 ball of radius 1 (on U[0,1] input this is the simplex problem)
        for start in ("condat", "zero"):
            for accum in ("f64", "f32"):
                kw = dict(lambda0=start, accum=accum)
                ctx.project_l1(y, 1.0, out=xs, **kw)
                ms = timed(lambda: ctx.project_l1(y, 1.0, out=xs, **kw), 5, sync)
                _, info = ctx.project_l1(y, 1.0, out=xs, **kw)
                ex[f"l1_{dist}_1e8_f32in_{accum}acc_{start}"] = {
                    "ms": ms, "elements_per_s": n / (ms * 1e-3), "iterations": info["iterations"],
                    "status": info["status_name"]}
        del y, xs
        torch.cuda.empty_cache()
    return ex


def extra_warm(ctx, dev, torch):
    """Warm starts as an outer loop uses them: the problem moves a little
    (a, or y, perturbed by 1e-3 of its deviation) and the previous solution
    is the estimate; cold solves of the same problem beside them."""
    from paper_2603_15910_amd import workloads as W
    sync = torch.cuda.synchronize
    ex = {}
    n = 100_000_000

    def entry(ms, info):
        return {"ms": ms, "elements_per_s": n / (ms * 1e-3), "iterations": info["iterations"],
                "lambda0": info["lambda0"], "lambda": info["lambda"],
                "status": info["status_name"]}

    inst = W.cqk_uniform(n, 1)
    t = [torch.from_numpy(inst[k]).to(dev) for k in "dablu"]
    r = inst["r"]
    xprev = torch.empty_like(t[0])
    ctx.solve(*t, r, out=xprev)
    t[1] = torch.from_numpy(W.perturbed(inst["a"], 2, 1e-3)).to(dev)
    del inst
    x = torch.empty_like(xprev)
    for name, kw in (("warm", dict(xbar=xprev)), ("cold", {})):
        ctx.solve(*t, r, out=x, **kw)
        ms = timed(lambda: ctx.solve(*t, r, out=x, **kw), 5, sync)
        _, info = ctx.solve(*t, r, out=x, **kw)
        ex[f"cqk_uniform_1e8_f64_perturbed_{name}"] = entry(ms, info)
    del t, x, xprev
    torch.cuda.empty_cache()

    y0 = W.simplex_input(n, 1, "normal", np.float32)
    y = torch.from_numpy(y0).to(dev)
    y1 = torch.from_numpy(W.perturbed(y0, 2, 1e-3)).to(dev)
    del y0
    for kind, fn, rad in (("simplex", ctx.project_simplex, 1.0), ("l1", ctx.project_l1, 1.0)):
        xprev = torch.empty_like(y)
        fn(y, rad, out=xprev)
        x = torch.empty_like(y)
        for name, kw in (("warm", dict(xbar=xprev)), ("cold", {})):
            fn(y1, rad, out=x, **kw)
            ms = timed(lambda: fn(y1, rad, out=x, **kw), 5, sync)
            _, info = fn(y1, rad, out=x, **kw)
            e = entry(ms, info)
            e["n_after_init"] = info["n_after_init"]
            ex[f"{kind}_normal_1e8_f32in_perturbed_{name}"] = e
        del xprev, x
    del y, y1
    torch.cuda.empty_cache()
    return ex


def extra_batched(ctx, dev, torch, row_loop=True):
    from paper_2603_15910_amd import workloads as W
    sync = torch.cuda.synchronize
    ex = {}
    # batched simplex: 8192 rows, lengths log-uniform in [64, 65536]
    off, yb = W.batched_simplex_input(8192, 64, 65536, 1)
    total = int(off[-1])
    offs = torch.from_numpy(off).to(dev)
    ybt = torch.from_numpy(yb).to(dev)
    xb = torch.empty_like(ybt)
    default_sched = ctx.batch_schedule()
    ctx.project_simplex_batched(ybt, offs, 1.0, out=xb)
    ms_default = timed(lambda: ctx.project_simplex_batched(ybt, offs, 1.0, out=xb), 10, sync)
    sched, tune_ms = ctx.tune_batched(ybt, offs, 1.0, repeats=3, out=xb)
    ms = timed(lambda: ctx.project_simplex_batched(ybt, offs, 1.0, out=xb), 10, sync)
    _, info = ctx.project_simplex_batched(ybt, offs, 1.0, out=xb)
    graph_ms = graph_replay_ms(torch, lambda: ctx.project_simplex_batched(
        ybt, offs, 1.0, out=xb, sync=False), 20)
    # comparator: one plain solve per row (same library, same stream)
    loop_ms = None
    if row_loop:
        views = [ybt[int(off[s]):int(off[s + 1])] for s in range(8192)]
        outs = [xb[int(off[s]):int(off[s + 1])] for s in range(8192)]
        sync()
        t0 = time.perf_counter()
        for v, o in zip(views, outs):
            ctx.project_simplex(v, 1.0, out=o)
        sync()
        loop_ms = (time.perf_counter() - t0) * 1e3
        del views, outs
    ex["batched_simplex_8192rows"] = {
        "rows": 8192, "elements": total, "ms": ms, "elements_per_s": total / (ms * 1e-3),
        "gbs_8B_per_elem": 8.0 * total / (ms * 1e-3) / 1e9, "status": info["status_name"],
        "graph_replay_ms": graph_ms,
        "graph_gbs_8B_per_elem": 8.0 * total / (graph_ms * 1e-3) / 1e9,
        "schedule": sched, "tuned_kernel_ms": tune_ms,
        "default_schedule": default_sched, "default_schedule_ms": ms_default,
        "rows_spilled": info["rows_spilled"],
        "per_row_loop_ms": loop_ms,
        "speedup_vs_per_row_loop": (loop_ms / ms) if loop_ms else None}
    del ybt, xb, offs
    torch.cuda.empty_cache()
    ex.update(extra_batched_cqk(ctx, dev, torch, row_loop))
    return ex


def extra_batched_cqk(ctx, dev, torch, row_loop=True):
    """Batched general CQK, FP64: 8192 rows of log-uniform length in
    [64, 65536], forward and the VJP w.r.t. a and r."""
    from paper_2603_15910_amd import workloads as W
    sync = torch.cuda.synchronize
    off, inst = W.cqk_batched(8192, 64, 65536, 1)
    total = int(off[-1])
    offs = torch.from_numpy(off).to(dev)
    t = [torch.from_numpy(inst[k]).to(dev) for k in "dablu"]
    r = torch.from_numpy(inst["r"]).to(dev)
    del inst
    x = torch.empty_like(t[0])
    ctx.solve_batched(*t, offs, r, out=x)
    ms_default = timed(lambda: ctx.solve_batched(*t, offs, r, out=x), 5, sync)
    sched, _ = ctx.tune_batched_cqk(*t, offs, r, repeats=2)
    ms = timed(lambda: ctx.solve_batched(*t, offs, r, out=x), 5, sync)
    _, info = ctx.solve_batched(*t, offs, r, out=x)
    g = torch.randn(total, dtype=torch.float64, device=dev,
                    generator=torch.Generator(device=dev).manual_seed(5))
    ga = torch.empty_like(g)
    gr = torch.empty(8192, dtype=torch.float64, device=dev)
    bwd = lambda: ctx.solve_batched_backward(x, g, t[0], t[2], t[3], t[4], offs, grad_a=ga,
                                             grad_r=gr)
    bwd()
    ms_b_default = timed(bwd, 5, sync)
    sched_b, _ = ctx.tune_batched_cqk(*t, offs, r, repeats=2, backward=True, x=x, g=g)
    ms_b = timed(bwd, 5, sync)
    # comparator: one plain solve per row over the first 512 rows, scaled
    loop_ms = None
    if row_loop:
        rr = r.cpu().numpy()
        k = 512
        sync()
        t0 = time.perf_counter()
        for s in range(k):
            lo, hi = int(off[s]), int(off[s + 1])
            ctx.solve(*[v[lo:hi] for v in t], float(rr[s]), out=x[lo:hi])
        sync()
        loop_ms = (time.perf_counter() - t0) * 1e3 * (8192 / k)
    out = {"batched_cqk_8192rows_f64": {
        "rows": 8192, "elements": total, "ms": ms, "elements_per_s": total / (ms * 1e-3),
        "mean_iterations": info["passes"] / 8192, "max_iterations": info["iterations"],
        "gbs_40B_per_elem_per_iteration": 40.0 * total * info["passes"] / 8192 / (ms * 1e-3) / 1e9,
        "status": info["status_name"], "schedule": sched, "default_schedule_ms": ms_default,
        "backward_ms": ms_b, "backward_schedule": sched_b,
        "backward_default_schedule_ms": ms_b_default,
        "backward_gbs_48B_per_elem": 48.0 * total / (ms_b * 1e-3) / 1e9,
        "per_row_loop_ms_scaled_from_512_rows": loop_ms,
        "speedup_vs_per_row_loop": (loop_ms / ms) if loop_ms else None}}
    # the same rows as float32 arrays (float64 arithmetic), schedules tuned on them
    t32 = [v.float() for v in t]
    x32 = torch.empty_like(t32[0])
    g32 = g.float()
    ga32 = torch.empty_like(g32)
    sched32, _ = ctx.tune_batched_cqk(*t32, offs, r, repeats=2)
    ctx.solve_batched(*t32, offs, r, out=x32)
    ms32 = timed(lambda: ctx.solve_batched(*t32, offs, r, out=x32), 5, sync)
    _, info32 = ctx.solve_batched(*t32, offs, r, out=x32)
    bwd32 = lambda: ctx.solve_batched_backward(x32, g32, t32[0], t32[2], t32[3], t32[4], offs,
                                               grad_a=ga32, grad_r=gr)
    bwd32()
    sched32_b, _ = ctx.tune_batched_cqk(*t32, offs, r, repeats=2, backward=True, x=x32, g=g32)
    ms32_b = timed(bwd32, 5, sync)
    out["batched_cqk_8192rows_f32"] = {
        "rows": 8192, "elements": total, "ms": ms32, "elements_per_s": total / (ms32 * 1e-3),
        "mean_iterations": info32["passes"] / 8192, "max_iterations": info32["iterations"],
        "gbs_20B_per_elem_per_iteration":
            20.0 * total * info32["passes"] / 8192 / (ms32 * 1e-3) / 1e9,
        "status": info32["status_name"], "schedule": sched32, "backward_ms": ms32_b,
        "backward_schedule": sched32_b,
        "backward_gbs_24B_per_elem": 24.0 * total / (ms32_b * 1e-3) / 1e9}
    del t32, x32, g32, ga32
    ctx.set_batch_schedule(8, 4, 0, general=True)
    ctx.set_batch_schedule(8, 4, 0, backward=True, general=True)
    del t, x, g, ga, gr, offs, r
    torch.cuda.empty_cache()
    return out


def extra_spg(ctx, dev, torch):
    """SPG on the l1-constrained least-squares problem of Section 5.2 with a
    random 2048 x 65536 FP64 matrix (1 GiB), a 200-sparse x_true and the
    radius ||x_true||_1; projections warm-started from the iterate, and
    cold, to the paper's tolerance 1e-4."""
    from paper_2603_15910_amd import workloads as W
    A, b, x_true = W.lasso_instance(2048, 65536, 200, 1)
    radius = float(np.sum(np.abs(x_true)))
    At = torch.from_numpy(A).to(dev)
    bt = torch.from_numpy(b).to(dev)
    del A
    x = torch.empty(65536, dtype=torch.float64, device=dev)
    out = {}
    for name, warm in (("warm", True), ("cold", False)):
        ctx.spg_l1_lasso(At, bt, radius, out=x, warm=warm, max_iter=5, check=False)
        _, info = ctx.spg_l1_lasso(At, bt, radius, out=x, warm=warm)
        it = max(1, info["iterations"])
        out[f"spg_l1_lasso_2048x65536_f64_{name}"] = {
            "ms": info["total_ms"], "iterations": info["iterations"],
            "ms_per_iteration": info["total_ms"] / it,
            "projection_ms": info["proj_ms"], "projections": info["projections"],
            "newton_iterations_per_projection": info["newton_iterations"] / max(1, info["projections"]),
            "objective": info["objective"], "pg": info["pg"], "status": info["status_name"],
            "matrix_gbs": 2 * 2048 * 65536 * 8 * it / ((info["total_ms"] - info["proj_ms"]) * 1e-3) / 1e9}
    del At, bt, x
    torch.cuda.empty_cache()
    return out


def extra_differentiable(ctx, dev, torch):
    import paper_2603_15910_amd as cqk
    from paper_2603_15910_amd import workloads as W
    sync = torch.cuda.synchronize
    ex = {}
    # differentiable batched projection: 4096 rows in [1024, 32768], y = 3 N(0,1)
    off, yb = W.batched_simplex_input(4096, 1024, 32768, 1, scale=3.0)
    total = int(off[-1])
    offs = torch.from_numpy(off).to(dev)
    yt = torch.from_numpy(yb).to(dev)
    g = torch.from_numpy(W.upstream_grad(total, 1)).to(dev)
    xf = torch.empty_like(yt)
    gy = torch.empty_like(yt)
    ctx.project_simplex_batched(yt, offs, 1.0, out=xf)
    fsched, _ = ctx.tune_batched(yt, offs, 1.0, repeats=3, out=xf)
    ctx.project_simplex_batched(yt, offs, 1.0, out=xf)
    bsched, _ = ctx.tune_batched_backward(xf, g, offs, repeats=3, grad_y=gy)
    fwd = timed(lambda: ctx.project_simplex_batched(yt, offs, 1.0, out=xf), 10, sync)
    bwd = timed(lambda: ctx.project_simplex_batched_backward(xf, g, offs, grad_y=gy), 10, sync)

    def fb():
        yy = yt.detach().requires_grad_(True)
        xx = cqk.SimplexProjection.apply(yy, offs, 1.0)
        xx.backward(g)

    fb()
    fwdbwd = timed(fb, 10, sync)
    ex["differentiable_batched_4096rows"] = {
        "rows": 4096, "elements": total, "forward_ms": fwd, "backward_ms": bwd,
        "forward_backward_autograd_ms": fwdbwd,
        "forward_gbs_8B": 8.0 * total / (fwd * 1e-3) / 1e9,
        "backward_gbs_12B": 12.0 * total / (bwd * 1e-3) / 1e9,
        "forward_schedule": fsched, "backward_schedule": bsched}
    return ex


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=10_000_000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--only", choices=EXTRA_SECTIONS, default=None,
                    help="run one extra workload alone (for profiling) and print its record")
    ap.add_argument("--theta", type=float, default=0.0,
                    help="use this compaction threshold instead of tuning it (profiling runs)")
    ap.add_argument("--no-row-loop", action="store_true",
                    help="skip the per-row loop comparator of the batched workload")
    ap.add_argument("--oracle-full", action="store_true",
                    help="also time the oracle on the whole n = 1e8 workload (best of 3, minutes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2603_15910_amd as cqk
    from paper_2603_15910_amd import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.only:
        ctx = cqk.Context(0)
        ex = extras(ctx, dev, torch, sections=(args.only,), row_loop=not args.no_row_loop)
        print(json.dumps({"only": args.only, "extras": ex}))
        return
    n = args.n
    log(f"bench: generating cqk_uniform n={n}")
    inst = W.cqk_uniform(n, 1)
    t = [torch.from_numpy(inst[k]).to(dev) for k in "dablu"]
    r = inst["r"]
    del inst
    x = torch.empty_like(t[0])
    ctx = cqk.Context(0)
    ctx.reserve(n)

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # the compaction threshold theta, tuned on this instance (every candidate
    # solved, the fastest kept in the context for the timed solves)
    if args.theta > 0.0:
        ctx.compact_theta = args.theta
        theta, theta_ms, theta_sweep = args.theta, None, {}
    else:
        log("bench: tuning theta")
        theta, theta_ms, theta_sweep = ctx.tune_theta(*t, r, repeats=3, out=x)
        log(f"bench: theta {theta} ({theta_ms:.3f} ms); sweep {theta_sweep}")
    log(f"bench: warmup {args.warmup}")
    for _ in range(args.warmup):
        ctx.solve(*t, r, out=x)
    torch.cuda.synchronize()

    log(f"bench: timing {args.steps} steps")
    infos, per_pass = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        # HIP events stamped by the dispatches of the first Newton pass and
        # of the x-writing pass (timing 2: the other kernels run without the
        # gaps the runtime leaves around a timed dispatch)
        _, info = ctx.solve(*t, r, out=x, timing=2)
        infos.append(info)
        per_pass.append(ctx.pass_ms())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt * 1e3 / args.steps
    assert all(i["status"] == 0 for i in infos), infos[-1]

    fin_ms = statistics.mean(i["finalize_ms"] for i in infos)
    fin_bytes = infos[-1]["finalize_bytes"]
    fin_gbs = fin_bytes / (fin_ms * 1e-3) / 1e9
    # after the timed region: every pass kernel timed, over a few solves
    all_infos = []
    for _ in range(3):
        _, info = ctx.solve(*t, r, out=x, timing=True)
        all_infos.append(info)
    pass_bytes = sum(i["pass_bytes"] for i in all_infos)
    pass_ms = sum(i["pass_ms"] for i in all_infos)
    passes = sum(i["pass_launches"] for i in all_infos)
    achieved = pass_bytes / (pass_ms * 1e-3) / 1e9 if pass_ms > 0 else 0.0
    # and the per-pass log with each pass's kernel time
    ctx.solve(*t, r, out=x, trace=True, timing=True)
    tr = ctx.trace()
    passes_tab, tail_us = pass_table(ctx)
    # the first Newton pass (over the caller's arrays, compacting for the
    # sampled bracket): its algorithmic bytes from the traced solve (the same
    # in every solve of this instance), its time in each timed solve
    first_bytes = next(p for p in passes_tab if p["kind"] == "evaluate")["bytes"]
    first_ms = statistics.mean(p[0] for p in per_pass)
    first_gbs = first_bytes / (first_ms * 1e-3) / 1e9
    # context beside the headline (not the metric): the eq. (CQKlambda0) start
    # on the same instance, and the device-copy ceiling of this part
    ctx.solve(*t, r, out=x, lambda0="formula")
    ms_formula = timed(lambda: ctx.solve(*t, r, out=x, lambda0="formula"), 5,
                       torch.cuda.synchronize)
    _, info_formula = ctx.solve(*t, r, out=x, lambda0="formula")
    copy_gbs = copy_ceiling(torch)
    log(f"bench: {ms:.3f} ms/solve, iterations={infos[-1]['iterations']}, "
        f"pass GB/s={achieved:.0f}, finalize GB/s={fin_gbs:.0f}")
    for rec in tr:
        log(f"  pass kind={rec['kind']} src={rec['source']} n_in={rec['n_in']} "
            f"n_out={rec['n_out']} lam={rec['lam']:.12g}")
    with open(KERNEL_SRC, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()

    out = {
        "metric": "CQK solve elements/sec (general CQK, FP64, n=1e8)",
        "value": n / (ms * 1e-3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"cqk_uniform n={n} fp64 (d~U[1,10], a~U[-10,10], b~U[1,10], "
                               "l~U[-5,0], u=l+U[0.1,5], r=b'(l+u)/2), lambda0=0, compaction=auto",
                   "n": n, "seed": 1},
        "roofline": {
            "bound": "hbm",
            "kernel": "gen_spec_pass_kernel<double> (the first Newton pass)",
            "achieved": first_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": first_gbs / HBM_PEAK_GBS,
            "traffic": measured_traffic(sha, "gen_spec_pass_kernel"),
            "launches": len(per_pass),
            "avg_launch_ms": first_ms,
            "avg_launch_bytes": first_bytes,
        },
        # the x-writing pass, about as long: 40 B read + 8 B written per index
        "roofline_finalize": {
            "bound": "hbm",
            "kernel": "gen_finalize_kernel<double>",
            "achieved": fin_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": fin_gbs / HBM_PEAK_GBS,
            "traffic": measured_traffic(sha, "gen_finalize_kernel"),
            "launches": len(infos),
            "avg_launch_ms": fin_ms,
            "avg_launch_bytes": fin_bytes,
        },
        # every pass kernel launch of three solves after the timed region,
        # each kernel timed (the sample kernels, the Newton passes, those
        # queued after the loop stopped)
        "passes_all": {"achieved": achieved, "frac": achieved / HBM_PEAK_GBS,
                       "launches": passes, "avg_launch_ms": pass_ms / max(passes, 1),
                       "avg_launch_bytes": pass_bytes / max(passes, 1)},
        "iterations": infos[-1]["iterations"],
        "theta": {"chosen": theta, "tuned": args.theta <= 0.0, "tuned_ms": theta_ms,
                  "sweep_ms": {str(k): v for k, v in theta_sweep.items()}},
        "passes": passes_tab,
        "passes_after_stop_us": tail_us,
        "finalize_gbs": fin_gbs,
        "formula_start": {"ms": ms_formula, "iterations": info_formula["iterations"],
                          "elements_per_s": n / (ms_formula * 1e-3)},
    }
    out["roofline"]["copy_ceiling_gbs"] = copy_gbs
    del t, x
    torch.cuda.empty_cache()
    if not args.no_extras:
        log("bench: C2 seeds 1-3 (uniform, correlated)")
        out["c2_seeds"] = {"cqk_uniform": c2_seeds(ctx, dev, torch, "cqk_uniform"),
                           "cqk_correlated": c2_seeds(ctx, dev, torch, "cqk_correlated")}
        log("bench: C1 (n = 1e5, seeds 1-20)")
        out["c1"] = c1_latency(ctx, dev, torch)
    if not args.no_extras:
        log("bench: extras")
        out["extras"] = extras(ctx, dev, torch)
    if not args.no_cpu_baseline:
        log(f"bench: cpu baseline (oracle) on n={args.cpu_sample}")
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample, full=args.oracle_full)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
