"""Benchmark: general CQK solve, n = 1e8, FP64, on one MI355X.

One step = one whole solve (cqk_solve_f64: Newton passes with compaction of
resolved indices, then the x-writing pass) over inputs already resident in
HBM.  Prints one JSON line (see the design doc for every field).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n N]
                    [--no-cpu-baseline] [--no-extras]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


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


def cpu_baseline(n_sample: int):
    """The oracle (exact breakpoint-sort solver), single-threaded, on a
    bounded sample of the same workload."""
    from oracle import cqk_oracle as O
    from paper_2603_15910_amd import workloads as W
    inst = W.cqk_uniform(n_sample, 1)
    t0 = time.perf_counter()
    res = O.solve_cqk(*[inst[k] for k in "dablu"], inst["r"])
    dt = time.perf_counter() - t0
    assert res.status == O.OK
    ncpu, model = host_cpu_desc()
    return {"value": n_sample / dt, "unit": "elements/s", "cores": 1, "kind": "oracle",
            "sample": f"cqk_uniform n={n_sample} seed=1, one exact solve (numpy, 1 thread), "
                      f"{dt:.2f} s on {model} ({ncpu} logical CPUs)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--variant", default="uniform", choices=["uniform", "correlated"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=10_000_000)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the method shards as described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2603_15910_amd as cqk
    from paper_2603_15910_amd import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.n
    log(f"bench: generating cqk_{args.variant} n={n}")
    gen = W.cqk_uniform if args.variant == "uniform" else W.cqk_correlated
    inst = gen(n, 1)
    t = [torch.from_numpy(inst[k]).to(dev) for k in "dablu"]
    r = inst["r"]
    del inst
    x = torch.empty_like(t[0])
    ctx = cqk.Context(0)
    ctx.reserve(n)

    log(f"bench: warmup {args.warmup}")
    for _ in range(args.warmup):
        ctx.solve(*t, r, out=x)
    torch.cuda.synchronize()

    log(f"bench: timing {args.steps} steps")
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, info = ctx.solve(*t, r, out=x, timing=True, trace=True)
        infos.append(info)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt * 1e3 / args.steps

    pass_bytes = sum(i["pass_bytes"] for i in infos)
    pass_ms = sum(i["pass_ms"] for i in infos)
    passes = sum(i["passes"] for i in infos)
    achieved = pass_bytes / (pass_ms * 1e-3) / 1e9 if pass_ms > 0 else 0.0
    fin_gbs = (sum(i["finalize_bytes"] for i in infos) /
               (sum(i["finalize_ms"] for i in infos) * 1e-3) / 1e9)
    tr = ctx.trace()
    log(f"bench: {ms:.3f} ms/solve, iterations={infos[-1]['iterations']}, "
        f"pass GB/s={achieved:.0f}, finalize GB/s={fin_gbs:.0f}")
    for rec in tr:
        log(f"  pass kind={rec['kind']} src={rec['source']} n_in={rec['n_in']} "
            f"n_out={rec['n_out']} lam={rec['lam']:.12g}")

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
        "config": {"workload": f"cqk_{args.variant} n={n} fp64, lambda0=0, compaction=auto",
                   "n": n, "seed": 1},
        "roofline": {
            "bound": "hbm",
            "kernel": "gen_iter_kernel<double> (evaluation pass)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "launches": passes,
            "avg_launch_ms": pass_ms / max(passes, 1),
            "avg_launch_bytes": pass_bytes / max(passes, 1),
        },
        "iterations": infos[-1]["iterations"],
        "finalize_gbs": fin_gbs,
    }
    if not args.no_cpu_baseline:
        log(f"bench: cpu baseline (oracle) on n={args.cpu_sample}")
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
