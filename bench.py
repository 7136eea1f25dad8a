"""Benchmark of the batched rigid-body step on one MI355X.

Workload (default): 4096 tray envs (a static tray holding 20 random boxes / spheres / capsules,
24 bodies per env, dt = 0.005 s, 8 TGS substeps), synthetic and seeded.  A step is one call of
ms_step advancing all envs by one dt (load, broadphase, narrowphase, rows, colouring, solve,
integration, store).  W untimed warm-up steps, then exactly K timed steps bracketed by device
synchronisation; per-step HIP events on the launch stream give p50 / p99 latency.

Prints one JSON line (metric, value, ...), plus the roofline of the step kernel and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="tray")
    ap.add_argument("--envs", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--steps-per-launch", type=int, default=1)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--extra", action="store_true", help="also time the other workloads")
    return ap.parse_args()


def time_batch(batch, steps, warmup, spl, targets=None):
    import numpy as np
    import torch
    for _ in range(max(1, warmup // spl)):
        batch.step(spl, targets)
    torch.cuda.synchronize()
    n_launch = max(1, steps // spl)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_launch + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(n_launch):
        batch.step(spl, targets)
        ev[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(n_launch)]) / spl  # ms per step
    total_ms = ev[0].elapsed_time(ev[-1])
    return dict(total_ms=total_ms, wall_s=wall, n_steps=n_launch * spl, p50_ms=float(np.percentile(per, 50)),
                p99_ms=float(np.percentile(per, 99)), mean_ms=float(per.mean()))


def cpu_baseline(name, seed, budget_s=15.0):
    """The oracle (float32) on all host threads over a bounded sample of the same workload."""
    import numpy as np
    from oracle.oracle import Oracle
    from paper_2410_00425_amd import scenes as S
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(threads, 64))
    n_env = 256
    sc = S.by_name(name, n_env, seed=seed)
    o = Oracle(sc, 32)
    o.step(5, n_threads=threads)  # warm
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        o.step(5, n_threads=threads)
        steps += 5
    dt = time.perf_counter() - t0
    return dict(value=n_env * steps / dt, unit="env-steps/s", cores=threads, kind="oracle",
                sample=f"{n_env} {name} envs x {steps} steps (float32 oracle, {threads} threads, {dt:.1f} s)")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU: the step has no cross-GPU work; "
                                   "--gpus above 1 is not supported"}))
        sys.exit(2)
    import torch
    from paper_2410_00425_amd import ms, scenes as S
    torch.cuda.init()
    sc = S.by_name(args.workload, args.envs, seed=args.seed)
    b = ms.Batch(sc, lanes_per_env=args.lanes)
    r = time_batch(b, args.steps, args.warmup, args.steps_per_launch)
    value = sc.n_envs * r["n_steps"] / (r["total_ms"] / 1e3)
    out = {
        "metric": "env-steps/sec at 4096 envs (plain vs batched/served); p50/p99 step latency",
        "value": value, "unit": "env-steps/s", "n_gpus": 1, "steps": r["n_steps"], "warmup": args.warmup,
        "ms_per_step": r["total_ms"] / r["n_steps"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {sc.n_envs} envs, {sc.n_bodies // sc.n_envs} bodies/env",
                   "steps_per_launch": args.steps_per_launch, "plan": {k: v for k, v in b.plan().items()
                                                                        if k != "lanes"}},
        "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"],
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.workload, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
