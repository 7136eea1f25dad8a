"""Benchmark of the batched rigid-body step on one MI355X.

Headline workload: 4096 tray envs (a static tray holding 20 random boxes / spheres / capsules
dropped from random poses; 24 bodies per env; dt = 0.005 s, 8 TGS substeps), synthetic and
seeded.  A step is one ms_step call advancing all 4096 envs by one dt: load from HBM, bounding
boxes, candidate pairs, narrowphase, contact rows, colouring, 8 substeps of the coloured
Gauss-Seidel solve with integration, store.  W untimed warm-up steps, then exactly K timed steps
bracketed by device synchronisation; HIP events on the launch stream time every launch (p50 /
p99) and the whole region.  Before the warm-up every workload first runs --settle untimed steps
(default 200 = 1 s of simulated time for the tray) from the generator state, so the timed window
is the contact-rich, settled phase of the scene whatever --steps / --warmup are; the line names
the window.

The line also carries:
  * roofline: the step kernel against the chip's FP32 vector peak; achieved = algorithmic FLOP
    per launch / measured launch time, the FLOP per launch from live per-env work counters
    (candidate pairs per shape kind, contact points, manifolds, joints, bodies) times per-unit
    FLOP counts taken from the kernel source (listed in FLOP_PER_UNIT);
  * cpu_baseline: the float32 CPU oracle on all host threads over a bounded sample;
  * extra: the other workloads (one box per env at 4096, the 7-link arm at 1024, the
    heterogeneous batch against its padded form) and the serving run (8 clients, continuous
    batching under an HBM budget: saturation throughput, p50 / p99 request latency under Poisson
    arrivals, and the same requests run without the server) unless --quick.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12     # MI355X FP32 vector FLOP/s (256 CUs x 2.4 GHz x 256 FLOP/clk with dual issue)
PEAK_HBM = 8.0e12        # bytes/s

# FLOP per unit (add, sub, mul, div, sqrt; compares excluded), counted in ms_step.hip.
FLOP_PER_UNIT = {
    "body_step": 81 + 54,       # per body per step: step-start pose + world inverse inertia + AABB
    "static_body_step": 54,     # AABB only
    "body_substep": 108,        # gravity, damping, integration of the offsets (dynamic bodies)
    # narrowphase per candidate, by kind: 0 sphere-sphere, 1 sphere-capsule, 2 sphere-box,
    # 4 capsule-capsule, 5 capsule-box, 8 box-box, 9 plane-sphere, 10 plane-capsule, 11 plane-box
    "narrow": {0: 95, 1: 130, 2: 130, 4: 185, 5: 340, 8: 1350, 9: 45, 10: 72, 11: 222},
    "point_prep": 104,          # normal row setup per contact point
    "manifold_prep": 220,       # friction patch setup per manifold
    "point_solve": 160,         # normal row per point per substep (separation, bias, impulse)
    "manifold_solve": 250,      # two tangent rows + twist per manifold per substep
    "point_warm": 63,           # warm start per point per substep after the first
    "manifold_warm": 115,
    "joint_solve": 1010,        # point block + angular block + drive per joint solve
    "joint_warm": 300,
}


def kernel_source_hash():
    """Hash of what determines the step kernel's code: its sources and the build flags."""
    h = hashlib.sha256()
    for f in ("csrc/ms_step.hip", "csrc/ms_dev.h", "build.py"):
        h.update(open(os.path.join(ROOT, "paper_2410_00425_amd", f), "rb").read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--settle", type=int, default=200,
                    help="untimed steps from the generator state before the warm-up (contact-rich window)")
    ap.add_argument("--workload", default="tray")
    ap.add_argument("--envs", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--steps-per-launch", type=int, default=1)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--serve-full", action="store_true",
                    help="serving sweep: arrival rates 0.1 .. 1.25 x saturation, budgets 48 MB / 128 MB / 256 MB / 1 GB")
    ap.add_argument("--phase-clock", action="store_true",
                    help="run the per-phase clock build (libms_clock.so) and report the step's phase split "
                         "(the headline then carries the clock reads' overhead)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for HBM counter scaling)")
    return ap.parse_args()




def settle(batch, steps, spl=10, targets=None):
    """Untimed steps from the generator state into the settled, contact-rich phase."""
    done = 0
    while done < steps:
        k = min(spl, steps - done)
        batch.step(k, targets)
        done += k


def time_batch(batch, steps, warmup, spl, targets=None):
    import numpy as np
    import torch
    torch.cuda.synchronize()
    for _ in range(max(1, warmup // spl)):
        batch.step(spl, targets)
    torch.cuda.synchronize()
    batch.stats(reset=True)
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
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(n_launch)])
    total_ms = ev[0].elapsed_time(ev[-1])
    st = batch.stats()
    return dict(total_ms=total_ms, wall_s=wall, n_steps=n_launch * spl, n_launch=n_launch,
                n_warm=max(1, warmup // spl) * spl,
                launch_ms=total_ms / n_launch, p50_ms=float(np.percentile(per, 50)) / spl,
                p99_ms=float(np.percentile(per, 99)) / spl, stats=st)


def algorithmic_flop(scene, stats, params):
    """FLOP of the step model for the counted work (all envs, all counted steps)."""
    import numpy as np
    S = int(params["pos_iters"]) if int(params["solver"]) == 0 else 1
    JI = max(1, int(params["joint_iters"]))
    steps = stats[:, 0].astype(np.float64)
    nb = np.diff(scene.body_off).astype(np.float64)
    nj = np.diff(scene.joint_off).astype(np.float64)
    static = np.add.reduceat((scene.bodies["flags"] & 1).astype(np.float64), scene.body_off[:-1])
    dyn = nb - static
    F = FLOP_PER_UNIT
    f = steps * (dyn * (F["body_step"] + S * F["body_substep"]) + static * F["static_body_step"])
    for k, c in F["narrow"].items():
        f = f + stats[:, 1 + k] * c
    pts, man = stats[:, 13].astype(np.float64), stats[:, 14].astype(np.float64)
    f = f + pts * F["point_prep"] + man * F["manifold_prep"]
    f = f + S * (pts * F["point_solve"] + man * F["manifold_solve"]) + (S - 1) * (pts * F["point_warm"] +
                                                                                 man * F["manifold_warm"])
    f = f + steps * nj * (S * JI * F["joint_solve"] + (S - 1) * F["joint_warm"])
    return float(f.sum())


def algorithmic_bytes(scene):
    """HBM bytes per launch: state read + written (52 B per body each way), body parameters
    (48 B), offsets (8 B per env), joints (72 B + 4 B target), status (4 B read + 4 written)."""
    return scene.n_bodies * (52 * 2 + 48) + scene.n_envs * (8 + 8) + scene.n_joints * 76


def time_graph(batch, steps, warmup, per_graph=10, spl=1):
    """Steps replayed from a captured graph of per_graph steps in launches of spl steps each."""
    import numpy as np
    import torch
    for _ in range(max(1, warmup)):
        batch.step(1)
    n_warm = max(1, warmup)
    per_graph = max(1, per_graph // spl) * spl   # whole launches per replay
    g = batch.graph(spl, per_graph // spl)
    g.launch()
    torch.cuda.synchronize()
    batch.stats(reset=True)
    n_rep = max(1, steps // per_graph)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_rep + 1)]
    ev[0].record()
    for i in range(n_rep):
        g.launch()
        ev[i + 1].record()
    torch.cuda.synchronize()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(n_rep)]) / per_graph
    total_ms = ev[0].elapsed_time(ev[-1])
    g.close()
    st = batch.stats()
    n_steps = n_rep * per_graph
    return dict(total_ms=total_ms, n_steps=n_steps, n_launch=n_steps // spl, launch_ms=total_ms / (n_steps // spl),
                n_warm=n_warm + per_graph,
                p50_ms=float(np.percentile(per, 50)), p99_ms=float(np.percentile(per, 99)), stats=st)


def run_workload(ms, S, name, n_envs, steps, warmup, spl, seed, lanes=0, pack=1, tune=False, graph=False, settle_steps=200,
                 warm_start=False, forces=False, targets=None):
    """Settle, (tune,) warm up, then time; returns the scene, the raw timing and the summary.
    warm_start: the cross-step contact cache on; forces: the contact-force readout on; targets:
    drive targets (numpy, [J]) set for every step."""
    import torch
    sc = S.by_name(name, n_envs, seed=seed)
    if warm_start:
        sc.params["warm_start"] = 1
    b = ms.Batch(sc, lanes_per_env=lanes, pack=pack)
    if forces:
        b.set_contact_forces(True)
    tg = None if targets is None else torch.from_numpy(targets).cuda()
    if tg is not None:
        b.step(1, tg)
    settle(b, settle_steps)
    if tune:
        # tune on the settled state (trials of 10 steps), then time from that same state
        saved = b.get_state()
        b.tune(10)
        b.reset_envs(torch.arange(n_envs, dtype=torch.int32, device="cuda"), saved)
    r = time_graph(b, steps, warmup, spl=spl) if graph else time_batch(b, steps, warmup, spl)
    flop = algorithmic_flop(sc, r["stats"], sc.params)
    plan = b.plan()
    b.close()
    launches = r["n_launch"]
    first = settle_steps + r["n_warm"] + 1
    return sc, r, dict(workload=name, envs=n_envs, bodies=sc.n_bodies, joints=sc.n_joints,
                       env_steps_per_s=n_envs * r["n_steps"] / (r["total_ms"] / 1e3), ms_per_step=r["total_ms"] / r["n_steps"],
                       p50_ms=r["p50_ms"], p99_ms=r["p99_ms"], flop_per_launch=flop / launches,
                       tflops=flop / (r["total_ms"] / 1e3) / 1e12, tiles=plan["n_tiles"], lds_bytes=plan["lds_bytes"],
                       timed_steps=f"{first}..{first + r['n_steps'] - 1}")


def cpu_baseline(name, seed, settle_steps=200, budget_s=15.0):
    """The float32 oracle on all host threads over a bounded sample of the same workload, timed
    in the same settled window as the GPU run (settle_steps untimed steps first)."""
    from oracle.oracle import Oracle
    from paper_2410_00425_amd import scenes as S
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(threads, 64))
    n_env = 256
    sc = S.by_name(name, n_env, seed=seed)
    o = Oracle(sc, 32)
    o.step(settle_steps, n_threads=threads)
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        o.step(5, n_threads=threads)
        steps += 5
    dt = time.perf_counter() - t0
    return dict(value=n_env * steps / dt, unit="env-steps/s", cores=threads, kind="oracle",
                sample=f"{n_env} {name} envs x {steps} steps ({settle_steps + 1}..{settle_steps + steps}) after "
                       f"{settle_steps} untimed settling steps (float32 oracle, {threads} threads, {dt:.1f} s)")


def cpu_variants(name, seed, settle_steps=200, budget_s=4.0):
    """The oracle at both precisions on one thread and on all host threads (short samples of the
    same workload), and the host CPU's model name."""
    from oracle.oracle import Oracle
    from paper_2410_00425_amd import scenes as S
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(threads, 64))
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    out = {"cpu_model": model, "runs": []}
    for prec in (32, 64):
        for th in (1, threads):
            n_env = 256 if th > 1 else 32
            sc = S.by_name(name, n_env, seed=seed)
            o = Oracle(sc, prec)
            o.step(settle_steps, n_threads=th)
            steps, t0 = 0, time.perf_counter()
            while time.perf_counter() - t0 < budget_s:
                o.step(2, n_threads=th)
                steps += 2
            dt = time.perf_counter() - t0
            o.close()
            out["runs"].append({"precision": f"f{prec}", "threads": th, "env_steps_per_s": n_env * steps / dt,
                                "sample": f"{n_env} {name} envs x {steps} steps after {settle_steps} settling steps, "
                                          f"{dt:.1f} s"})
    return out


def measured_peaks(ms):
    """Rates this device reaches for the step's kinds of work: FP32 multiply-then-add issue on
    independent chains (ms_peak_fp32, 8 wavefronts per SIMD) and a 512 MiB device copy."""
    import torch
    n_waves, iters = 8192, 4096
    buf = torch.empty(n_waves * 64, dtype=torch.float32, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ms.peak_fp32(buf, n_waves, iters)
    torch.cuda.synchronize()
    ev[0].record()
    flop = sum(ms.peak_fp32(buf, n_waves, iters) for _ in range(5))
    ev[1].record()
    torch.cuda.synchronize()
    tflops = flop / (ev[0].elapsed_time(ev[1]) / 1e3) / 1e12
    n = 128 << 20
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(5):
        y.copy_(x)
    ev[1].record()
    torch.cuda.synchronize()
    gbps = 5 * 2 * 4 * n / (ev[0].elapsed_time(ev[1]) / 1e3) / 1e9
    return {"fp32_mul_add_tflops": tflops, "hbm_copy_GBps": gbps,
            "how": "ms_peak_fp32: 8192 wavefronts x 4096 rounds x 8 chains of one multiply and one add; "
                   "copy: 512 MiB read + 512 MiB written per copy, 5 copies"}


def serving(ms, full=False, seed=0):
    """Continuous batching of step requests from 8 clients (2-step requests on sessions of one of
    the three scene families with 2**U{6..12} envs): saturation throughput (closed loop), latency
    under Poisson arrivals at a fraction of it, and the same requests run plainly (one batch per
    session, one synchronised ms_step per request, no server)."""
    from paper_2410_00425_amd import serve_load as L
    pool = L.ScenePool(seed)
    spc, rps = (63, 20) if full else (2, 20)   # full: 8 x 63 x 20 = 10,080 requests per arrival rate
    out = {}
    # 48 MB binds: the arena peaks at 72-86 MB when nothing limits it
    budgets = (48 << 20, 128 << 20, 256 << 20, 1 << 30) if full else (256 << 20,)
    for budget in budgets:
        srv = ms.Server(budget)
        recs, wall = L.run_clients(ms, srv, pool, float("inf"), n_clients=8, sessions_per_client=spc,
                                   reqs_per_session=rps, seed=seed)
        sat = L.summarize(recs, wall)
        st = srv.stats()
        res = {"saturation": sat, "server": st}
        fracs = (0.1, 0.25, 0.5, 0.75, 1.0, 1.25) if full else (0.75,)
        for f in fracs:
            recs, wall = L.run_clients(ms, srv, pool, f * sat["requests_per_s"], n_clients=8, sessions_per_client=spc,
                                       reqs_per_session=rps, seed=seed + 1)
            res[f"poisson_{f}"] = L.summarize(recs, wall)
        srv.close()
        out[f"budget_{budget >> 20}MB"] = res
    out["plain"] = L.run_plain(ms, pool, n_clients=8, sessions_per_client=spc, reqs_per_session=rps, seed=seed)
    key = f"budget_{256}MB"
    out["served_vs_plain"] = out[key]["saturation"]["env_steps_per_s"] / out["plain"]["env_steps_per_s"]
    return out


PHASES = ["load", "pose_aabb", "broadphase", "narrowphase_rows", "contact_cache", "colouring", "block_lists",
          "gravity_warm_start", "bias_joint_prep", "joint_wave_warm_start", "sweeps", "force_sums", "integration",
          "velocity_restitution", "guard_exports", "store"]


def phase_split(ms, S, name, n_envs, seed, settle_steps, steps=100):
    """Wave-cycles per phase of the step over `steps` one-step launches after settling (per-phase
    clock build only), as fractions of the total."""
    import torch
    sc = S.by_name(name, n_envs, seed=seed)
    b = ms.Batch(sc)
    settle(b, settle_steps)
    torch.cuda.synchronize()
    b.phase_clocks(reset=True)
    for _ in range(steps):
        b.step(1)
    torch.cuda.synchronize()
    cyc = b.phase_clocks()
    b.close()
    tot = float(cyc.sum())
    return {"steps": steps, "window": f"{settle_steps + 1}..{settle_steps + steps}",
            "fractions": {p: float(c) / tot for p, c in zip(PHASES, cyc) if c > 0},
            "wave_cycles_per_env_step": tot / (steps * n_envs)}


def traffic_from_profile(name):
    """HBM bytes per launch from the committed counter summary, if it matches this kernel."""
    p = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(p):
        return None
    rec = json.load(open(p))
    if rec.get("kernel_source") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU (the batched step has no cross-GPU work); "
                                   f"--gpus {args.gpus} is not supported"}), flush=True)
        sys.exit(2)
    import torch
    if args.phase_clock:
        from paper_2410_00425_amd import build as B
        os.environ["MS_LIBRARY"] = B.CLOCK_LIB
        if not os.path.exists(B.CLOCK_LIB):
            print(json.dumps({"error": f"{B.CLOCK_LIB} is missing: build it with "
                                       "`python -m paper_2410_00425_amd.build clock`"}), flush=True)
            sys.exit(2)
    from paper_2410_00425_amd import ms, scenes as S
    torch.cuda.init()
    sc, r, head = run_workload(ms, S, args.workload, args.envs, args.steps, args.warmup, args.steps_per_launch,
                               args.seed, args.lanes, settle_steps=args.settle)
    value = head["env_steps_per_s"]
    achieved = head["flop_per_launch"] / (r["launch_ms"] / 1e3)
    out = {
        "metric": "env-steps/sec at 4096 envs (plain vs batched/served); p50/p99 step latency",
        "value": value, "unit": "env-steps/s", "n_gpus": 1, "steps": r["n_steps"], "warmup": args.warmup,
        "ms_per_step": r["total_ms"] / r["n_steps"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload} x {sc.n_envs} envs ({sc.n_bodies // sc.n_envs} bodies/env), "
                               f"dt {float(sc.params['dt'])}, {int(sc.params['pos_iters'])} TGS substeps, "
                               f"{args.steps_per_launch} step(s) per launch; timed steps {head['timed_steps']} "
                               f"after {args.settle} untimed settling steps and {r['n_warm']} warm-up steps",
                   "envs": sc.n_envs, "bodies": sc.n_bodies, "tiles": head["tiles"], "lds_bytes": head["lds_bytes"]},
        "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"],
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": traffic_from_profile(args.workload),
                     "flop_per_launch": head["flop_per_launch"], "launch_ms": r["launch_ms"],
                     "algorithmic_bytes_per_launch": algorithmic_bytes(sc),
                     "hbm_frac": algorithmic_bytes(sc) / (r["launch_ms"] / 1e3) / PEAK_HBM,
                     "kernel_source": kernel_source_hash()},
    }
    if args.phase_clock:
        out["phase_split"] = phase_split(ms, S, args.workload, args.envs, args.seed, args.settle)
    if args.copy_calibration:
        n = 64 << 20
        x = torch.empty(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": 4 * n, "write": 4 * n}
    if not args.quick:
        extra = {}
        # the padded baseline is the plain launch: one tile per env, one LDS size for all (pack=0)
        for name, n, pack in (("drop_boxes", 4096, 1), ("arm_cube", 1024, 1), ("hetero", 4096, 1),
                              ("hetero_padded", 4096, 0)):
            _, _, res = run_workload(ms, S, name, n, 100, 20, 1, args.seed, pack=pack, settle_steps=args.settle)
            extra[name] = res
        # the batched form with the autotuned tiling, its steps replayed from a captured graph
        _, _, res = run_workload(ms, S, "hetero", 4096, 100, 20, 1, args.seed, tune=True, graph=True,
                                 settle_steps=args.settle)
        extra["hetero_tuned_graph"] = res
        extra["hetero_speedup_vs_padded"] = extra["hetero"]["env_steps_per_s"] / extra["hetero_padded"]["env_steps_per_s"]
        extra["hetero_tuned_graph_speedup_vs_padded"] = (extra["hetero_tuned_graph"]["env_steps_per_s"] /
                                                         extra["hetero_padded"]["env_steps_per_s"])
        # persistent launches of one 60 Hz control step (2 steps of the 120 Hz simulation) each,
        # replayed from a graph: the batched form and, like for like, the padded form
        _, _, res = run_workload(ms, S, "hetero", 4096, 100, 20, 2, args.seed, tune=True, graph=True,
                                 settle_steps=args.settle)
        extra["hetero_tuned_graph_2spl"] = res
        _, _, res = run_workload(ms, S, "hetero_padded", 4096, 100, 20, 2, args.seed, pack=0, graph=True,
                                 settle_steps=args.settle)
        extra["hetero_padded_graph_2spl"] = res
        extra["hetero_2spl_speedup_vs_padded_plain"] = (extra["hetero_tuned_graph_2spl"]["env_steps_per_s"] /
                                                                extra["hetero_padded"]["env_steps_per_s"])
        extra["hetero_2spl_speedup_vs_padded_2spl"] = (extra["hetero_tuned_graph_2spl"]["env_steps_per_s"] /
                                                       extra["hetero_padded_graph_2spl"]["env_steps_per_s"])
        # the paper's simulation-only workload: cart-poles at 120 Hz, 4 position / 0 velocity
        # iterations, one 60 Hz control step (2 simulation steps) per launch, cart targets set
        ids = list(range(4096))
        _, _, res = run_workload(ms, S, "cartpole", 4096, 200, 20, 2, args.seed, settle_steps=args.settle,
                                 targets=S.cartpole_targets(args.seed, ids, 0))
        extra["cartpole"] = res
        # compound bodies: the tray with about half of its 12 objects made of 2-3 primitive parts
        _, _, res = run_workload(ms, S, "compound_tray", 4096, 100, 20, 1, args.seed, tune=True,
                                 settle_steps=args.settle)
        extra["compound_tray"] = res
        # the headline workload with the cross-step contact cache, and with the contact-force readout
        _, _, res = run_workload(ms, S, args.workload, args.envs, 100, 20, 1, args.seed, settle_steps=args.settle,
                                 warm_start=True)
        extra[f"{args.workload}_warm_start"] = res
        _, _, res = run_workload(ms, S, args.workload, args.envs, 100, 20, 1, args.seed, settle_steps=args.settle,
                                 forces=True)
        extra[f"{args.workload}_contact_forces"] = res
        extra["serving"] = serving(ms, full=args.serve_full, seed=args.seed)
        pk = measured_peaks(ms)
        extra["measured_peaks"] = pk
        # the headline's FLOP rate against the rate its instruction kinds can reach on this device
        out["roofline"]["peak_measured_mul_add"] = pk["fp32_mul_add_tflops"]
        out["roofline"]["frac_measured"] = out["roofline"]["achieved"] / pk["fp32_mul_add_tflops"]
        out["extra"] = extra
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.workload, args.seed, settle_steps=args.settle)
        if not args.quick:
            out.setdefault("extra", {})["cpu_oracle_variants"] = cpu_variants(args.workload, args.seed,
                                                                              settle_steps=args.settle)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
