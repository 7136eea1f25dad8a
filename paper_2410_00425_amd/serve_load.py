"""Load generator for the serving path: client threads driving an ms_server.

Workload (synthetic, seeded): every session is a batch of one of the three scene families (one
falling box per env, the 7-link arm with a cube, the tray of 20 bodies), chosen uniformly, with
2**U{6..12} envs; a session is opened, runs `reqs_per_session` requests of `steps` steps each
(2 steps: one 60 Hz control step of the 120 Hz simulation of the paper's benchmark setup) and
is closed.  Each client runs its sessions one after another; request arrivals of a client are a
Poisson process of rate lam / n_clients (lam = inf: closed loop, the next request as soon as
the previous completes).  A session's request cannot exist before its previous request
completed, so its arrival is max(Poisson arrival, previous completion); latency = completion
- arrival, which includes queueing and admission.
"""
from __future__ import annotations

import math
import threading

import numpy as np

from . import scenes as S

FAMILIES = ("drop_boxes", "arm_cube", "tray")


class ScenePool:
    """One scene per (family, n_envs), generated on first use (sessions of the same kind share
    the initial state; they are still independent batches)."""

    def __init__(self, seed=0):
        self.seed = seed
        self._cache = {}
        self._lock = threading.Lock()

    def get(self, family, n):
        key = (family, n)
        with self._lock:
            if key not in self._cache:
                self._cache[key] = S.by_name(family, n, seed=self.seed)
            return self._cache[key]

    def prepare(self, seed, n_clients, sessions_per_client):
        """Generate ahead of time the scenes the clients will open."""
        for ci in range(n_clients):
            for family, n in session_plan(seed, ci, sessions_per_client):
                self.get(family, n)


def session_plan(seed, client, n_sessions):
    """(family, n_envs) of each session of a client, from a counter-based stream."""
    u = S.uniforms(seed, np.array([client]), 0x5E55, 2 * n_sessions).reshape(-1)
    fam = [FAMILIES[min(2, int(3 * u[2 * i]))] for i in range(n_sessions)]
    n = [1 << (6 + min(6, int(7 * u[2 * i + 1]))) for i in range(n_sessions)]
    return list(zip(fam, n))


def run_clients(ms, server, pool, lam, n_clients=8, sessions_per_client=2, reqs_per_session=20, steps=2, seed=0):
    """Drive the server from n_clients threads; returns per-request records and the wall time."""
    clock = ms.server_clock
    pool.prepare(seed, n_clients, sessions_per_client)
    recs, errors = [], []
    lock = threading.Lock()
    t_begin = clock() + 0.05
    rate = lam / n_clients if lam and not math.isinf(lam) else None

    def client(ci):
        rng = np.random.default_rng([seed, ci])
        t_next = t_begin
        mine = []
        try:
            for family, n in session_plan(seed, ci, sessions_per_client):
                sc = pool.get(family, n)
                sid = None
                done_prev = None
                for r in range(reqs_per_session):
                    if rate is not None:
                        t_next += rng.exponential(1.0 / rate)
                    # closed loop: the first request of a client arrives at the common start time
                    arrival = t_next if rate is not None else (done_prev if done_prev is not None else t_begin)
                    if done_prev is not None:
                        arrival = max(arrival, done_prev)
                    wait = arrival - clock()
                    if wait > 0:
                        threading.Event().wait(wait)
                    if sid is None:
                        sid = server.open(sc)
                    rid = server.submit(sid, steps)
                    info = server.wait(rid)
                    done_prev = info["t_done"]
                    mine.append(dict(family=family, envs=n, arrival=arrival, submit=info["t_submit"],
                                     start=info["t_start"], done=info["t_done"], fused=info["fused"],
                                     env_steps=n * steps))
                    if rate is None:
                        t_next = done_prev
                server.close_session(sid)
        except Exception as e:  # reported by the caller
            errors.append(repr(e))
        with lock:
            recs.extend(mine)

    th = [threading.Thread(target=client, args=(ci,)) for ci in range(n_clients)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    server.drain()
    if errors:
        raise RuntimeError("client errors: " + "; ".join(errors[:3]))
    t_end = max(r["done"] for r in recs)
    return recs, t_end - t_begin


def summarize(recs, wall):
    lat = np.array([r["done"] - r["arrival"] for r in recs]) * 1e3
    svc = np.array([r["done"] - r["start"] for r in recs]) * 1e3
    es = sum(r["env_steps"] for r in recs)
    return dict(requests=len(recs), wall_s=wall, requests_per_s=len(recs) / wall, env_steps_per_s=es / wall,
                p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                mean_ms=float(lat.mean()), p50_service_ms=float(np.percentile(svc, 50)),
                mean_fused=float(np.mean([r["fused"] for r in recs])))


def run_plain(ms, pool, n_clients=8, sessions_per_client=2, reqs_per_session=20, steps=2, seed=0):
    """The same sessions and requests without a server: one batch per session, one ms_step per
    request, synchronised after each (no fusion, no overlap); returns env-steps/s and latencies."""
    import torch
    clock = ms.server_clock
    pool.prepare(seed, n_clients, sessions_per_client)
    lat, es = [], 0
    t0 = clock()
    for ci in range(n_clients):
        for family, n in session_plan(seed, ci, sessions_per_client):
            b = ms.Batch(pool.get(family, n))
            for _ in range(reqs_per_session):
                ta = clock()
                b.step(steps)
                torch.cuda.current_stream().synchronize()
                lat.append(clock() - ta)
                es += n * steps
            b.close()
    wall = clock() - t0
    lat = np.array(lat) * 1e3
    return dict(requests=len(lat), wall_s=wall, env_steps_per_s=es / wall, p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)))
