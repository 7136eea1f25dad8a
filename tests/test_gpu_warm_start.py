"""Cross-step warm start (the contact cache, S4b) on the GPU against the float32 oracle: the
cache written by one step and read by the next gives the same bits on both sides (states and
every contact point's final normal impulse), in one-step launches and in multi-step launches
(the cache then passes between steps inside one launch), with PGS, after partial resets (which
clear the listed envs' caches), and around the autotuner (which saves and restores the cache).
The physical effect: a box on an incline below the friction angle holds still."""
import math

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2410_00425_amd import scenes as S

from parity import compare_states

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def ms():
    from paper_2410_00425_amd import ms as m
    return m


def warm(sc, debug=False, **kw):
    p = sc.params.copy()
    p["warm_start"] = 1
    p["warm_radius"] = kw.pop("radius", 0.01)
    p["debug_export"] = 1 if debug else 0
    for k, v in kw.items():
        p[k] = v
    sc.params = p
    return sc


def same_bits(sc, g, w):
    bo = sc.body_off
    return np.array([all(np.array_equal(g[k][:, bo[e]:bo[e + 1]], w[k][:, bo[e]:bo[e + 1]].astype(np.float32))
                         for k in ("pos", "quat", "linvel", "angvel")) for e in range(sc.n_envs)])


@pytest.mark.parametrize("name,n,steps,spl", [("tray", 64, 40, 1), ("tray", 64, 40, 5), ("drop_boxes", 128, 60, 3),
                                              ("arm_cube", 32, 40, 2), ("hetero", 128, 30, 1), ("cartpole", 64, 40, 2)])
def test_warm_start_runs_match_oracle(name, n, steps, spl):
    print(f"warm: {name} x {n}, {steps} steps, {spl} per launch", flush=True)
    sc = warm(S.by_name(name, n, seed=61))
    b = ms().Batch(sc)
    o = Oracle(sc, 32)
    for _ in range(steps // spl):
        b.step(spl)
        o.step(spl)
    g, w = b.state_numpy(), o.state()
    same = same_bits(sc, g, w)
    _, mm = o.counters()
    bad, excused = compare_states(sc, g, w, mm)
    print(f"warm: {name}: {same.sum()}/{n} envs bit-identical", flush=True)
    assert not bad, bad
    assert same.sum() >= n - max(2, n // 16), same.sum()


def test_warm_start_impulses_match_oracle():
    """Contact points and their final normal impulses of a step that starts from the cache."""
    print("warm: impulses", flush=True)
    sc = warm(S.tray(32, seed=62), debug=True)
    o64 = Oracle(sc, 64)
    o64.step(80)
    st = {k: np.float32(v) for k, v in o64.state().items() if k != "status"}
    b = ms().Batch(sc)
    ids = torch.arange(32, dtype=torch.int32, device="cuda")
    b.reset_envs(ids, {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in st.items()})
    o = Oracle(sc, 32)
    o.set_state(*[st[k].astype(np.float64) for k in ("pos", "quat", "linvel", "angvel")])
    b.step(1)
    o.step(1)               # both caches now hold this step
    b.step(1)
    o.step(1, record=True)  # and this step starts from them
    g, w = b.state_numpy(), o.state()
    rec = o.record()
    assert np.any(rec["points"][:, 8] > 0)
    gc = b.contacts()
    ok = same_bits(sc, g, w)
    assert ok.sum() >= 31, ok.sum()
    g_env = np.repeat(gc["pairs"][:, 0], np.maximum(gc["pairs"][:, 3], 0))
    o_env = rec["point_ids"][:, 0]
    for e in np.nonzero(ok)[0]:
        ge, oe = gc["points"][g_env == e], rec["points"][o_env == e]
        assert len(ge) == len(oe)
        assert np.array_equal(ge[:, 7], oe[:, 7].astype(np.float32)), e


def test_warm_start_pgs_and_incline():
    print("warm: PGS and incline", flush=True)
    a = math.radians(20.0)
    g = (9.81 * math.sin(a), 0.0, -9.81 * math.cos(a))
    box = S.body(S.BOX, (0.05, 0.05, 0.05), (0.0, 0.0, 0.05), mass=1.0, mu=0.5)
    for solver in (S.TGS, S.PGS):
        sc = warm(S.replicate(S.single([box], dt=0.01, pos_iters=4, gravity=g, solver=solver), 4))
        b = ms().Batch(sc)
        o = Oracle(sc, 32)
        b.step(100)
        o.step(100)
        x0 = b.state_numpy()["pos"][0].copy()
        b.step(100)
        o.step(100)
        st = b.state_numpy()
        assert np.array_equal(st["pos"], o.state()["pos"].astype(np.float32))
        if solver == S.TGS:
            assert np.all(np.abs(st["pos"][0] - x0) < 1e-6)


def test_reset_clears_and_tuning_keeps_the_cache():
    print("warm: reset and tuning", flush=True)
    sc = warm(S.tray(48, seed=63))
    b = ms().Batch(sc)
    o = Oracle(sc, 32)
    b.step(30)
    o.step(30)
    # a partial reset clears those envs' caches on both sides
    ids = np.array([0, 5, 47], np.int32)
    b.reset_envs_random(torch.from_numpy(ids).cuda(), xy_half=0.02, yaw_half=0.3, seed=9)
    o.reset_random(ids, xy_half=0.02, yaw_half=0.3, seed=9)
    # tuning saves and restores state and cache: the steps after it are unchanged
    b.tune(3)
    b.step(10)
    o.step(10)
    g, w = b.state_numpy(), o.state()
    same = same_bits(sc, g, w)
    assert same.sum() >= 46, same.sum()
    _, mm = o.counters()
    bad, _ = compare_states(sc, g, w, mm)
    assert not bad
