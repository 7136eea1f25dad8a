"""The serving runtime (ms_server_*) on the GPU: continuous batching must not change a bit of
any session's result (a session served in a mix of other sessions equals the same batch
stepped alone with ms_step), admission must respect the HBM arena, and errors come back as
statuses."""
import threading

import numpy as np
import pytest

from paper_2410_00425_amd import scenes as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def ms():
    from paper_2410_00425_amd import ms as m
    return m


def alone(sc, n_req, steps, targets=None):
    b = ms().Batch(sc)
    for r in range(n_req):
        t = None if targets is None else torch.from_numpy(targets[r]).cuda()
        b.step(steps, t)
    st = b.state_numpy()
    b.close()
    return st


def test_served_mix_equals_alone():
    m = ms()
    scenes = [S.tray(96, seed=21), S.drop_boxes(200, seed=22), S.arm_cube(40, seed=23), S.hetero(64, seed=24),
              S.tray(8, seed=25)]
    n_req = [5, 7, 4, 6, 3]
    steps = [2, 1, 2, 3, 2]
    arm_t = [S.arm_targets(23, np.arange(40), r).reshape(-1).astype(np.float32) for r in range(4)]
    srv = m.Server(256 << 20)
    sids = [srv.open(sc) for sc in scenes]
    fused = []

    def drive(i):
        for r in range(n_req[i]):
            t = arm_t[r] if i == 2 else None
            info = srv.wait(srv.submit(sids[i], steps[i], t))
            fused.append(info["fused"])

    th = [threading.Thread(target=drive, args=(i,)) for i in range(len(scenes))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    got = [srv.get_state(s) for s in sids]
    st = srv.stats()
    for s in sids:
        srv.close_session(s)
    srv.drain()
    srv.close()
    assert st["requests_done"] == sum(n_req)
    assert st["env_steps"] == sum(sc.n_envs * n * k for sc, n, k in zip(scenes, n_req, steps))
    assert max(fused) > 1, "no request was fused with another session's"
    for i, sc in enumerate(scenes):
        ref = alone(sc, n_req[i], steps[i], arm_t if i == 2 else None)
        for k in ("pos", "quat", "linvel", "angvel", "status"):
            assert np.array_equal(got[i][k], ref[k]), (i, k)


def test_admission_waits_for_budget():
    m = ms()
    big = S.tray(512, seed=26)
    need = m.ms_query_batch_bytes(big)
    # room for one such session (plus the scratch reserve), not two
    srv = m.Server(int(need * 1.6) + (1 << 20), scratch_bytes=1 << 20)
    a = srv.open(big)
    b = srv.open(big)
    ra = srv.submit(a, 2)
    rb = srv.submit(b, 2)
    ia = srv.wait(ra)
    srv.close_session(a)
    ib = srv.wait(rb)
    assert ib["t_start"] >= ia["t_done"], "second session ran before the first released its block"
    srv.close_session(b)
    srv.drain()
    st = srv.stats()
    assert st["sessions_admitted"] == 2
    assert st["peak_arena_bytes"] < 2 * need
    srv.close()


def test_budget_rejection_and_errors():
    m = ms()
    srv = m.Server(4 << 20, scratch_bytes=1 << 20)
    with pytest.raises(m.MsError) as e:
        srv.open(S.tray(2048, seed=0))   # about 10 MB of workspace
    assert e.value.code == m.MS_E_BUDGET
    sid = srv.open(S.drop_boxes(8, seed=0))
    with pytest.raises(m.MsError):
        srv.submit(sid, 0)
    srv.wait(srv.submit(sid, 1))
    srv.close_session(sid)
    with pytest.raises(m.MsError):
        srv.submit(sid, 1)
    srv.close()


def test_load_generator_runs():
    m = ms()
    from paper_2410_00425_amd import serve_load as L
    pool = L.ScenePool(seed=0)
    srv = m.Server(256 << 20)
    recs, wall = L.run_clients(m, srv, pool, float("inf"), n_clients=3, sessions_per_client=1, reqs_per_session=3)
    s = L.summarize(recs, wall)
    srv.close()
    assert s["requests"] == 9 and s["p99_ms"] >= s["p50_ms"] > 0


def test_served_session_matches_oracle():
    """A session served next to other sessions, compared directly with the float32 oracle (not
    only with the same batch stepped alone): tray and arm sessions over 10 two-step requests,
    the arm's targets redrawn at each request."""
    from oracle.oracle import Oracle
    from parity import compare_states
    m = ms()
    tray, arm, boxes = S.tray(48, seed=51), S.arm_cube(24, seed=52), S.drop_boxes(100, seed=53)
    srv = m.Server(256 << 20)
    st, sa, sb = srv.open(tray), srv.open(arm), srv.open(boxes)
    o_t, o_a = Oracle(tray, 32), Oracle(arm, 32)
    for r in range(10):
        t = S.arm_targets(52, np.arange(24), r).reshape(-1).astype(np.float32)
        reqs = [srv.submit(st, 2), srv.submit(sa, 2, t), srv.submit(sb, 1)]
        for q in reqs:
            srv.wait(q)
        o_t.step(2, n_threads=8)
        o_a.set_targets(t)
        o_a.step(2, n_threads=8)
    for sid, sc, o in ((st, tray, o_t), (sa, arm, o_a)):
        g, w = srv.get_state(sid), o.state()
        _, mm = o.counters()
        bad, excused = compare_states(sc, g, w, mm)
        assert not bad, (sc.name, bad)
        same = sum(all(np.array_equal(g[k][:, sc.body_off[e]:sc.body_off[e + 1]],
                                      w[k][:, sc.body_off[e]:sc.body_off[e + 1]].astype(np.float32))
                       for k in ("pos", "quat", "linvel", "angvel")) for e in range(sc.n_envs))
        assert same >= sc.n_envs - 2, (sc.name, same)
    for s in (st, sa, sb):
        srv.close_session(s)
    srv.drain()
    srv.close()
