"""Compound bodies on the GPU (libms through its C ABI) against the float32 oracle: bodies made of
up to 4 primitive parts, the convex pieces of decomposed objects (Sec. III-B; App. B,
Environment Setup), each pair of parts with its own manifold.

One step from a common state gives bit-identical candidate lists, identical per-pair point
counts and decision codes (64 + the first pair of parts with points), and states within the
parity rule; whole runs stay bit-identical env by env; a one-part compound steps exactly like
its primitive; the tiling, the capacity rule, the work counters per shape kind, the contact
cache and the contact-force readout hold for compounds as for primitives."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2410_00425_amd import scenes as S

from parity import compare_states
from test_gpu_parity import one_step_parity, oracle_state, set_all

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FIELDS = ("pos", "quat", "linvel", "angvel")


def ms():
    from paper_2410_00425_amd import ms as m
    return m


def same_envs(sc, g, w):
    bo = sc.body_off
    out = []
    for e in range(sc.n_envs):
        sl = slice(bo[e], bo[e + 1])
        out.append(all(np.array_equal(g[k][:, sl], w[k][:, sl].astype(np.float32)) for k in FIELDS))
    return np.array(out)


@pytest.mark.parametrize("warm", [12, 60, 150])
def test_compound_tray_one_step(warm):
    print(f"compound: one step after {warm}", flush=True)
    sc = S.compound_tray(96, seed=7)
    one_step_parity(sc, oracle_state(sc, warm), max_excused=1)


def test_compound_tray_run_matches_oracle():
    print("compound: 120-step run", flush=True)
    sc = S.compound_tray(128, seed=8)
    b = ms().Batch(sc)
    o = Oracle(sc, 32)
    for _ in range(4):
        b.step(30)
        o.step(30, n_threads=16)
    g, w = b.state_numpy(), o.state()
    assert np.array_equal(g["status"], w["status"])
    same = same_envs(sc, g, w)
    print(f"compound: {same.sum()}/{sc.n_envs} envs bit-identical after 120 steps", flush=True)
    assert same.mean() >= 0.75
    # the counters per shape kind of the last step agree env by env where the env is identical
    b.stats(reset=True)
    b.step(1)
    o.step(1, n_threads=16)
    st = b.stats()
    c, _ = o.counters()
    same = same_envs(sc, b.state_numpy(), o.state())
    assert same.sum() > 0
    assert np.array_equal(st[same, 1:13], c[same, 8:20])
    assert np.array_equal(st[same, 13], c[same, 2]) and np.array_equal(st[same, 14], c[same, 3])
    # compound part pairs were counted (sphere, capsule and box parts against the ground)
    assert c[:, 8 + 9:8 + 12].sum() > 0
    b.close()


def one_part_scenes(n=8):
    prim, comp = [], []
    rng = np.random.default_rng(3)
    recs = []
    for e in range(n):
        shape = [S.SPHERE, S.CAPSULE, S.BOX][e % 3]
        dims = [(0.04,), (0.03, 0.05), (0.05, 0.03, 0.02)][e % 3]
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        other = S.body(S.BOX, (0.04, 0.04, 0.04), (0.03, 0.02, 0.25), mass=0.5, mu=0.6, angvel=(1.0, 0.0, 2.0))
        kw = dict(quat=tuple(q), density=800.0, mu=0.7, angvel=(0.5, 2.0, 0.0))
        prim.append(np.concatenate([S.body(shape, dims, (0.0, 0.0, 0.12), **kw), other]))
        comp.append(np.concatenate([S.body(S.COMPOUND, (float(e),), (0.0, 0.0, 0.12), **kw), other]))
        recs.append(S.compound_record([(shape, dims, (0.0, 0.0, 0.0), (1.0, 0.0, 0.0, 0.0))]))
    p = S.make_params(dt=0.005, pos_iters=8)
    a = S.concat_envs("one_part_prim", p, prim, [np.zeros(0, S.JOINT_DTYPE)] * n, {})
    c = S.concat_envs("one_part_comp", p.copy(), comp, [np.zeros(0, S.JOINT_DTYPE)] * n, {})
    c.compounds = np.array(recs, dtype=S.COMPOUND_DTYPE)
    return a, c


def test_one_part_compound_is_the_primitive():
    print("compound: one-part identity", flush=True)
    a, c = one_part_scenes()
    ba, bc = ms().Batch(a), ms().Batch(c)
    o = Oracle(c, 32)
    for _ in range(4):
        ba.step(40)
        bc.step(40)
        o.step(40)
        ga, gc, w = ba.state_numpy(), bc.state_numpy(), o.state()
        for k in FIELDS:
            assert np.array_equal(ga[k], gc[k]), k
            assert np.array_equal(gc[k], w[k].astype(np.float32)), k
    ba.close()
    bc.close()


@pytest.mark.parametrize("lanes", [16, 32, 64])
def test_compound_tiling_is_bit_identical(lanes):
    print(f"compound: lanes {lanes}", flush=True)
    sc = S.compound_tray(40, seed=11)
    ref = ms().Batch(sc)
    alt = ms().Batch(sc, lanes_per_env=lanes)
    ref.step(25)
    alt.step(25)
    g, h = ref.state_numpy(), alt.state_numpy()
    for k in FIELDS + ("status",):
        assert np.array_equal(g[k], h[k]), k
    ref.close()
    alt.close()


def test_compound_capacity_overflow_matches_oracle():
    print("compound: capacity overflow", flush=True)
    sc = S.compound_tray(48, seed=12)
    sc.params["max_contacts_per_env"] = 28
    sc.params["max_manifolds_per_env"] = 12
    b = ms().Batch(sc)
    o = Oracle(sc, 32)
    for _ in range(3):
        b.step(25)
        o.step(25, n_threads=16)
    g, w = b.state_numpy(), o.state()
    assert np.any(w["status"] & 2)
    same = same_envs(sc, g, w)
    assert same.mean() >= 0.75
    assert np.array_equal(g["status"][same], w["status"][same])
    b.close()
    # one step from a common state: point counts per pair equal under the capacity rule
    one_step_parity(sc, oracle_state(sc, 80), max_excused=1)


def test_compound_warm_start_and_forces_match_oracle():
    print("compound: cache and forces", flush=True)
    sc = S.compound_tray(48, seed=13)
    sc.params["warm_start"] = 1
    st = oracle_state(sc, 150)
    b = ms().Batch(sc)
    o = Oracle(sc, 32)
    set_all(b, st)
    o.set_state(*[st[k].astype(np.float64) for k in FIELDS])
    b.set_contact_forces(True)
    for k in range(3):
        b.step(1)
        o.step(1, n_threads=16)
    g, w = b.state_numpy(), o.state()
    _, mm = o.counters()
    bad, excused = compare_states(sc, g, w, mm)
    assert not bad and len(excused) <= 1, (bad, excused)
    same = same_envs(sc, g, w)
    assert same.mean() >= 0.9
    f = b.contact_forces().cpu().numpy()
    fo = o.contact_forces().astype(np.float32)
    ok = np.repeat(same, np.diff(sc.body_off))
    assert np.array_equal(f[:, ok], fo[:, ok])
    assert np.abs(f[2]).max() > 0.1
    b.close()


def test_compound_batch_in_fused_and_served_steps():
    """A compound batch fused with primitive batches (ms_step_many, its no-allocation form) and
    served in a mix (ms_server) gives the same bits as stepped alone."""
    print("compound: fused and served", flush=True)
    import threading
    m = ms()
    scs = [S.compound_tray(48, seed=14), S.tray(32, seed=15), S.drop_boxes(40, seed=16)]

    def alone(sc, steps):
        b = m.Batch(sc)
        b.step(steps)
        st = b.state_numpy()
        b.close()
        return st

    refs = [alone(sc, 6) for sc in scs]
    for fn in (m.step_many, m.step_many_noalloc):
        bs = [m.Batch(sc) for sc in scs]
        for _ in range(3):
            fn(bs, 2)
        torch.cuda.synchronize()
        for b, ref in zip(bs, refs):
            st = b.state_numpy()
            for k in FIELDS + ("status",):
                assert np.array_equal(st[k], ref[k]), (fn.__name__, b.scene.name, k)
            b.close()
    srv = m.Server(128 << 20)
    sids = [srv.open(sc) for sc in scs]

    def drive(s):
        for _ in range(3):
            srv.wait(srv.submit(s, 2))

    th = [threading.Thread(target=drive, args=(s,)) for s in sids]
    for t in th:
        t.start()
    for t in th:
        t.join()
    got = [srv.get_state(s) for s in sids]
    for s in sids:
        srv.close_session(s)
    srv.drain()
    srv.close()
    for g, ref in zip(got, refs):
        for k in FIELDS + ("status",):
            assert np.array_equal(g[k], ref[k]), ("served", k)


def test_articulated_compound_matches_oracle():
    """Compound bodies on joints: a dumbbell pendulum swinging through two spheres, and the arm
    with its cube replaced by a bench compound; bit for bit against the oracle."""
    print("compound: on joints", flush=True)
    import math
    rec = S.dumbbell(0.03, 0.1, 0.01)
    qy = (math.sqrt(0.5), -math.sqrt(0.5), 0.0, 0.0)
    envs = []
    for e in range(16):
        th0 = 0.4 + 0.05 * e
        d = 0.3
        pos = (-d * math.sin(th0), 0.0, 1.0 - d * math.cos(th0))
        quat = (math.cos(th0 / 2), 0.0, math.sin(th0 / 2), 0.0)
        bodies = [S.body(S.COMPOUND, (0.0,), pos, quat=quat, mass=1.0),
                  S.body(S.SPHERE, (0.04,), (0.05, 0.0, 0.62), mass=0.3),
                  S.body(S.SPHERE, (0.03,), (0.12, 0.01, 0.66), mass=0.2)]
        envs.append(np.concatenate(bodies))
    joints = [S.joint(-1, 0, (0.0, 0.0, 1.0) + qy, (0.0, 0.0, 0.3) + qy, kd=0.01)] * 16
    p = S.make_params(dt=0.005, pos_iters=8, plane_enabled=0)
    sc = S.concat_envs("compound_pendulum", p, envs, joints, {})
    sc.compounds = np.array([rec], dtype=S.COMPOUND_DTYPE)
    # the arm, its cube a bench and its last link a dumbbell (the capsule link with a sphere at
    # each end), both compounds
    arm = S.arm_cube(8, seed=17)
    cube = np.nonzero(arm.bodies["shape"] == S.BOX)[0]
    recs = [S.bench(0.03, 0.02, 0.004, 0.004, 0.012)]
    arm.bodies["shape"][cube] = S.COMPOUND
    arm.bodies["dims"][cube] = 0.0
    arm.bodies["mass"][cube] = 0.2
    last = cube - 1
    assert np.all(arm.bodies["shape"][last] == S.CAPSULE)
    for e, i in enumerate(last):
        r, hl = float(arm.bodies["dims"][i][0]), float(arm.bodies["dims"][i][1])
        recs.append(S.dumbbell(1.2 * r, hl, r))
        arm.bodies["shape"][i] = S.COMPOUND
        arm.bodies["dims"][i] = (float(e + 1), 0.0, 0.0)
    arm.compounds = np.array(recs, dtype=S.COMPOUND_DTYPE)
    tg = S.arm_targets(17, np.arange(8), 1).reshape(-1)
    for scene, targets in ((sc, None), (arm, tg)):
        b = ms().Batch(scene)
        o = Oracle(scene, 32)
        t = None
        if targets is not None:
            o.set_targets(targets)
            t = torch.from_numpy(targets).cuda()
        for _ in range(4):
            b.step(50, t)
            o.step(50)
        g, w = b.state_numpy(), o.state()
        same = same_envs(scene, g, w)
        assert same.all(), (scene.name, np.nonzero(~same)[0])
        assert np.array_equal(g["status"], w["status"])
        b.close()


def test_static_compounds_pgs_and_restitution():
    """Static compound obstacles (benches as tables) under falling primitives and compounds, with
    the PGS solver, velocity iterations and restitution; one step from oracle states and a run."""
    print("compound: static compounds, PGS, restitution", flush=True)
    sc = S.compound_tray(48, seed=18)
    # the first object of every env becomes a static compound table
    first = sc.body_off[:-1]
    sc.bodies["shape"][first] = S.COMPOUND
    sc.bodies["dims"][first] = (float(len(sc.compounds)), 0.0, 0.0)
    sc.bodies["flags"][first] = 1
    sc.bodies["pos"][first] = (0.0, 0.0, 0.03)
    sc.bodies["quat"][first] = (1.0, 0.0, 0.0, 0.0)
    sc.compounds = np.concatenate([sc.compounds, np.array([S.bench(0.1, 0.08, 0.008, 0.01, 0.02)],
                                                          dtype=S.COMPOUND_DTYPE)])
    sc.params["solver"] = S.PGS
    sc.params["vel_iters"] = 2
    sc.bodies["restitution"] = 0.3
    one_step_parity(sc, oracle_state(sc, 100), max_excused=1)
    b = ms().Batch(sc)
    o = Oracle(sc, 32)
    b.step(150)
    o.step(150, n_threads=16)
    g, w = b.state_numpy(), o.state()
    same = same_envs(sc, g, w)
    assert same.mean() >= 0.75, same.sum()
    # the tables did not move
    assert np.array_equal(g["pos"][:, first], sc.bodies["pos"][first].T)
    b.close()


def four_part_scene(n_envs=32, seed=19):
    """Pairs of 4-part compounds (two spheres on x, two capsules on y: 16 pairs of parts per
    body pair, the most a candidate expands to) thrown at each other above the ground."""
    rec = S.compound_record([(S.SPHERE, (0.025,), (0.05, 0.0, 0.0), (1.0, 0.0, 0.0, 0.0)),
                             (S.SPHERE, (0.025,), (-0.05, 0.0, 0.0), (1.0, 0.0, 0.0, 0.0)),
                             (S.CAPSULE, (0.015, 0.03), (0.0, 0.05, 0.0), (1.0, 0.0, 0.0, 0.0)),
                             (S.CAPSULE, (0.015, 0.03), (0.0, -0.05, 0.0), (1.0, 0.0, 0.0, 0.0))])
    rng = np.random.default_rng(seed)
    envs = []
    for e in range(n_envs):
        q = rng.normal(size=(2, 4))
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        x = rng.uniform(0.09, 0.12)
        bodies = [S.body(S.COMPOUND, (0.0,), (-x, 0.0, 0.2), quat=tuple(q[0]), density=800.0, linvel=(0.6, 0.0, 0.0),
                         angvel=tuple(rng.normal(size=3))),
                  S.body(S.COMPOUND, (0.0,), (x, 0.01, 0.21), quat=tuple(q[1]), density=800.0, linvel=(-0.6, 0.0, 0.0)),
                  S.body(S.BOX, (0.05, 0.05, 0.01), (0.0, 0.0, 0.01), mass=1.0)]
        envs.append(np.concatenate(bodies))
    sc = S.concat_envs("four_part", S.make_params(dt=0.005, pos_iters=8, max_contacts_per_env=128,
                                                   max_manifolds_per_env=48),
                       envs, [np.zeros(0, S.JOINT_DTYPE)] * n_envs, {})
    sc.compounds = np.array([rec], dtype=S.COMPOUND_DTYPE)
    return sc


def test_four_part_compounds_match_oracle():
    print("compound: 4-part pairs", flush=True)
    sc = four_part_scene()
    for warm in (25, 40, 80):
        one_step_parity(sc, oracle_state(sc, warm), max_excused=1)
    b = ms().Batch(sc)
    o = Oracle(sc, 32)
    b.step(150)
    o.step(150)
    g, w = b.state_numpy(), o.state()
    assert same_envs(sc, g, w).all()
    assert np.all(w["status"] == 0)
    b.close()


def test_full_size_compound_tray_sampled_envs():
    """4096 compound-tray envs in the benchmark's launch configuration (200 settling steps, the
    autotuner, 5 more steps); 48 sampled envs run by the oracle alone over the same 205 steps
    from the same generator state (an env does not depend on its batch), compared bit for bit."""
    print("compound: full size, sampled envs", flush=True)
    sc = S.compound_tray(4096, seed=0)
    rng = np.random.default_rng(1)
    sample = np.sort(rng.choice(4096, 48, replace=False))
    sub = sc.subset(sample)
    b = ms().Batch(sc)
    b.step(200)
    b.tune(5)   # trial steps restore the state
    b.step(5)
    g = b.state_numpy()
    o = Oracle(sub, 32)
    o.step(205, n_threads=16)
    w = o.state()
    bo = sc.body_off
    gs = {k: np.concatenate([g[k][:, bo[e]:bo[e + 1]] for e in sample], axis=1) for k in FIELDS}
    same = same_envs(sub, gs, w)
    assert same.mean() >= 0.9, same.sum()
    assert np.all(g["status"][sample] == w["status"])
    b.close()
