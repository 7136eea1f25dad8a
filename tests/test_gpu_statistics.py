"""Full-length runs of every workload on the GPU against the float32 oracle, compared by
statistics (piles of contacting bodies are chaotic, so single trajectories may part after a
near-tie decision): final centre-of-mass heights by shape, fraction of envs at rest, contact
points per env at the last step and kinetic energy over time, each by a two-sample
Kolmogorov-Smirnov test (p > 0.01) and a difference of means within 3 standard errors; no env
may overflow its contact or colour capacity, and the number of envs that stay bit-identical is
reported and bounded below.  Workloads at their own lengths: one box per env (200 steps), the
7-link arm with targets redrawn every 50 steps (1000 steps), the tray of 20 bodies (500 steps),
the heterogeneous batch (500 steps), the tray of 12 objects about half of them compound bodies
(500 steps); 512 envs each.  Plus a scene that overflows the 64
parallel colours, against the oracle."""
import numpy as np
import pytest
from scipy import stats
from scipy.spatial.transform import Rotation

from oracle.oracle import Oracle, compound_mass_props, mass_props
from paper_2410_00425_amd import scenes as S

from parity import compare_states

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N_ENVS = 512
THREADS = 16


def ms():
    from paper_2410_00425_amd import ms as m
    return m


def mass_inertia(sc):
    bd = sc.bodies
    m = np.zeros(sc.n_bodies)
    inertia = np.zeros((sc.n_bodies, 3))
    for i in range(sc.n_bodies):
        if bd["flags"][i] & 1:
            continue
        dims = bd["dims"][i].astype(np.float64)
        if bd["shape"][i] == S.COMPOUND:
            rec = sc.compounds[int(dims[0])]
            vol, _ = compound_mass_props(rec, 1.0)
            mi = float(bd["mass"][i]) if bd["mass"][i] > 0 else float(bd["density"][i]) * vol
            _, inertia[i] = compound_mass_props(rec, mi)
        else:
            vol, _ = mass_props(int(bd["shape"][i]), dims, 1.0)
            mi = float(bd["mass"][i]) if bd["mass"][i] > 0 else float(bd["density"][i]) * vol
            _, inertia[i] = mass_props(int(bd["shape"][i]), dims, mi)
        m[i] = mi
    return m, inertia


def kinetic_energy(sc, st, m, inertia):
    q = np.asarray(st["quat"], np.float64)
    rot = Rotation.from_quat(np.stack([q[1], q[2], q[3], q[0]], axis=1))
    wb = rot.inv().apply(np.asarray(st["angvel"], np.float64).T)
    v = np.asarray(st["linvel"], np.float64).T
    ke = 0.5 * m * np.sum(v * v, axis=1) + 0.5 * np.sum(inertia * wb * wb, axis=1)
    return np.add.reduceat(ke, sc.body_off[:-1])


def same_distribution(a, b, what, floor=1e-9):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    if np.array_equal(np.sort(a), np.sort(b)):
        return
    p = stats.ks_2samp(a, b).pvalue
    se = np.sqrt(a.var(ddof=1) / len(a) + b.var(ddof=1) / len(b)) if len(a) > 1 else 0.0
    assert p > 0.01, f"{what}: KS p = {p:.3g}"
    assert abs(a.mean() - b.mean()) <= 3.0 * se + floor, f"{what}: means {a.mean():.6g} vs {b.mean():.6g} (SE {se:.3g})"


def run_both(name, steps, chunk=10, redraw_every=0, seed=5):
    sc = S.by_name(name, N_ENVS, seed=seed)
    b = ms().Batch(sc)
    o = Oracle(sc, 32)
    m, inertia = mass_inertia(sc)
    ids = np.arange(N_ENVS)
    ke_g, ke_o = [], []
    done = 0
    while done < steps:
        tg = None
        if redraw_every and done % redraw_every == 0:
            t = S.arm_targets(seed, ids, done // redraw_every).reshape(-1)
            tg = torch.from_numpy(t).cuda()
            o.set_targets(t)
        k = min(chunk, steps - done)
        if done + k == steps:
            # the last step alone, to read its contact counts on both sides
            if k > 1:
                b.step(k - 1, tg)
                o.step(k - 1, n_threads=THREADS)
                tg = None
            b.stats(reset=True)
            b.step(1, tg)
            o.step(1, n_threads=THREADS)
        else:
            b.step(k, tg)
            o.step(k, n_threads=THREADS)
        done += k
        g, w = b.state_numpy(), o.state()
        ke_g.append(kinetic_energy(sc, g, m, inertia))
        ke_o.append(kinetic_energy(sc, w, m, inertia))
    pts_g = b.stats()[:, 13]
    pts_o = o.counters()[0][:, 2]
    b.close()
    return sc, g, w, np.array(ke_g), np.array(ke_o), pts_g, pts_o


@pytest.mark.parametrize("name,steps,redraw,min_same", [
    ("drop_boxes", 200, 0, 0.95),
    ("arm_cube", 1000, 50, 0.5),
    ("tray", 500, 0, 0.25),
    ("hetero", 500, 0, 0.5),
    ("compound_tray", 500, 0, 0.5),
])
def test_full_length_statistics(name, steps, redraw, min_same):
    print(f"stats: {name} x {N_ENVS}, {steps} steps", flush=True)
    sc, g, w, ke_g, ke_o, pts_g, pts_o = run_both(name, steps, redraw_every=redraw)
    # no capacity overflow on either side, nothing frozen
    assert np.all(g["status"] == 0) and np.all(w["status"] == 0), (np.unique(g["status"]), np.unique(w["status"]))
    # envs that stayed bit-identical
    bo = sc.body_off
    same = 0
    for e in range(sc.n_envs):
        sl = slice(bo[e], bo[e + 1])
        if all(np.array_equal(g[k][:, sl], w[k][:, sl].astype(np.float32)) for k in ("pos", "quat", "linvel", "angvel")):
            same += 1
    print(f"stats: {name}: {same}/{sc.n_envs} envs bit-identical after {steps} steps", flush=True)
    assert same >= min_same * sc.n_envs, f"{same}/{sc.n_envs} bit-identical"
    dyn = (sc.bodies["flags"] & 1) == 0
    # final COM height by shape
    for shape, label in ((S.SPHERE, "sphere"), (S.CAPSULE, "capsule"), (S.BOX, "box"), (S.COMPOUND, "compound")):
        sel = dyn & (sc.bodies["shape"] == shape)
        if sel.sum() > 1:
            same_distribution(g["pos"][2, sel], w["pos"][2, sel], f"{name} final z ({label})")
    # fraction at rest (every dynamic body of the env below 1 cm/s)
    env_of = np.repeat(np.arange(sc.n_envs), np.diff(bo))

    def at_rest(st):
        spd = np.linalg.norm(np.asarray(st["linvel"], np.float64), axis=0)
        moving = np.zeros(sc.n_envs, bool)
        np.logical_or.at(moving, env_of[dyn], spd[dyn] >= 1e-2)
        return ~moving
    same_distribution(at_rest(g).astype(float), at_rest(w).astype(float), f"{name} at rest")
    # contact points per env at the last step
    same_distribution(pts_g, pts_o, f"{name} contact points")
    # kinetic energy over time (every 10 steps) and at the end
    for t in range(len(ke_g)):
        same_distribution(ke_g[t], ke_o[t], f"{name} KE at record {t}", floor=1e-9 * (1 + abs(ke_o[t]).max()))


def colour_overflow_scene():
    """A box on the ground hinged to the world by 64 identical revolute joints about the
    vertical through its centre (64 joint blocks on one body: colours 0..63), spinning, with
    three spheres on it: its ground and sphere contacts fall in the serial overflow colour."""
    box = S.body(S.BOX, (0.1, 0.1, 0.025), (0.0, 0.0, 0.025), mass=2.0, mu=0.02, angvel=(0.0, 0.0, 2.0))
    spheres = [S.body(S.SPHERE, (0.02,), (x, y, 0.07), mass=0.1, mu=0.5) for x, y in
               ((0.05, 0.0), (-0.04, 0.03), (0.0, -0.05))]
    fp = (0.0, 0.0, 0.025, 1.0, 0.0, 0.0, 0.0)
    fc = (0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0)
    joints = [S.joint(-1, 0, fp, fc, kp=0.0, kd=0.01 if j == 0 else 0.0) for j in range(64)]
    return S.single([box] + spheres, joints, dt=0.005, pos_iters=8)


def test_colour_overflow_matches_oracle():
    print("stats: colour overflow", flush=True)
    one = colour_overflow_scene()
    sc = S.replicate(one, 8)
    b = ms().Batch(sc)
    o = Oracle(sc, 32)
    for steps in (1, 9, 40):
        b.step(steps)
        o.step(steps)
        g, w = b.state_numpy(), o.state()
        assert np.all(g["status"] == 4) and np.all(w["status"] == 4), (g["status"], w["status"])
        _, mm = o.counters()
        bad, excused = compare_states(sc, g, w, mm)
        assert not bad and not excused, (steps, bad, excused)
        for k in ("pos", "quat", "linvel", "angvel"):
            assert np.array_equal(g[k], w[k].astype(np.float32)), (steps, k)
    # the box kept spinning about its hinge and the spheres stayed on it
    assert abs(g["angvel"][2, 0]) > 0.03
    assert np.all(g["pos"][2, 1:4] > 0.06)
    b.close()
