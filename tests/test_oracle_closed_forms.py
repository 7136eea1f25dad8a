"""Oracle pins against closed-form mechanics (CPU only).

Each case is a configuration whose answer follows from textbook mechanics, independent of the
oracle's code: the discrete free-fall sum of symplectic Euler, Coulomb sliding deceleration mu g,
stick / slip on an incline, the small-angle physical-pendulum period, and restitution.  The
solver settings of the paper's simulation benchmark (App. E, Setup: 120 Hz, 4 position and 0
velocity iterations) and its PD joint drive (App. B, Controller) are the regime exercised.
"""
import math

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2410_00425_amd import scenes as S

G32 = float(np.float32(9.81))


def _one(bodies, joints=None, **kw):
    return S.single(bodies, joints, **kw)


@pytest.mark.parametrize("prec,tol", [(64, 1e-12), (32, 1e-6)])
@pytest.mark.parametrize("S_sub,n", [(4, 10), (8, 25), (1, 7)])
def test_free_fall_exact_discrete(prec, tol, S_sub, n):
    # Symplectic Euler with S substeps of h = dt/S: after n steps (N = nS substeps)
    # z = z0 - g h^2 N (N + 1) / 2 = z0 - g dt^2 n (nS + 1) / (2S), v = -g n dt.
    dt, z0 = 0.01, 10.0
    sc = _one([S.body(S.SPHERE, (0.1,), (0.3, -0.2, z0), mass=2.0)], dt=dt, pos_iters=S_sub, plane_enabled=0)
    o = Oracle(sc, prec)
    o.step(n)
    st = o.state()
    g = G32
    dt32 = float(np.float32(dt))
    z = z0 - g * dt32 ** 2 * n * (n * S_sub + 1) / (2 * S_sub)
    assert abs(st["pos"][2, 0] - z) <= tol * max(1.0, abs(z))
    assert abs(st["linvel"][2, 0] + g * n * dt32) <= tol * 10
    # inputs are float32 records: horizontal position is unchanged
    assert st["pos"][0, 0] == pytest.approx(float(np.float32(0.3)), abs=tol)
    assert st["pos"][1, 0] == pytest.approx(float(np.float32(-0.2)), abs=tol)


def test_free_fall_golden_table():
    # tests/golden/free_fall.txt: closed-form values (dt=0.01, S=4, n=10: 0.05027625 m drop).
    rows = [l.split() for l in open(__file__.replace("test_oracle_closed_forms.py", "golden/free_fall.txt"))
            if l.strip() and not l.startswith("#")]
    for S_sub, n, dz in ((int(a), int(b), float(c)) for a, b, c in rows):
        sc = _one([S.body(S.SPHERE, (0.1,), (0, 0, 5.0), mass=1.0)], dt=0.01, pos_iters=S_sub, plane_enabled=0,
                  gravity=(0, 0, -9.81))
        o = Oracle(sc, 64)
        o.step(n)
        drop = 5.0 - o.state()["pos"][2, 0]
        # the table uses g = 9.81 and dt = 0.01 exactly; the oracle reads float32 inputs
        scale = (G32 / 9.81) * (float(np.float32(0.01)) / 0.01) ** 2
        assert drop == pytest.approx(dz * scale, rel=1e-9)


@pytest.mark.parametrize("prec", [64, 32])
def test_sliding_box_coulomb(prec):
    # A 0.1 m, 1 kg box resting on the ground and sliding at 2 m/s with mu = 0.5 decelerates at
    # mu g and stops after v0 / (mu g) = 0.4077 s having travelled v0^2 / (2 mu g) = 0.4077 m.
    mu, v0 = 0.5, 2.0
    sc = _one([S.body(S.BOX, (0.05, 0.05, 0.05), (0, 0, 0.05), mass=1.0, mu=mu, linvel=(v0, 0, 0))],
              dt=0.01, pos_iters=4, plane_friction=mu)
    o = Oracle(sc, prec)
    v, x = [], []
    for _ in range(70):
        o.step(1)
        st = o.state()
        v.append(st["linvel"][0, 0])
        x.append(st["pos"][0, 0])
    v, x = np.array(v), np.array(x)
    a = mu * 9.81
    # deceleration from the sliding phase (steps 5..30), fitted
    t = 0.01 * np.arange(1, 71)
    sl = slice(5, 30)
    slope = np.polyfit(t[sl], v[sl], 1)[0]
    assert -slope == pytest.approx(a, rel=0.02)
    stop = np.argmax(v < 1e-4)
    assert stop > 0
    assert 0.01 * (stop + 1) == pytest.approx(v0 / a, abs=0.02)
    assert x[-1] == pytest.approx(v0 ** 2 / (2 * a), rel=0.02)
    # at rest: the box no longer moves (position change over the last 20 steps)
    assert abs(x[-1] - x[-21]) < 1e-4


@pytest.mark.parametrize("alpha_deg,mu,sub,sticks,creep", [(10.0, 0.5, 4, True, 1e-3), (20.0, 0.5, 8, True, 1e-3),
                                                            (20.0, 0.5, 4, True, 1e-2), (35.0, 0.5, 4, False, 0),
                                                            (40.0, 0.3, 8, False, 0)])
def test_incline_stick_slip(alpha_deg, mu, sub, sticks, creep):
    # An incline is a ground plane under gravity rotated by alpha about y.  A box sticks when
    # tan(alpha) < mu; otherwise it accelerates at g (sin(alpha) - mu cos(alpha)).  The step
    # model keeps no impulses across steps, so a sticking box creeps at a small rate (each
    # step's first substep starts from zero impulses): < 1 mm in 1 s at 10 degrees with 4
    # substeps and at 20 degrees with 8 substeps; < 1 cm at 20 degrees with 4 substeps.
    al = math.radians(alpha_deg)
    g = (9.81 * math.sin(al), 0.0, -9.81 * math.cos(al))
    sc = _one([S.body(S.BOX, (0.05, 0.05, 0.05), (0, 0, 0.05), mass=1.0, mu=mu)], dt=0.01, pos_iters=sub,
              plane_friction=mu, gravity=g)
    o = Oracle(sc, 64)
    xs = []
    for _ in range(100):
        o.step(1)
        xs.append(o.state()["pos"][0, 0])
    xs = np.array(xs)
    if sticks:
        assert abs(xs[-1]) < creep
        # no runaway: the second half-second moves no more than 1.25x the first
        assert abs(xs[-1] - xs[49]) <= 1.25 * abs(xs[49]) + 1e-6
    else:
        t = 0.01 * np.arange(1, 101)
        acc = 2 * np.polyfit(t[20:], xs[20:], 2)[0]
        gs, gc = 9.81 * math.sin(al), 9.81 * math.cos(al)
        # gravity is stored in float32; the expected value uses the same components
        gs, gc = float(np.float32(gs)), float(np.float32(gc))
        assert acc == pytest.approx(gs - mu * gc, rel=0.02)


@pytest.mark.parametrize("prec", [64, 32])
def test_pendulum_small_angle_period(prec):
    # Sphere r = 0.05, m = 1 hung d = 0.5 m below a world revolute joint (axis y), released at
    # 0.05 rad: T0 = 2 pi sqrt((2/5 m r^2 + m d^2) / (m g d)) = 1.4213 s (finite-amplitude
    # factor 1.00016).  Measured over 5 periods; the anchor must stay within 1e-3 m.
    d, r, th0 = 0.5, 0.05, 0.05
    qy = (math.sqrt(0.5), -math.sqrt(0.5), 0.0, 0.0)
    piv = (0.0, 0.0, 1.0)
    # rotation by th0 about +y maps the body's z axis to (sin th0, 0, cos th0); the anchor sits
    # d along that axis from the centre, at the pivot
    pos = (-d * math.sin(th0), 0.0, piv[2] - d * math.cos(th0))
    quat = (math.cos(th0 / 2), 0.0, math.sin(th0 / 2), 0.0)
    sc = _one([S.body(S.SPHERE, (r,), pos, quat=quat, mass=1.0)],
              [S.joint(-1, 0, piv + qy, (0.0, 0.0, d) + qy)], dt=0.01, pos_iters=4, plane_enabled=0)
    o = Oracle(sc, prec)
    xs, drift = [], 0.0
    for _ in range(1000):
        o.step(1)
        st = o.state()
        p = st["pos"][:, 0]
        q = st["quat"][:, 0]
        # anchor of the body = p + R(q) (0, 0, d)
        w, x, y, z = q
        anchor = p + d * np.array([2 * (x * z + w * y), 2 * (y * z - w * x), 1 - 2 * (x * x + y * y)])
        drift = max(drift, np.linalg.norm(anchor - np.array(piv)))
        xs.append(p[0])
    xs = np.array(xs)
    down = np.nonzero((xs[:-1] > 0) & (xs[1:] <= 0))[0]
    # sub-step interpolation of the crossings
    tc = [(k + xs[k] / (xs[k] - xs[k + 1])) * 0.01 for k in down]
    T = (tc[5] - tc[0]) / 5
    T0 = 2 * math.pi * math.sqrt((0.4 * r * r + d * d) / (9.81 * d)) * 1.00016
    assert T == pytest.approx(T0, rel=0.005)
    assert drift <= 1e-3


@pytest.mark.parametrize("e,h", [(0.5, 0.5), (0.8, 0.3)])
def test_restitution_rebound(e, h):
    # A sphere dropped from height h (bottom above ground) hits at sqrt(2 g h) and leaves at
    # e sqrt(2 g h).  Velocity iterations run the restitution pass; threshold 1 m/s.
    r = 0.05
    sc = _one([S.body(S.SPHERE, (r,), (0, 0, r + h), mass=1.0, e=e)], dt=0.002, pos_iters=4, vel_iters=1,
              plane_restitution=0.0)
    o = Oracle(sc, 64)
    vz = []
    for _ in range(400):
        o.step(1)
        vz.append(o.state()["linvel"][2, 0])
    vz = np.array(vz)
    k = np.argmax(vz > 0)
    assert k > 0
    v_in = math.sqrt(2 * 9.81 * h)
    assert vz[k] == pytest.approx(e * v_in, rel=0.03)


def test_drop_box_rests():
    # 16 boxes of 0.1 m dropped with random orientation settle flat: after 200 steps the centre
    # is at the half-extent 0.05 m within 1e-3 m and the speed is below 1e-2 m/s.
    sc = S.drop_boxes(16, seed=0)
    o = Oracle(sc, 32)
    o.step(200)
    st = o.state()
    assert np.all(np.abs(st["pos"][2] - 0.05) < 1e-3)
    assert np.all(np.linalg.norm(st["linvel"], axis=0) < 1e-2)
    assert np.all(st["status"] == 0)
    # resting penetration is within the tolerance
    assert np.all(st["pos"][2] > 0.05 - 1e-3)
