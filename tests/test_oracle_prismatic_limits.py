"""Oracle pins for prismatic joints, joint limits and the cart-pole (CPU).

The paper's simulation-only benchmark is a cart-pole (App. E, Setup: 120 Hz simulation, 4
position and 0 velocity iterations); its classic-control tasks drive such robots with joint
position controllers (App. A, Classic Control), and its locomotion robots use constrained joint
limits (App. A, Locomotion).  Pins from textbook mechanics, independent of the oracle's code:
  * a frictionless slider inclined at alpha: motion along the rail is exact symplectic Euler
    under g sin(alpha); the body stays on the rail and does not rotate;
  * a PD-driven vertical slider sags to x = -m g / kp;
  * a cart-pole with a free cart and a hanging pole oscillates at
    w^2 = m g l / (I_c + m l^2 M / (M + m)) and conserves horizontal momentum;
  * limits: a pendulum thrown at its limit never passes it and one resting on it under gravity
    stays there; a slider driven past its limit stops at it.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle.oracle import Oracle, mass_props
from paper_2410_00425_amd import scenes as S

G32 = float(np.float32(9.81))
QY = (math.sqrt(0.5), -math.sqrt(0.5), 0.0, 0.0)   # frame whose z is the world y


def _quat_z_to(v):
    """(w, x, y, z) of a rotation taking +z to unit v."""
    R = Rotation.align_vectors([v], [[0, 0, 1]])[0]
    x, y, z, w = R.as_quat()
    return (w, x, y, z)


def _axis(q):
    """The z axis of float32 quaternion q (what the oracle reads)."""
    w, x, y, z = (float(np.float32(c)) for c in q)
    return Rotation.from_quat([x, y, z, w]).apply([0, 0, 1])


@pytest.mark.parametrize("alpha_deg,sub", [(30.0, 4), (60.0, 8)])
def test_prismatic_incline_exact_slide(alpha_deg, sub):
    # A box on a world slider whose axis points down an incline at alpha.  The rows across the
    # rail remove the perpendicular velocity exactly (anchor at the centre of mass: no rotation
    # coupling), so the distance along the rail after N substeps is g_a h^2 N (N + 1) / 2 with
    # g_a = g . axis, and the body stays on the rail without rotating.
    al = math.radians(alpha_deg)
    u = np.array([math.cos(al), 0.0, -math.sin(al)])
    q = _quat_z_to(u)
    x0 = (0.1, -0.2, 2.0)
    b = S.body(S.BOX, (0.05, 0.04, 0.03), x0, mass=1.5)
    j = S.joint(-1, 0, x0 + q, (0.0, 0.0, 0.0) + q, type=S.PRISMATIC)
    dt, n = 0.01, 40
    sc = S.single([b], [j], dt=dt, pos_iters=sub, plane_enabled=0)
    o = Oracle(sc, 64)
    o.step(n)
    st = o.state()
    ax = _axis(q)
    h = float(np.float32(dt)) / sub
    N = n * sub
    ga = np.array([0.0, 0.0, -G32]) @ ax
    disp = st["pos"][:, 0] - np.array([float(np.float32(c)) for c in x0])
    # (the frame quaternion is a float32 record, unit only to ~1e-8: the rail axis the oracle
    # builds from it differs from the unit axis at that level)
    assert disp @ ax == pytest.approx(ga * h * h * N * (N + 1) / 2, rel=1e-6)
    assert np.linalg.norm(disp - (disp @ ax) * ax) < 1e-7
    assert np.allclose(st["quat"][:, 0], [1, 0, 0, 0], atol=1e-12)
    assert st["linvel"][:, 0] @ ax == pytest.approx(ga * h * N, rel=1e-6)


def test_prismatic_drive_static_sag():
    # A vertical slider (axis +z) held by a PD drive toward 0: equilibrium kp x = -m g.
    m, kp, kd = 2.0, 4000.0, 200.0
    q = (1.0, 0.0, 0.0, 0.0)
    x0 = (0.0, 0.0, 1.0)
    b = S.body(S.SPHERE, (0.05,), x0, mass=m)
    j = S.joint(-1, 0, x0 + q, (0.0, 0.0, 0.0) + q, kp=kp, kd=kd, target=0.0, type=S.PRISMATIC)
    sc = S.single([b], [j], dt=0.01, pos_iters=4, plane_enabled=0)
    o = Oracle(sc, 64)
    o.step(400)
    z = o.state()["pos"][2, 0] - 1.0
    assert z == pytest.approx(-m * G32 / kp, rel=1e-3)
    assert abs(o.state()["linvel"][2, 0]) < 1e-6


def test_cartpole_free_cart_hanging_pole_period():
    # Cart M on a frictionless rail (no drive, no limit) and a pole (mass m, centre at l from the
    # hinge, inertia I_c about its centre) hanging down, released at 0.05 rad: small oscillations
    # at w^2 = m g l / (I_c + m l^2 M / (M + m)); horizontal momentum stays zero.
    bodies, joints = S.cartpole_bodies_joints(math.pi - 0.05)
    rail, hinge = joints
    rail["kp"], rail["kd"], rail["limited"] = 0.0, 0.0, 0
    sc = S.single(bodies, [rail, hinge], dt=1.0 / 240.0, pos_iters=8, plane_enabled=0)
    o = Oracle(sc, 64)
    M, m = S.CART_MASS, S.POLE_MASS
    l = S.POLE_HL + S.POLE_R
    _, I = mass_props(S.CAPSULE, [S.POLE_R, S.POLE_HL, 0.0], m)
    w2 = m * G32 * l / (I[0] + m * l * l * M / (M + m))
    T = 2 * math.pi / math.sqrt(w2) * (1 + 0.05 ** 2 / 16)
    dt = float(np.float32(1.0 / 240.0))
    rel, mom = [], []
    for _ in range(int(6 * T / dt)):
        o.step(1)
        st = o.state()
        rel.append(st["pos"][0, 1] - st["pos"][0, 0])
        mom.append(M * st["linvel"][0, 0] + m * st["linvel"][0, 1])
    rel = np.array(rel) - np.mean(rel)
    t = dt * np.arange(1, len(rel) + 1)
    up = np.where((rel[:-1] < 0) & (rel[1:] >= 0))[0]
    tc = t[up] - rel[up] * dt / (rel[up + 1] - rel[up])   # linear interpolation of the crossings
    periods = np.diff(tc)
    assert len(periods) >= 4
    assert np.mean(periods) == pytest.approx(T, rel=5e-3)
    # the rail axis comes from a float32 frame quaternion and tilts from the horizontal by
    # ~3e-8 rad, so gravity pushes the pair along it by (M + m) g 3e-8 per second
    assert np.max(np.abs(mom)) < (M + m) * G32 * 1e-7 * t[-1]


def _pendulum(limits, theta0, w0, kp=0.0, kd=0.0, target=0.0):
    # a 1 kg sphere 0.5 m below a world hinge about y; theta = rotation about y from hanging
    d = 0.5
    c, s = math.cos(theta0), math.sin(theta0)
    qb = (math.cos(0.5 * theta0), 0.0, math.sin(0.5 * theta0), 0.0)
    b = S.body(S.SPHERE, (0.05,), (-d * s, 0.0, 2.0 - d * c), qb, mass=1.0, angvel=(0.0, w0, 0.0),
               linvel=(-d * c * w0, 0.0, d * s * w0))
    j = S.joint(-1, 0, (0.0, 0.0, 2.0) + QY, (0.0, 0.0, d) + QY, kp=kp, kd=kd, target=target, limits=limits)
    return S.single([b], [j], dt=0.01, pos_iters=4, plane_enabled=0)


def _hinge_angle(st):
    # twist of the child's frame about the hinge axis relative to the world frame (both QY)
    w, x, y, z = st["quat"][:, 0]
    R = Rotation.from_quat([x, y, z, w])
    qf = Rotation.from_quat([QY[1], QY[2], QY[3], QY[0]])
    rel = (qf.inv() * R * qf).as_quat()
    if rel[3] < 0:
        rel = -rel
    return 2 * math.atan2(rel[2], rel[3])


def test_revolute_limit_is_never_passed():
    # Thrown at 4 rad/s toward an upper limit of 0.3 rad (the swing would reach ~0.6 rad): the
    # angle stays at or below the limit (within the Baumgarte correction) and reaches it.
    sc = _pendulum((-0.3, 0.3), 0.1, -4.0)
    o = Oracle(sc, 64)
    ang = []
    for _ in range(200):
        o.step(1)
        ang.append(_hinge_angle(o.state()))
    ang = np.array(ang)
    # the drive angle's sign convention: the hinge frame's z is world y, so the thrown swing
    # runs toward one limit; the check covers both
    assert np.max(np.abs(ang)) <= 0.3 + 2e-3
    assert np.max(np.abs(ang)) >= 0.3 - 2e-3


def test_revolute_limit_holds_under_gravity():
    # Limits [0.2, 0.5] rad, the pendulum released at 0.35 rad (a rotation by 0.35 about world y,
    # which is the hinge frame's z): gravity swings it down toward 0 and it comes to rest on the
    # lower limit.
    sc = _pendulum((0.2, 0.5), 0.35, 0.0)
    o = Oracle(sc, 64)
    o.step(1)
    assert _hinge_angle(o.state()) == pytest.approx(0.35, abs=0.01)
    o.step(300)
    a = _hinge_angle(o.state())
    assert a == pytest.approx(0.2, abs=1e-3)
    assert np.linalg.norm(o.state()["angvel"][:, 0]) < 1e-3


@pytest.mark.parametrize("target,limit", [(3.0, 1.0), (-3.0, -1.0)])
def test_prismatic_limit_stops_a_driven_slider(target, limit):
    q = _quat_z_to([1.0, 0.0, 0.0])
    x0 = (0.0, 0.0, 1.0)
    b = S.body(S.BOX, (0.05, 0.05, 0.05), x0, mass=1.0)
    j = S.joint(-1, 0, x0 + q, (0.0, 0.0, 0.0) + q, kp=500.0, kd=20.0, target=target, type=S.PRISMATIC,
                limits=(-1.0, 1.0))
    sc = S.single([b], [j], dt=0.01, pos_iters=4, plane_enabled=0)
    o = Oracle(sc, 64)
    xs = []
    for _ in range(300):
        o.step(1)
        xs.append(o.state()["pos"][0, 0])
    xs = np.array(xs)
    assert np.max(np.abs(xs)) <= 1.0 + 2e-3
    assert xs[-1] == pytest.approx(limit, abs=1e-3)


def test_prismatic_parent_anchor_slides_freely_along_the_rail():
    # Two free bodies (no gravity) on a prismatic joint, spinning and sliding.  The rail is a
    # line: moving the parent's anchor along the rail changes nothing physical (no drive, no
    # limit), so two descriptions differing only in where along the rail the parent anchor sits
    # must step identically; the joint's impulses act on both bodies at the child anchor.
    # Linear momentum is conserved (internal impulses) and the child stays on the rail.
    q = _quat_z_to([1.0, 0.0, 0.0])

    def scene(shift):
        a = S.body(S.BOX, (0.1, 0.05, 0.04), (0.0, 0.0, 1.0), mass=2.0, linvel=(0.1, 0.2, -0.1),
                   angvel=(0.5, -0.3, 0.8))
        b = S.body(S.BOX, (0.03, 0.03, 0.03), (0.15, 0.02, 1.01), mass=0.7, linvel=(0.4, 0.1, 0.3),
                   angvel=(0.5, -0.3, 0.8))
        j = S.joint(0, 1, (shift, 0.02, 0.01) + q, (0.0, 0.0, 0.0) + q, type=S.PRISMATIC)
        return S.single([a, b], [j], dt=0.005, pos_iters=8, plane_enabled=0, gravity=(0.0, 0.0, 0.0))

    runs = []
    for shift in (0.0, 0.125, -0.25):
        o = Oracle(scene(shift), 64)
        o.step(30)
        runs.append(o.state())
    for r in runs[1:]:
        for k in ("pos", "quat", "linvel", "angvel"):
            assert np.allclose(r[k], runs[0][k], atol=1e-9), k
    st = runs[0]
    P0 = 2.0 * np.array([0.1, 0.2, -0.1]) + 0.7 * np.array([0.4, 0.1, 0.3])
    P1 = 2.0 * st["linvel"][:, 0] + 0.7 * st["linvel"][:, 1]
    assert np.allclose(P1, np.float32(P0), atol=1e-6)
    qa = st["quat"][:, 0]
    Ra = Rotation.from_quat([qa[1], qa[2], qa[3], qa[0]])
    rel = Ra.inv().apply(st["pos"][:, 1] - st["pos"][:, 0])
    assert np.allclose(rel[1:], [0.02, 0.01], atol=1e-3)


def test_prismatic_velocity_lock_with_offset_anchor():
    # kp = 0 and a very large kd make the drive a velocity lock along the rail (gamma -> 0).  With
    # the anchor off the centre of mass the row's inverse effective mass includes the arm terms
    # (its impulse also spins the body); the drive is the last row of the block, so after a
    # single substep the anchor's velocity along the rail is zero (to gamma) although the body
    # slid at 1 m/s and now spins.  (With more substeps the rotation lock would hide a wrong
    # effective mass by converging anyway.)
    q = _quat_z_to([1.0, 0.0, 0.0])
    b = S.body(S.BOX, (0.1, 0.05, 0.04), (0.0, 0.0, 1.0), mass=1.0, linvel=(1.0, 0.0, 0.0))
    j = S.joint(-1, 0, (0.05, 0.03, 1.0) + q, (0.05, 0.03, 0.0) + q, kp=0.0, kd=1e9, type=S.PRISMATIC)
    sc = S.single([b], [j], dt=0.01, pos_iters=1, plane_enabled=0, gravity=(0.0, 0.0, 0.0))
    o = Oracle(sc, 64)
    o.step(1)
    st = o.state()
    assert abs(st["angvel"][2, 0]) > 1e-2
    qq = st["quat"][:, 0]
    R = Rotation.from_quat([qq[1], qq[2], qq[3], qq[0]])
    r = R.apply([0.05, 0.03, 0.0])
    v_anchor = st["linvel"][:, 0] + np.cross(st["angvel"][:, 0], r)
    assert abs(v_anchor[0]) < 1e-6
