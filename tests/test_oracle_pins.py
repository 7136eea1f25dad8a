"""Further oracle pins (CPU): the parts whose earlier tests accepted a plausible mistake.

Each expectation is derived by hand from geometry or mechanics, or computed independently of the
oracle's code (support functions, convex minimisation, geometric series):
  * the <= 4 point manifold reduction on a hand-built point set whose picks are unique under
    each criterion (deepest, farthest, largest triangle, largest added area) and on ties;
  * the face / edge preference of the separating-axis choice at its tolerance, just inside and
    just outside (box-box: B face over A face, face over edge);
  * the capsule-box edge-axis branch and the boundary-edge fallback when the capsule lies
    outside the reference face's prism, against exact segment-edge distances;
  * torsional friction: a flat box spinning on the ground decelerates at mu r_t m g / I_zz
    (the model's twist limit, r_t the mean point distance to the patch centroid);
  * PGS (one substep, K iterations): Coulomb sliding mu g and exact free fall with S = 1;
  * linear and angular damping: the per-substep geometric series v <- (v + h g) / (1 + h c).
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle.oracle import Oracle, narrow, reduce4
from paper_2410_00425_amd import scenes as S

G32 = float(np.float32(9.81))
DELTA = 0.01


def pose(p, R=None):
    if R is None:
        return list(p) + [1, 0, 0, 0]
    x, y, z, w = R.as_quat()
    return list(p) + [w, x, y, z]


# ----------------------------------------------------------------------------- reduce4
def test_reduce4_hand_built_selection():
    # Points on the plane z = 0.  By hand:
    #   deepest: p0 (s = -0.002, the only negative separation);
    #   farthest from p0: p1 at 0.100 (p3 0.078, p5 0.085, p6 0.092);
    #   largest triangle with p0 p1 (base 0.1 along x): |y| largest -> p3 (y = -0.06);
    #   largest area added outside p0 p1 p3: p2 on the far side of p0 p1 (0.1 * 0.04 / 2),
    #   more than p5 (0.1 * 0.03 / 2), p6 (0.1 * 0.035 / 2 = 0.00175 < 0.002) or p4.
    P = [[0.0, 0.0, 0], [0.1, 0.0, 0], [0.05, 0.04, 0], [0.05, -0.06, 0], [0.02, 0.01, 0], [0.08, 0.03, 0],
         [0.06, 0.035, 0], [0.03, -0.01, 0]]
    s = [-0.002, 0, 0, 0, 0, 0, 0, 0]
    picked, n = reduce4(P, s)
    assert n == 4
    assert picked == [0, 1, 3, 2]


def test_reduce4_each_criterion_is_the_stated_one():
    # Moving one point changes exactly the pick its criterion governs.
    P = [[0.0, 0.0, 0], [0.1, 0.0, 0], [0.05, 0.04, 0], [0.05, -0.06, 0], [0.02, 0.01, 0], [0.08, 0.03, 0]]
    s = [-0.002, 0, 0, 0, 0, 0]
    assert reduce4(P, s)[0] == [0, 1, 3, 2]
    # a deeper point elsewhere becomes the first pick
    s2 = list(s)
    s2[4] = -0.003
    assert reduce4(P, s2)[0][0] == 4
    # a point farther from p0 than p1 becomes the second pick
    P2 = [list(p) for p in P]
    P2[5] = [0.11, 0.03, 0]
    assert reduce4(P2, s)[0][:2] == [0, 5]
    # a point far on the positive-y side becomes the triangle pick, and then the added-area pick
    # moves to the other side (p3 at y = -0.06)
    P3 = [list(p) for p in P]
    P3[2] = [0.05, 0.08, 0]
    assert reduce4(P3, s)[0] == [0, 1, 2, 3]


def test_reduce4_ties_take_the_lowest_index():
    # four corners of a square and its centre, all at the same depth: the deepest is p0 (lowest
    # index); the farthest from p0 is its diagonal opposite p2; the largest triangle with the
    # diagonal is tied between p1 and p3 -> p1; the added area is then p3's (p4 adds none).
    P = [[0, 0, 0], [0.1, 0, 0], [0.1, 0.1, 0], [0, 0.1, 0], [0.05, 0.05, 0]]
    s = [-0.001] * 5
    picked, n = reduce4(P, s)
    assert n == 4 and picked == [0, 2, 1, 3]
    # the same square listed from another corner: the picks follow the indices
    P = [P[2], P[3], P[0], P[1], P[4]]
    assert reduce4(P, s)[0] == [0, 2, 1, 3]


def test_reduce4_keeps_at_most_four_in_list_order():
    rng = np.random.default_rng(11)
    for n in range(1, 9):
        P = rng.uniform(-0.05, 0.05, (n, 3))
        P[:, 2] = 0
        s = rng.uniform(-0.005, 0.005, n)
        picked, m = reduce4(P, s)
        assert m == min(n, 4)
        if n <= 4:
            assert picked == [-1] * 4
        else:
            assert len(set(picked)) == 4 and picked[0] == int(np.argmin(s))


# ----------------------------------------------------------------------------- SAT preferences
def _box_axes(R):
    return R.as_matrix().T  # rows = the box's axes in the world


def _sep(L, d, ha, Ra, hb, Rb):
    """Gap of two boxes along unit axis L: |d . L| minus both support half-widths."""
    ea = sum(h * abs(a @ L) for h, a in zip(ha, _box_axes(Ra)))
    eb = sum(h * abs(a @ L) for h, a in zip(hb, _box_axes(Rb)))
    return abs(d @ L) - ea - eb


def _face_and_edge_seps(d, ha, Ra, hb, Rb):
    A, B = _box_axes(Ra), _box_axes(Rb)
    fa = [_sep(A[i], d, ha, Ra, hb, Rb) for i in range(3)]
    fb = [_sep(B[i], d, ha, Ra, hb, Rb) for i in range(3)]
    fe = []
    for i in range(3):
        for j in range(3):
            c = np.cross(A[i], B[j])
            l = np.linalg.norm(c)
            fe.append(_sep(c / l, d, ha, Ra, hb, Rb) if l >= 1e-6 else -1e30)
    return fa, fb, fe


def _tol(s, hmin):
    # the documented tie tolerance: 0.05 |s| + 0.01 x the smallest half-extent
    return 0.05 * abs(s) + 0.01 * hmin


@pytest.mark.parametrize("sign,want", [(-1, "B"), (+1, "A")])
def test_box_box_prefers_b_face_within_tolerance(sign, want):
    # A flat box A under a cube B tilted about x by theta: A's z face gap exceeds B's by
    # ~0.17 theta.  Bisect theta to where that excess equals the tolerance, then step 1e-7 rad
    # to either side: below, B's face (axis 5) is kept; above, A's face (axis 2) wins.
    ha, hb = np.array([0.2, 0.2, 0.05]), np.array([0.03, 0.03, 0.03])
    Ra = Rotation.identity()
    hmin = 0.03

    def excess(th):
        Rb = Rotation.from_euler("x", th)
        dz = 0.05 + 0.03 * (abs(math.sin(th)) + abs(math.cos(th))) - 0.002   # A's z gap = -0.002
        d = np.array([0.0, 0.0, dz])
        fa, fb, _ = _face_and_edge_seps(d, ha, Ra, hb, Rb)
        return max(fa) - (max(fb) + _tol(max(fb), hmin)), d, Rb

    lo, hi = 1e-5, 0.05
    assert excess(lo)[0] < 0 < excess(hi)[0]
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if excess(mid)[0] < 0:
            lo = mid
        else:
            hi = mid
    th = 0.5 * (lo + hi) + sign * 1e-7
    ex, d, Rb = excess(th)
    assert (ex < 0) == (sign < 0)
    _, dec = narrow(S.BOX, ha, pose([0, 0, 0]), S.BOX, hb, pose(d, Rb), DELTA)
    assert dec == (5 if want == "B" else 2)


@pytest.mark.parametrize("sign", [-1, +1])
def test_box_box_prefers_face_over_edge_within_tolerance(sign):
    # A rotated 45 degrees about x (a ridge along x on top), B above it rotated by phi about y.
    # At phi = 0 B's bottom face lies flat on the ridge (face contact); as phi grows the
    # edge-edge axis gap exceeds the best face gap.  At the tolerance crossing +- 1e-7 rad the
    # choice flips from a face axis (< 6) to an edge axis (>= 6).
    ha, hb = np.array([0.05, 0.05, 0.05]), np.array([0.05, 0.05, 0.05])
    Ra = Rotation.from_euler("x", 45, degrees=True)
    hmin = 0.05
    zr = 0.05 * math.sqrt(2)

    def excess(phi):
        Rb = Rotation.from_euler("y", phi)
        dz = zr + 0.05 * (abs(math.sin(phi)) + abs(math.cos(phi))) - 0.001
        d = np.array([0.0, 0.0, dz])
        fa, fb, fe = _face_and_edge_seps(d, ha, Ra, hb, Rb)
        best = max(fb)
        if max(fa) > best + _tol(best, hmin):
            best = max(fa)
        return max(fe) - (best + _tol(best, hmin)), d, Rb

    lo, hi = 1e-4, math.radians(45)
    assert excess(lo)[0] < 0 < excess(hi)[0]
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if excess(mid)[0] < 0:
            lo = mid
        else:
            hi = mid
    phi = 0.5 * (lo + hi) + sign * 1e-7
    ex, d, Rb = excess(phi)
    _, dec = narrow(S.BOX, ha, pose([0, 0, 0], Ra), S.BOX, hb, pose(d, Rb), DELTA)
    if sign < 0:
        assert ex < 0 and dec < 6
    else:
        assert ex > 0 and dec >= 6


# ----------------------------------------------------------------------------- capsule-box
def _rigid(rng):
    return Rotation.from_quat(rng.normal(size=4)), rng.uniform(-0.2, 0.2, 3)


@pytest.mark.parametrize("g1,g2", [(0.004, 0.006), (0.006, 0.004), (0.001, 0.008), (0.0075, 0.0005)])
def test_capsule_box_outside_face_prism_uses_boundary_edge(g1, g2):
    # A horizontal capsule parallel to the box's top +y edge, offset outward by g1 (y) and
    # upward by g2 (z): its axis lies outside the prism of the best face, so the clipped segment
    # is empty and the contact comes from the nearest boundary edge of that face, the +y top
    # edge: separation sqrt(g1^2 + g2^2) - r exactly, normal along (0, g1, g2).  The best face
    # is z (decision 6 + 2) when g2 > g1, else y (6 + 1).  A rigid motion of the whole
    # configuration changes neither the decision nor the separation.
    h = np.array([0.05, 0.04, 0.03])
    r, hl = 0.005, 0.02
    Rc = Rotation.from_euler("y", 90, degrees=True)      # capsule axis along x
    c = np.array([0.01, h[1] + g1, h[2] + g2])
    want = math.hypot(g1, g2) - r
    nwant = np.array([0.0, g1, g2]) / math.hypot(g1, g2)
    pts, dec = narrow(S.BOX, h, pose([0, 0, 0]), S.CAPSULE, [r, hl, 0], pose(c, Rc), DELTA)
    assert dec == (8 if g2 > g1 else 7)
    assert len(pts) == 1
    assert pts[0, 6] == pytest.approx(want, abs=1e-12)
    assert np.allclose(pts[0, 3:6], nwant, atol=1e-12)
    rng = np.random.default_rng(21)
    for _ in range(5):
        R, t = _rigid(rng)
        p2, d2 = narrow(S.BOX, h, pose(t, R), S.CAPSULE, [r, hl, 0], pose(R.apply(c) + t, R * Rc), DELTA)
        assert d2 == dec and len(p2) == 1
        assert p2[0, 6] == pytest.approx(want, abs=1e-12)
        assert np.allclose(p2[0, 3:6], R.apply(nwant), atol=1e-12)


@pytest.mark.parametrize("gap", [0.001, 0.003, 0.008])
def test_capsule_box_edge_axis_branch(gap):
    # A capsule crossing over the box's top +y edge (an edge along x), its axis along
    # (0, 1, -1)/sqrt(2) and its centre at distance t = r + gap from the edge along
    # (0, 1, 1)/sqrt(2).  The axis (capsule dir) x (box x) = (0, 1, 1)/sqrt(2) gives the gap
    # exactly (the capsule's extent along it is zero); the face axes give only
    # (t - hl)/sqrt(2) - r, so the edge axis wins (decision 3 + 0) and the one point's separation
    # is the true segment-edge distance minus r.
    h = np.array([0.05, 0.04, 0.03])
    r, hl = 0.005, 0.01
    u = np.array([0.0, 1.0, -1.0]) / math.sqrt(2)
    L = np.array([0.0, 1.0, 1.0]) / math.sqrt(2)
    Rc = Rotation.align_vectors([u], [[0, 0, 1]])[0]
    assert np.allclose(Rc.apply([0, 0, 1]), u)
    c = np.array([0.01, h[1], h[2]]) + (r + gap) * L
    pts, dec = narrow(S.BOX, h, pose([0, 0, 0]), S.CAPSULE, [r, hl, 0], pose(c, Rc), DELTA)
    assert dec == 3
    assert len(pts) == (1 if gap < DELTA else 0)
    if len(pts):
        assert pts[0, 6] == pytest.approx(gap, abs=1e-12)
        assert np.allclose(pts[0, 3:6], L, atol=1e-12)
        # the point is the midpoint of the edge point (0.01, hy, hz) and the capsule surface point
        mid = np.array([0.01, h[1], h[2]]) + 0.5 * gap * L
        assert np.allclose(pts[0, :3], mid, atol=1e-12)
    rng = np.random.default_rng(22)
    for _ in range(5):
        R, t = _rigid(rng)
        p2, d2 = narrow(S.BOX, h, pose(t, R), S.CAPSULE, [r, hl, 0], pose(R.apply(c) + t, R * Rc), DELTA)
        assert d2 == 3 and len(p2) == len(pts)
        if len(pts):
            assert p2[0, 6] == pytest.approx(gap, abs=1e-12)


# ----------------------------------------------------------------------------- torsional friction
@pytest.mark.parametrize("prec", [64, 32])
def test_spinning_flat_box_torsional_deceleration(prec):
    # A flat box (half-extents a = b = 0.2, c = 0.02) resting on the ground and spinning about z
    # at w0 = 4 rad/s.  Its 4 bottom corners form one patch with centroid under the centre and
    # mean point radius r_t = sqrt(a^2 + b^2); the centroid does not slide, so only the twist
    # row acts: |tau| = mu r_t m g, I_zz = m (a^2 + b^2) / 3, deceleration
    # alpha = 3 mu g / sqrt(a^2 + b^2) = 10.405 rad/s^2 at mu = 0.1; stop after w0 / alpha = 0.384 s.
    a, c, mu, w0 = 0.2, 0.02, 0.1, 4.0
    sc = S.single([S.body(S.BOX, (a, a, c), (0, 0, c), mass=1.0, mu=mu, angvel=(0, 0, w0))],
                  dt=0.01, pos_iters=4, plane_friction=mu)
    o = Oracle(sc, prec)
    w, xy = [], []
    for _ in range(80):
        o.step(1)
        st = o.state()
        w.append(st["angvel"][2, 0])
        xy.append(np.hypot(st["pos"][0, 0], st["pos"][1, 0]))
    w = np.array(w)
    alpha = 3 * mu * G32 / math.hypot(a, a)
    t = 0.01 * np.arange(1, len(w) + 1)
    sl = slice(2, 30)
    slope = np.polyfit(t[sl], w[sl], 1)[0]
    assert -slope == pytest.approx(alpha, rel=0.02)
    stop = int(np.argmax(w < 1e-3))
    assert stop > 0 and 0.01 * (stop + 1) == pytest.approx(w0 / alpha, abs=0.015)
    assert np.all(w[stop:] > -1e-3)          # friction stops the spin, never reverses it
    assert max(xy) < 1e-3                    # the centroid does not wander


# ----------------------------------------------------------------------------- PGS
@pytest.mark.parametrize("iters", [4, 8])
def test_pgs_sliding_box_coulomb(iters):
    # PGS runs one substep of `iters` iterations; Coulomb sliding still decelerates at mu g.
    mu, v0 = 0.5, 2.0
    sc = S.single([S.body(S.BOX, (0.05, 0.05, 0.05), (0, 0, 0.05), mass=1.0, mu=mu, linvel=(v0, 0, 0))],
                  dt=0.01, pos_iters=iters, solver=S.PGS, plane_friction=mu)
    o = Oracle(sc, 64)
    v, x = [], []
    for _ in range(70):
        o.step(1)
        st = o.state()
        v.append(st["linvel"][0, 0])
        x.append(st["pos"][0, 0])
    v, x = np.array(v), np.array(x)
    a = mu * 9.81
    t = 0.01 * np.arange(1, 71)
    slope = np.polyfit(t[5:30], v[5:30], 1)[0]
    assert -slope == pytest.approx(a, rel=0.02)
    # one substep per step: x advances by dt v_k with v_k = v0 - k a dt (k = 1 .. K while
    # positive), the discrete sum dt (K v0 - a dt K (K + 1) / 2)
    dt = 0.01
    K = int(v0 / (a * dt))
    assert x[-1] == pytest.approx(dt * (K * v0 - a * dt * K * (K + 1) / 2), rel=2e-3)
    assert abs(x[-1] - x[-21]) < 1e-4


@pytest.mark.parametrize("prec,tol", [(64, 1e-12), (32, 1e-6)])
def test_pgs_free_fall_exact_one_substep(prec, tol):
    # PGS is one substep per step: z = z0 - g dt^2 n (n + 1) / 2, v = -g n dt, whatever K.
    dt, z0, n = 0.01, 10.0, 13
    sc = S.single([S.body(S.SPHERE, (0.1,), (0, 0, z0), mass=1.0)], dt=dt, pos_iters=6, solver=S.PGS,
                  plane_enabled=0)
    o = Oracle(sc, prec)
    o.step(n)
    st = o.state()
    dt32 = float(np.float32(dt))
    assert abs(st["pos"][2, 0] - (z0 - G32 * dt32 ** 2 * n * (n + 1) / 2)) <= tol * z0
    assert abs(st["linvel"][2, 0] + G32 * n * dt32) <= tol * 10


# ----------------------------------------------------------------------------- damping
@pytest.mark.parametrize("prec,tol", [(64, 1e-12), (32, 2e-6)])
def test_damping_geometric_series(prec, tol):
    # Free flight with damping c_l, c_a: every substep v <- (v + h g) r_l, w <- w r_a with
    # r = 1 / (1 + h c).  After N substeps v_N = r^N v0 + h g r (1 - r^N) / (1 - r) and
    # w_N = r_a^N w0 (per component; no contacts, no gyroscopic term).
    dt, sub, n = 0.01, 4, 30
    cl, ca = 0.7, 1.3
    v0, w0 = np.array([1.0, -0.5, 2.0]), np.array([3.0, -2.0, 1.5])
    sc = S.single([S.body(S.SPHERE, (0.05,), (0, 0, 5.0), mass=1.0, linvel=tuple(v0), angvel=tuple(w0))],
                  dt=dt, pos_iters=sub, plane_enabled=0, lin_damping=cl, ang_damping=ca)
    o = Oracle(sc, prec)
    o.step(n)
    st = o.state()
    f = lambda x: float(np.float32(x))   # the records hold float32 inputs
    h = f(dt) / sub
    rl, ra = 1 / (1 + h * f(cl)), 1 / (1 + h * f(ca))
    N = n * sub
    g = np.array([0.0, 0.0, -G32])
    v_want = rl ** N * np.array([f(x) for x in v0]) + h * g * rl * (1 - rl ** N) / (1 - rl)
    w_want = ra ** N * np.array([f(x) for x in w0])
    assert np.allclose(st["linvel"][:, 0], v_want, rtol=tol, atol=tol)
    assert np.allclose(st["angvel"][:, 0], w_want, rtol=tol, atol=tol)
