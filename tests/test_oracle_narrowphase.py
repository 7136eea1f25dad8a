"""Oracle narrowphase and mass-property pins (CPU, float64).

Each expected value comes from geometry computed independently of the oracle: exact
sphere distances, axis-aligned overlap rectangles, support functions over random directions
(the separating-axis theorem), convex minimisation by ternary search, rotations built with
scipy, and Monte-Carlo integration for volumes and inertia.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle.oracle import box_box_sat, mass_props, narrow
from paper_2410_00425_amd import scenes as S

ID = [0, 0, 0, 1, 0, 0, 0]
DELTA = 0.01


def pose(p, R=None):
    """(px, py, pz, qw, qx, qy, qz) from a position and a scipy Rotation."""
    if R is None:
        return list(p) + [1, 0, 0, 0]
    x, y, z, w = R.as_quat()
    return list(p) + [w, x, y, z]


def rand_rot(rng):
    return Rotation.from_quat(rng.normal(size=4))


def ternary(f, lo=0.0, hi=1.0, it=90):
    """Minimum of a convex function on [lo, hi] by ternary search ((2/3)^90 ~ 1e-16)."""
    for _ in range(it):
        m1, m2 = lo + (hi - lo) / 3, hi - (hi - lo) / 3
        if f(m1) < f(m2):
            hi = m2
        else:
            lo = m1
    return f(0.5 * (lo + hi))


def seg_point_dist(a, b, x):
    return ternary(lambda t: np.linalg.norm(a + t * (b - a) - x))


def seg_seg_dist(a0, a1, b0, b1):
    """Distance of two segments: the squared distance is a convex quadratic in (s, t) on the
    unit square; grid search, then bounded quasi-Newton refinement."""
    from scipy.optimize import minimize
    g = np.linspace(0, 1, 41)
    S_, T_ = np.meshgrid(g, g, indexing="ij")
    P = a0 + S_[..., None] * (a1 - a0) - (b0 + T_[..., None] * (b1 - b0))
    d2 = np.sum(P * P, axis=-1)
    i, j = np.unravel_index(np.argmin(d2), d2.shape)

    def f(st):
        v = a0 + st[0] * (a1 - a0) - b0 - st[1] * (b1 - b0)
        return float(v @ v)

    r = minimize(f, [g[i], g[j]], method="L-BFGS-B", bounds=[(0, 1), (0, 1)],
                 options=dict(ftol=1e-30, gtol=1e-16, maxiter=500))
    return math.sqrt(min(r.fun, d2[i, j]))


def point_box_dist(x, c, R, h):
    l = R.inv().apply(x - c)
    q = np.clip(l, -h, h)
    return np.linalg.norm(l - q)


# ----------------------------------------------------------------------------- spheres
def test_sphere_sphere_exact():
    rng = np.random.default_rng(1)
    for _ in range(200):
        ca, cb = rng.uniform(-0.1, 0.1, 3), rng.uniform(-0.1, 0.1, 3)
        ra, rb = rng.uniform(0.01, 0.05, 2)
        pts, _ = narrow(S.SPHERE, [ra, 0, 0], pose(ca), S.SPHERE, [rb, 0, 0], pose(cb), DELTA)
        d = cb - ca
        s = np.linalg.norm(d) - ra - rb
        if s >= DELTA:
            assert len(pts) == 0
            continue
        assert len(pts) == 1
        n = d / np.linalg.norm(d)
        assert pts[0, 6] == pytest.approx(s, abs=1e-14)
        assert np.allclose(pts[0, 3:6], n, atol=1e-14)
        assert np.allclose(pts[0, :3], 0.5 * ((ca + ra * n) + (cb - rb * n)), atol=1e-14)


def test_sphere_sphere_coincident_uses_up_normal():
    pts, _ = narrow(S.SPHERE, [0.05, 0, 0], pose([0, 0, 0.3]), S.SPHERE, [0.02, 0, 0], pose([0, 0, 0.3]), DELTA)
    assert len(pts) == 1 and np.allclose(pts[0, 3:6], [0, 0, 1]) and pts[0, 6] == pytest.approx(-0.07)


def test_sphere_plane_and_capsule_plane():
    pts, _ = narrow(-1, None, None, S.SPHERE, [0.05, 0, 0], pose([0.1, 0.2, 0.053]), DELTA)
    assert len(pts) == 1 and pts[0, 6] == pytest.approx(0.003) and np.allclose(pts[0, 3:6], [0, 0, 1])
    assert np.allclose(pts[0, :3], [0.1, 0.2, 0.0015])
    # horizontal capsule: two end spheres at the same height
    R = Rotation.from_euler("y", 90, degrees=True)
    pts, _ = narrow(-1, None, None, S.CAPSULE, [0.03, 0.1, 0], pose([0, 0, 0.029], R), DELTA)
    assert len(pts) == 2
    assert np.allclose(pts[:, 6], -0.001) and np.allclose(sorted(pts[:, 0]), [-0.1, 0.1])
    # upright capsule: only the lower end sphere touches
    pts, _ = narrow(-1, None, None, S.CAPSULE, [0.03, 0.1, 0], pose([0, 0, 0.13]), DELTA)
    assert len(pts) == 1 and pts[0, 6] == pytest.approx(0.0)


def test_sphere_capsule_vs_ternary():
    rng = np.random.default_rng(2)
    n_hit = 0
    for _ in range(300):
        R = rand_rot(rng)
        cc = rng.uniform(-0.05, 0.05, 3)
        r, hl = rng.uniform(0.01, 0.03), rng.uniform(0.0, 0.05)
        xs, rs = rng.uniform(-0.08, 0.08, 3), rng.uniform(0.01, 0.03)
        ax = R.apply([0, 0, 1])
        d = seg_point_dist(cc - hl * ax, cc + hl * ax, xs) - r - rs
        # sphere as A (lower index) and capsule as B, and the reverse
        p1, _ = narrow(S.SPHERE, [rs, 0, 0], pose(xs), S.CAPSULE, [r, hl, 0], pose(cc, R), DELTA)
        p2, _ = narrow(S.CAPSULE, [r, hl, 0], pose(cc, R), S.SPHERE, [rs, 0, 0], pose(xs), DELTA)
        if d < DELTA - 1e-9:
            n_hit += 1
            assert len(p1) == 1 and len(p2) == 1
            assert p1[0, 6] == pytest.approx(d, abs=1e-9) and p2[0, 6] == pytest.approx(d, abs=1e-9)
            assert np.allclose(p1[0, 3:6], -p2[0, 3:6], atol=1e-12)
        elif d > DELTA + 1e-9:
            assert len(p1) == 0 and len(p2) == 0
    assert n_hit > 30


# ----------------------------------------------------------------------------- capsules
def test_capsule_capsule_vs_ternary():
    rng = np.random.default_rng(3)
    n_hit = 0
    for _ in range(300):
        Ra, Rb = rand_rot(rng), rand_rot(rng)
        ca, cb = rng.uniform(-0.05, 0.05, 3), rng.uniform(-0.05, 0.05, 3)
        ra, rb = rng.uniform(0.01, 0.03, 2)
        ha, hb = rng.uniform(0.01, 0.05, 2)
        aa, ab = Ra.apply([0, 0, 1]), Rb.apply([0, 0, 1])
        d = seg_seg_dist(ca - ha * aa, ca + ha * aa, cb - hb * ab, cb + hb * ab) - ra - rb
        pts, dec = narrow(S.CAPSULE, [ra, ha, 0], pose(ca, Ra), S.CAPSULE, [rb, hb, 0], pose(cb, Rb), DELTA)
        assert dec == 0  # random axes are never parallel
        if d < DELTA - 1e-9:
            n_hit += 1
            assert len(pts) == 1
            assert pts[0, 6] == pytest.approx(d, abs=1e-8)
        elif d > DELTA + 1e-9:
            assert len(pts) == 0
    assert n_hit > 30


def test_capsule_capsule_parallel_two_points():
    # two parallel horizontal capsules side by side, overlapping in x over [-0.02, 0.05]
    R = Rotation.from_euler("y", 90, degrees=True)
    pts, dec = narrow(S.CAPSULE, [0.02, 0.05, 0], pose([0, 0, 0], R), S.CAPSULE, [0.02, 0.05, 0],
                      pose([0.03, 0.039, 0], R), DELTA)
    assert dec == 1 and len(pts) == 2
    assert np.allclose(pts[:, 6], 0.039 - 0.04)
    assert np.allclose(sorted(pts[:, 0]), [-0.02, 0.05])
    assert np.allclose(pts[:, 3:6], [[0, 1, 0], [0, 1, 0]])


# ----------------------------------------------------------------------------- boxes
def test_box_plane_corners():
    h = np.array([0.05, 0.03, 0.02])
    pts, _ = narrow(-1, None, None, S.BOX, h, pose([0.1, 0, 0.025]), DELTA)
    assert len(pts) == 4 and np.allclose(pts[:, 6], 0.005)
    assert np.allclose(np.sort(pts[:, 0]), np.sort([0.05, 0.15, 0.05, 0.15]))
    # tilted about y: one edge down; corner heights are c_z + R (+-h)
    rng = np.random.default_rng(4)
    for _ in range(50):
        R = rand_rot(rng)
        c = np.array([0, 0, rng.uniform(0.0, 0.08)])
        pts, _ = narrow(-1, None, None, S.BOX, h, pose(c, R), DELTA)
        corners = np.array([[sx, sy, sz] for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)]) * h
        z = c[2] + R.apply(corners)[:, 2]
        want = np.sort(z[z < DELTA])
        assert len(pts) == min(len(want), 4)
        if len(want) <= 4:
            assert np.allclose(np.sort(pts[:, 6]), want, atol=1e-12)
        else:
            assert pts[:, 6].min() == pytest.approx(want[0], abs=1e-12)  # the deepest is kept


def test_manifold_reduction_keeps_deepest_and_spread():
    # a tiny box whose 8 corners all lie within the contact offset: reduced to 4 points
    pts, _ = narrow(-1, None, None, S.BOX, [0.002, 0.002, 0.002], pose([0, 0, 0.0021],
                    Rotation.from_euler("xyz", [0.2, 0.1, 0.3])), DELTA)
    assert len(pts) == 4
    full = np.array([[sx, sy, sz] for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)]) * 0.002
    z = 0.0021 + Rotation.from_euler("xyz", [0.2, 0.1, 0.3]).apply(full)[:, 2]
    assert pts[:, 6].min() == pytest.approx(z.min())


def test_box_box_axis_aligned_overlap_rectangle():
    # B resting on A with overlap 0.004 m along z and offset in x, y: the contact points are the
    # corners of the overlap rectangle, each at separation -0.004, normal +z.
    ha, hb = np.array([0.1, 0.1, 0.05]), np.array([0.04, 0.03, 0.02])
    cb = np.array([0.08, -0.09, 0.05 + 0.02 - 0.004])
    pts, dec = narrow(S.BOX, ha, pose([0, 0, 0]), S.BOX, hb, pose(cb), DELTA)
    assert dec in (2, 5)  # a z face axis
    assert len(pts) == 4
    assert np.allclose(pts[:, 6], -0.004)
    assert np.allclose(pts[:, 3:6], [0, 0, 1])
    xs = sorted(set(np.round(pts[:, 0], 9)))
    ys = sorted(set(np.round(pts[:, 1], 9)))
    assert np.allclose(xs, [0.04, 0.1]) and np.allclose(ys, [-0.1, -0.06])



def test_box_box_sat_vs_random_directions():
    # Overlapping boxes: the penetration depth is attained on one of the 15 SAT axes, so no
    # direction shows a larger gap than the best SAT axis; the best of 10^4 random directions,
    # refined locally on the sphere, comes within 1e-6 of it.
    from scipy.optimize import minimize
    rng = np.random.default_rng(5)
    for _ in range(20):
        Ra, Rb = rand_rot(rng), rand_rot(rng)
        ha, hb = rng.uniform(0.02, 0.06, 3), rng.uniform(0.02, 0.06, 3)
        cb = rng.uniform(-0.03, 0.03, 3)
        sep, valid = box_box_sat(ha, pose([0, 0, 0], Ra), hb, pose(cb, Rb))
        smax = sep[valid].max()
        if smax >= 0:
            continue
        L = rng.normal(size=(10000, 3))
        L /= np.linalg.norm(L, axis=1, keepdims=True)
        Ma, Mb = Ra.as_matrix(), Rb.as_matrix()
        ea = np.abs(L @ Ma) @ ha
        eb = np.abs(L @ Mb) @ hb
        gap = np.abs(L @ cb) - ea - eb
        assert gap.max() <= smax + 1e-9

        def neg_gap(ang):
            u = np.array([math.sin(ang[0]) * math.cos(ang[1]), math.sin(ang[0]) * math.sin(ang[1]), math.cos(ang[0])])
            return -(abs(u @ cb) - np.abs(u @ Ma) @ ha - np.abs(u @ Mb) @ hb)

        best = -1e9
        for k in np.argsort(-gap)[:5]:
            u = L[k]
            a0 = [math.acos(np.clip(u[2], -1, 1)), math.atan2(u[1], u[0])]
            r = minimize(neg_gap, a0, method="Nelder-Mead", options=dict(xatol=1e-12, fatol=1e-14, maxiter=4000))
            best = max(best, -r.fun)
        assert best <= smax + 1e-9
        assert smax - best < 1e-6


def test_box_box_face_contact_rotated_about_normal():
    # B sits on A's top face, rotated about z by 30 degrees: face contact, 4 points at -0.002
    R = Rotation.from_euler("z", 30, degrees=True)
    hb = np.array([0.02, 0.02, 0.02])
    pts, dec = narrow(S.BOX, [0.2, 0.2, 0.05], pose([0, 0, 0]), S.BOX, hb, pose([0.01, 0.02, 0.068], R), DELTA)
    assert len(pts) == 4 and np.allclose(pts[:, 6], -0.002) and np.allclose(pts[:, 3:6], [0, 0, 1])
    corners = np.array([[sx, sy, -1] for sy in (-1, 1) for sx in (-1, 1)]) * hb
    want = np.array([0.01, 0.02, 0.068]) + R.apply(corners)
    got = pts[:, :3] - np.array([0, 0, 0.001])  # midpoints sit half the separation above B's face
    for w in want:
        assert np.min(np.linalg.norm(got - w, axis=1)) < 1e-12


def test_box_box_edge_edge():
    # two boxes touching edge to edge (crossed edges): one point at the edge-edge closest points
    Ra = Rotation.from_euler("x", 45, degrees=True)
    Rb = Rotation.from_euler("y", 45, degrees=True)
    h = np.array([0.05, 0.05, 0.05])
    gap = 0.003
    zb = 2 * 0.05 * math.sqrt(2) + gap
    pts, dec = narrow(S.BOX, h, pose([0, 0, 0], Ra), S.BOX, h, pose([0, 0, zb], Rb), DELTA)
    assert dec >= 6 and len(pts) == 1
    assert pts[0, 6] == pytest.approx(gap, abs=1e-12)
    assert np.allclose(pts[0, 3:6], [0, 0, 1], atol=1e-12)
    assert np.allclose(pts[0, :3], [0, 0, zb / 2], atol=1e-12)


def test_sphere_box_outside_and_inside():
    rng = np.random.default_rng(6)
    n_out = 0
    for _ in range(300):
        R = rand_rot(rng)
        c = rng.uniform(-0.02, 0.02, 3)
        h = rng.uniform(0.01, 0.04, 3)
        x, r = rng.uniform(-0.07, 0.07, 3), rng.uniform(0.005, 0.02)
        pts, dec = narrow(S.BOX, h, pose(c, R), S.SPHERE, [r, 0, 0], pose(x), DELTA)
        d = point_box_dist(x, c, R, h)
        if d > 0:
            want = d - r
            if want < DELTA - 1e-9:
                n_out += 1
                assert dec == 0 and len(pts) == 1 and pts[0, 6] == pytest.approx(want, abs=1e-12)
            elif want > DELTA + 1e-9:
                assert len(pts) == 0
        else:
            # centre inside: least-penetration face
            l = R.inv().apply(x - c)
            depth = h - np.abs(l)
            i = int(np.argmin(depth))
            assert dec == 1 + i and pts[0, 6] == pytest.approx(-depth[i] - r, abs=1e-12)
    assert n_out > 20
    # argument order only flips the normal
    p1, _ = narrow(S.BOX, [0.05, 0.05, 0.05], pose([0, 0, 0]), S.SPHERE, [0.02, 0, 0], pose([0.06, 0.01, 0]), DELTA)
    p2, _ = narrow(S.SPHERE, [0.02, 0, 0], pose([0.06, 0.01, 0]), S.BOX, [0.05, 0.05, 0.05], pose([0, 0, 0]), DELTA)
    assert np.allclose(p1[:, :3], p2[:, :3]) and np.allclose(p1[:, 3:6], -p2[:, 3:6]) and np.allclose(p1[:, 6], p2[:, 6])


def test_capsule_box_face_case():
    # horizontal capsule above the box top face, tilted slightly: two clipped end points whose
    # separations are the end-sphere heights above the face
    R = Rotation.from_euler("y", 85, degrees=True)
    hl, r = 0.04, 0.01
    c = np.array([0.0, 0.01, 0.05 + r + 0.002])
    pts, dec = narrow(S.BOX, [0.1, 0.1, 0.05], pose([0, 0, 0]), S.CAPSULE, [r, hl, 0], pose(c, R), DELTA)
    assert dec == 2 and len(pts) == 2
    ax = R.apply([0, 0, 1])
    ends = np.array([c - hl * ax, c + hl * ax])
    want = np.sort(ends[:, 2] - 0.05 - r)
    assert np.allclose(np.sort(pts[:, 6]), want, atol=1e-12)
    assert np.allclose(pts[:, 3:6], [0, 0, 1])


def test_capsule_box_distance_vs_ternary():
    # Separated configurations: the smallest reported separation equals the segment-to-box
    # distance minus the radius when the capsule hovers over a face (clipped face case).
    rng = np.random.default_rng(7)
    n = 0
    for _ in range(200):
        h = rng.uniform(0.03, 0.06, 3)
        R = rand_rot(rng)
        r, hl = rng.uniform(0.005, 0.015), rng.uniform(0.005, 0.02)
        # capsule centre above the top face, inside its footprint
        c = np.array([rng.uniform(-0.5, 0.5) * h[0], rng.uniform(-0.5, 0.5) * h[1], h[2] + hl + r + rng.uniform(0, 0.008)])
        ax = R.apply([0, 0, 1])
        a0, a1 = c - hl * ax, c + hl * ax
        if max(abs(a0[0]), abs(a1[0])) > h[0] or max(abs(a0[1]), abs(a1[1])) > h[1]:
            continue
        d = ternary(lambda t: point_box_dist(a0 + t * (a1 - a0), np.zeros(3), Rotation.identity(), h)) - r
        pts, dec = narrow(S.BOX, h, pose([0, 0, 0]), S.CAPSULE, [r, hl, 0], pose(c, R), DELTA)
        if d < DELTA - 1e-7:
            n += 1
            assert len(pts) >= 1
            assert pts[:, 6].min() == pytest.approx(d, abs=1e-7)
    assert n > 20


# ----------------------------------------------------------------------------- mass properties
@pytest.mark.parametrize("shape,dims", [(S.BOX, [0.05, 0.03, 0.02]), (S.SPHERE, [0.04, 0, 0]),
                                        (S.CAPSULE, [0.02, 0.05, 0]), (S.CAPSULE, [0.04, 0.01, 0])])
def test_mass_properties_monte_carlo(shape, dims):
    rng = np.random.default_rng(8)
    mass = 2.0
    vol, inertia = mass_props(shape, dims, mass)
    ext = np.array([dims[0], dims[0], dims[0]]) if shape == S.SPHERE else (
        np.array([dims[0], dims[0], dims[0] + dims[1]]) if shape == S.CAPSULE else np.array(dims))
    N = 400000
    x = rng.uniform(-1, 1, size=(N, 3)) * ext
    if shape == S.BOX:
        inside = np.ones(N, bool)
    elif shape == S.SPHERE:
        inside = np.linalg.norm(x, axis=1) <= dims[0]
    else:
        zc = np.clip(x[:, 2], -dims[1], dims[1])
        inside = np.linalg.norm(x - np.stack([0 * zc, 0 * zc, zc], 1), axis=1) <= dims[0]
    box_vol = np.prod(2 * ext)
    f = inside.mean()
    v_mc = f * box_vol
    sd = math.sqrt(f * (1 - f) / N) * box_vol
    assert abs(vol - v_mc) <= 4 * sd + 1e-12
    xi = x[inside]
    rho_m = mass / len(xi)
    I_mc = np.array([np.sum(xi[:, 1] ** 2 + xi[:, 2] ** 2), np.sum(xi[:, 0] ** 2 + xi[:, 2] ** 2),
                     np.sum(xi[:, 0] ** 2 + xi[:, 1] ** 2)]) * rho_m
    for k in range(3):
        q = np.array([xi[:, 1] ** 2 + xi[:, 2] ** 2, xi[:, 0] ** 2 + xi[:, 2] ** 2, xi[:, 0] ** 2 + xi[:, 1] ** 2])[k]
        sd_i = q.std() / math.sqrt(len(xi)) * mass
        assert abs(inertia[k] - I_mc[k]) <= 4 * sd_i
