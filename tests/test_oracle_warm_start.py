"""Oracle pins for the cross-step warm start (S4b, the contact cache): the paper tunes solver
position / velocity iteration counts for speed (App. E, Setup: 4 position iterations) and the
simulator it builds on warm-starts contacts across steps; the reading here caches each contact
point's final normal impulse with its position in body B's frame, and each friction patch's
tangential impulse vector and twist, and starts the next step from them for points of the same
body pair within warm_radius.

Pins: a resting box starts every step from exactly the previous step's impulses, which sum to
m g h per substep (the weight over one substep, exact once settled); a box on an incline below
the friction angle stops creeping (it creeps without the cache); the match is by position in
body B's frame: a skidding sphere (contact point fixed in the world, moving over the body) keeps
its cache below the radius and loses it above; set_state and the random reset clear the cache;
without the flag every start impulse is zero.  Each pin fails on a one-line mutation of the
matching (frame, radius test, key) or of the first-substep warm start."""
import math

import numpy as np

from oracle.oracle import Oracle
from paper_2410_00425_amd import scenes as S

G = 9.81


def box_scene(warm, gravity=(0.0, 0.0, -G), mu=0.5, radius=0.01):
    b = S.body(S.BOX, (0.05, 0.05, 0.05), (0.0, 0.0, 0.05), mass=1.0, mu=mu)
    return S.single([b], dt=0.01, pos_iters=4, warm_start=warm, warm_radius=radius, gravity=gravity,
                    plane_friction=mu)


def two_records(o, settle):
    o.step(settle)
    o.step(1, record=True)
    r1 = o.record()
    o.step(1, record=True)
    return r1, o.record()


def test_resting_box_carries_its_impulses():
    o = Oracle(box_scene(1), 32)
    r1, r2 = two_records(o, 48)
    ln, ln0 = r1["points"][:, 7], r2["points"][:, 8]
    assert len(ln) == 4 and np.array_equal(ln0, ln)
    # settled: the four normal impulses of a substep carry the weight over the substep
    h = np.float32(0.01) / np.float32(4)
    assert abs(r2["points"][:, 7].sum() - G * float(h)) < 1e-6
    # without the cache every step starts from zero
    o = Oracle(box_scene(0), 32)
    _, r2 = two_records(o, 48)
    assert np.all(r2["points"][:, 8] == 0)


def test_incline_creep_stops_with_the_cache():
    a = math.radians(20.0)   # tan 20 deg = 0.36 < mu = 0.5: the box should stick
    g = (G * math.sin(a), 0.0, -G * math.cos(a))
    creep = []
    for warm in (0, 1):
        o = Oracle(box_scene(warm, gravity=g), 64)
        o.step(100)
        x0 = o.state()["pos"][0, 0]
        o.step(100)
        creep.append(abs(o.state()["pos"][0, 0] - x0))   # m over 1 s
    assert creep[0] > 1e-3          # the cold start lets it creep by millimetres per second
    assert creep[1] < 1e-9          # the warm start holds it


def skidding_sphere(omega, radius=0.01):
    """A sphere (r = 0.05) resting on the ground, spinning about x with no linear velocity: its
    contact point stays under the centre in the world and moves over the sphere's surface by
    about r omega dt per step."""
    b = S.body(S.SPHERE, (0.05,), (0.0, 0.0, 0.05), mass=1.0, mu=0.5, angvel=(omega, 0.0, 0.0))
    return S.single([b], dt=0.01, pos_iters=4, warm_start=1, warm_radius=radius)


def test_match_is_in_body_frame_within_the_radius():
    # 10 rad/s: the contact point moves ~4.5 mm per step over the sphere (but only ~0.4 mm in the
    # world): it matches with a 1 cm radius and not with a 2 mm one
    o = Oracle(skidding_sphere(10.0), 32)
    r1, r2 = two_records(o, 0)
    assert r2["points"][0, 8] == r1["points"][0, 7] and r1["points"][0, 7] > 0
    o = Oracle(skidding_sphere(10.0, radius=0.002), 32)
    r1, r2 = two_records(o, 0)
    assert r1["points"][0, 7] > 0 and r2["points"][0, 8] == 0
    # a slow spin (0.5 rad/s: ~0.2 mm per step) matches with 2 mm
    o = Oracle(skidding_sphere(0.5, radius=0.002), 32)
    r1, r2 = two_records(o, 0)
    assert r1["points"][0, 7] > 0 and r2["points"][0, 8] == r1["points"][0, 7]


def test_cache_is_per_pair():
    # two boxes side by side on the ground: each plane pair keeps its own impulses
    b0 = S.body(S.BOX, (0.05, 0.05, 0.05), (0.0, 0.0, 0.05), mass=1.0)
    b1 = S.body(S.BOX, (0.05, 0.05, 0.05), (0.3, 0.0, 0.05), mass=3.0)
    sc = S.single([b0, b1], dt=0.01, pos_iters=4, warm_start=1, warm_radius=0.01)
    o = Oracle(sc, 32)
    r1, r2 = two_records(o, 40)
    ids1, ids2 = r1["point_ids"][:, 1], r2["point_ids"][:, 1]
    for pair in np.unique(ids2):
        ln = r1["points"][ids1 == pair, 7]
        ln0 = r2["points"][ids2 == pair, 8]
        assert np.array_equal(ln, ln0)
    sums = [r2["points"][ids2 == p, 7].sum() for p in np.unique(ids2)]
    assert abs(sums[1] / sums[0] - 3.0) < 1e-4


def test_set_state_and_random_reset_clear_the_cache():
    sc = box_scene(1)
    o = Oracle(sc, 32)
    o.step(20)
    st = o.state()
    o.set_state(st["pos"], st["quat"], st["linvel"], st["angvel"])
    o.step(1, record=True)
    assert np.all(o.record()["points"][:, 8] == 0)
    o.step(5)
    o.reset_random([0], xy_half=0.0)
    o.step(1, record=True)
    assert np.all(o.record()["points"][:, 8] == 0)
