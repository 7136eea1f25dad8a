"""Seeded synthetic scene generators (inputs only; no step arithmetic).

Every random number is drawn from a counter-based Philox4x32-10 stream (Salmon et al., SC'11,
"Parallel random numbers: as easy as 1, 2, 3") keyed by the base seed and addressed by
(env id, purpose, draw block), so a scene never depends on batch size, packing or env order.
The paper motivates this with explicit per-parallel-env seeding so that runs can be replayed
with a different number of envs (Sec. III-G, demonstration datasets).

Workloads (all synthetic; the paper's assets are YCB / PartNet-Mobility meshes, which stand in
here as primitive shapes of the same scale):
  * drop_boxes   -- one 0.1 m, 1 kg box per env above the ground, uniform random orientation.
  * arm_cube     -- a fixed-base 7-link capsule arm with PD-driven revolute joints and a cube.
  * tray         -- a static tray and 20 random boxes / spheres / capsules dropped into it.
  * hetero       -- per-env body counts from a truncated geometric law on 1..64, with or
                    without the 7-link arm; optionally padded to 64 bodies with far static pads.
  * cartpole     -- the paper's simulation-only benchmark workload (prismatic cart, revolute pole).
  * compound_tray -- the tray with 12 bodies, half of them compound bodies (dumbbells, benches,
                    jacks: rigid unions of up to 4 primitives, the stand-in for the paper's
                    convex-decomposed meshes, App. A, Room Scale Environments).
The descriptor records match ``ms_body_desc`` / ``ms_joint_desc`` / ``ms_sim_params``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------- record layouts
BODY_DTYPE = np.dtype([
    ("shape", "<i4"), ("flags", "<i4"), ("dims", "<f4", 3), ("mass", "<f4"), ("density", "<f4"),
    ("friction", "<f4"), ("restitution", "<f4"), ("pos", "<f4", 3), ("quat", "<f4", 4),
    ("linvel", "<f4", 3), ("angvel", "<f4", 3),
])
JOINT_DTYPE = np.dtype([
    ("parent", "<i4"), ("child", "<i4"), ("frame_parent", "<f4", 7), ("frame_child", "<f4", 7),
    ("kp", "<f4"), ("kd", "<f4"), ("target", "<f4"), ("type", "<i4"), ("limited", "<i4"),
    ("lower", "<f4"), ("upper", "<f4"),
])
# A compound body's parts (ms_compound_desc): up to 4 primitives with poses in the body frame.
COMPOUND_DTYPE = np.dtype([
    ("n_children", "<i4"), ("shape", "<i4", 4), ("dims", "<f4", (4, 3)), ("pose", "<f4", (4, 7)),
])
assert COMPOUND_DTYPE.itemsize == 180
PARAMS_DTYPE = np.dtype([
    ("dt", "<f4"), ("pos_iters", "<i4"), ("vel_iters", "<i4"), ("solver", "<i4"),
    ("gravity", "<f4", 3), ("plane_z", "<f4"), ("plane_enabled", "<i4"), ("plane_friction", "<f4"),
    ("plane_restitution", "<f4"), ("contact_offset", "<f4"), ("baumgarte", "<f4"),
    ("max_depen_vel", "<f4"), ("joint_baumgarte", "<f4"), ("bounce_threshold", "<f4"),
    ("lin_damping", "<f4"), ("ang_damping", "<f4"), ("max_contacts_per_env", "<i4"),
    ("debug_export", "<i4"), ("joint_iters", "<i4"), ("max_manifolds_per_env", "<i4"),
    ("warm_start", "<i4"), ("warm_radius", "<f4"),
])
assert BODY_DTYPE.itemsize == 88 and JOINT_DTYPE.itemsize == 92 and PARAMS_DTYPE.itemsize == 96

SPHERE, CAPSULE, BOX, COMPOUND = 0, 1, 2, 3
REVOLUTE, PRISMATIC = 0, 1
STATIC = 1
TGS, PGS = 0, 1


def make_params(**kw) -> np.ndarray:
    """A sim-parameter record with the documented defaults, overridden by keyword."""
    p = np.zeros((), dtype=PARAMS_DTYPE)
    defaults = dict(dt=0.01, pos_iters=4, vel_iters=0, solver=TGS, gravity=(0.0, 0.0, -9.81),
                    plane_z=0.0, plane_enabled=1, plane_friction=0.5, plane_restitution=0.0,
                    contact_offset=0.01, baumgarte=0.2, max_depen_vel=1.0, joint_baumgarte=0.2,
                    bounce_threshold=1.0, lin_damping=0.0, ang_damping=0.0,
                    max_contacts_per_env=0, debug_export=0, joint_iters=4,
                    max_manifolds_per_env=0, warm_start=0, warm_radius=0.01)
    defaults.update(kw)
    for k, v in defaults.items():
        p[k] = v
    return p


@dataclass
class Scene:
    """A batch of envs in compressed form plus its step parameters."""
    name: str
    params: np.ndarray
    body_off: np.ndarray
    bodies: np.ndarray
    joint_off: np.ndarray
    joints: np.ndarray
    meta: dict = field(default_factory=dict)
    compounds: np.ndarray = field(default_factory=lambda: np.zeros(0, COMPOUND_DTYPE))

    @property
    def n_envs(self) -> int:
        return int(self.body_off.shape[0] - 1)

    @property
    def n_bodies(self) -> int:
        return int(self.body_off[-1])

    @property
    def n_joints(self) -> int:
        return int(self.joint_off[-1])

    def initial_state(self):
        """Full-batch SoA arrays pos[3][B], quat[4][B], linvel[3][B], angvel[3][B] (float32)."""
        b = self.bodies
        return (np.ascontiguousarray(b["pos"].T), np.ascontiguousarray(b["quat"].T),
                np.ascontiguousarray(b["linvel"].T), np.ascontiguousarray(b["angvel"].T))

    def targets(self) -> np.ndarray:
        return np.ascontiguousarray(self.joints["target"].astype(np.float32))

    def subset(self, env_ids) -> "Scene":
        """The listed envs as a new scene (same parameters)."""
        env_ids = np.asarray(env_ids, dtype=np.int64)
        bo, jo = self.body_off, self.joint_off
        nb = bo[env_ids + 1] - bo[env_ids]
        nj = jo[env_ids + 1] - jo[env_ids]
        bsel = np.concatenate([np.arange(bo[e], bo[e + 1]) for e in env_ids]) if len(env_ids) else np.zeros(0, np.int64)
        jsel = np.concatenate([np.arange(jo[e], jo[e + 1]) for e in env_ids]) if len(env_ids) else np.zeros(0, np.int64)
        return Scene(self.name, self.params.copy(),
                     np.concatenate([[0], np.cumsum(nb)]).astype(np.int32), self.bodies[bsel].copy(),
                     np.concatenate([[0], np.cumsum(nj)]).astype(np.int32), self.joints[jsel].copy(),
                     dict(self.meta), self.compounds.copy())


def concat_envs(name, params, env_bodies, env_joints, meta=None) -> Scene:
    nb = [len(b) for b in env_bodies]
    nj = [len(j) for j in env_joints]
    bodies = np.concatenate(env_bodies) if env_bodies else np.zeros(0, BODY_DTYPE)
    joints = np.concatenate(env_joints) if sum(nj) else np.zeros(0, JOINT_DTYPE)
    return Scene(name, params, np.concatenate([[0], np.cumsum(nb)]).astype(np.int32), bodies,
                 np.concatenate([[0], np.cumsum(nj)]).astype(np.int32), joints, meta or {})


# ----------------------------------------------------------------------------- Philox4x32-10
_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint32(0x9E3779B9), np.uint32(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32(counter, key, rounds: int = 10):
    """Philox4x32 block function on arrays: counter (..., 4) uint32, key (..., 2) uint32."""
    c = [np.asarray(counter[..., i], dtype=np.uint32) for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint32).copy()
    k1 = np.asarray(key[..., 1], dtype=np.uint32).copy()
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r:
                k0 = (k0 + _W0).astype(np.uint32)
                k1 = (k1 + _W1).astype(np.uint32)
            p0 = c[0].astype(np.uint64) * _M0
            p1 = c[2].astype(np.uint64) * _M1
            hi0, lo0 = (p0 >> np.uint64(32)).astype(np.uint32), (p0 & _MASK).astype(np.uint32)
            hi1, lo1 = (p1 >> np.uint64(32)).astype(np.uint32), (p1 & _MASK).astype(np.uint32)
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1)


def uniforms(seed: int, env_ids, purpose: int, n: int, sub: int = 0) -> np.ndarray:
    """n doubles in (0, 1) per env: array (len(env_ids), n).  The stream of (seed, env, purpose,
    sub) is counter = (block, env, purpose, sub), key = (seed low 32 bits, seed high 32 bits)."""
    env_ids = np.asarray(env_ids, dtype=np.uint32).reshape(-1)
    nblk = (n + 3) // 4
    E = env_ids.shape[0]
    ctr = np.zeros((E, nblk, 4), dtype=np.uint32)
    ctr[..., 0] = np.arange(nblk, dtype=np.uint32)[None, :]
    ctr[..., 1] = env_ids[:, None]
    ctr[..., 2] = np.uint32(purpose)
    ctr[..., 3] = np.uint32(sub)
    key = np.zeros((E, nblk, 2), dtype=np.uint32)
    key[..., 0] = np.uint32(seed & 0xFFFFFFFF)
    key[..., 1] = np.uint32((seed >> 32) & 0xFFFFFFFF)
    out = philox4x32(ctr, key).reshape(E, nblk * 4)[:, :n]
    return (out.astype(np.float64) + 0.5) * (1.0 / 4294967296.0)


# purposes (stream ids)
P_HEIGHT, P_QUAT, P_SIZE, P_SHAPE, P_MU, P_POS, P_LINK, P_CUBE, P_TARGET, P_COUNT, P_ARM, P_POLE, P_CART, P_COMP = range(14)


def shoemake_quat(u):
    """Uniform random rotation from three uniforms (Shoemake, Graphics Gems III); (w, x, y, z)."""
    u1, u2, u3 = u[..., 0], u[..., 1], u[..., 2]
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    return np.stack([b * np.cos(2 * np.pi * u3), a * np.sin(2 * np.pi * u2),
                     a * np.cos(2 * np.pi * u2), b * np.sin(2 * np.pi * u3)], axis=-1)


def _rot_rows_z(q):
    """Third row of the rotation matrix of (w, x, y, z) quaternions (for placing shapes)."""
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    return np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], axis=-1)


def _body(shape, dims, pos, quat=(1, 0, 0, 0), mass=0.0, density=1000.0, mu=0.5, e=0.0, flags=0,
          linvel=(0, 0, 0), angvel=(0, 0, 0)):
    b = np.zeros(1, dtype=BODY_DTYPE)
    b["shape"], b["flags"] = shape, flags
    d = list(dims) + [0.0] * (3 - len(dims))
    b["dims"] = d
    b["mass"], b["density"], b["friction"], b["restitution"] = mass, density, mu, e
    b["pos"], b["quat"], b["linvel"], b["angvel"] = pos, quat, linvel, angvel
    return b


def _joint(parent, child, fp, fc, kp=0.0, kd=0.0, target=0.0, type=REVOLUTE, limits=None):
    """A joint record; limits = (lower, upper) in rad (revolute) or m (prismatic), None = free."""
    j = np.zeros(1, dtype=JOINT_DTYPE)
    j["parent"], j["child"], j["frame_parent"], j["frame_child"] = parent, child, fp, fc
    j["kp"], j["kd"], j["target"] = kp, kd, target
    j["type"] = type
    if limits is not None:
        j["limited"], j["lower"], j["upper"] = 1, limits[0], limits[1]
    return j


# ----------------------------------------------------------------------------- drop_boxes
def drop_boxes(n_envs: int = 16, seed: int = 0, first_env: int = 0) -> Scene:
    """One 0.1 m, 1 kg box per env; its lowest point starts U[0.05, 0.3] m above the ground
    with a uniform random orientation; mu = 0.5, restitution 0; dt = 0.01 s, 4 iterations."""
    ids = np.arange(first_env, first_env + n_envs)
    q = shoemake_quat(uniforms(seed, ids, P_QUAT, 3))
    clear = 0.05 + 0.25 * uniforms(seed, ids, P_HEIGHT, 1)[:, 0]
    h = 0.05
    r3 = np.abs(_rot_rows_z(q))
    z = clear + h * r3.sum(axis=1)
    bodies = np.zeros(n_envs, dtype=BODY_DTYPE)
    bodies["shape"], bodies["dims"], bodies["mass"], bodies["friction"] = BOX, (h, h, h), 1.0, 0.5
    bodies["pos"] = np.stack([np.zeros(n_envs), np.zeros(n_envs), z], axis=1)
    bodies["quat"] = q
    params = make_params(dt=0.01, pos_iters=4)
    return Scene("drop_boxes", params, np.arange(n_envs + 1, dtype=np.int32), bodies,
                 np.zeros(n_envs + 1, dtype=np.int32), np.zeros(0, JOINT_DTYPE),
                 dict(seed=seed, steps=200))


# ----------------------------------------------------------------------------- arm
ARM_R = 0.04
ARM_KP, ARM_KD = 1000.0, 100.0
_Q_Z = (1.0, 0.0, 0.0, 0.0)
_Q_Y = (math.sqrt(0.5), -math.sqrt(0.5), 0.0, 0.0)  # joint frame whose z is the body's y


def arm_bodies_joints(u_len, u_mass, base_index=0):
    """7 capsule links stacked along +z from a world joint at (0, 0, 0.1); joint axes z, y, z, y,
    z, y, z; each link centred half_len + r above its joint; upright at zero joint angles."""
    bodies, joints = [], []
    zj = 0.1
    prev_hl = None
    for i in range(7):
        L = 0.1 + 0.2 * u_len[i]
        hl = 0.5 * L
        m = 1.0 + 2.0 * u_mass[i]
        cz = zj + hl + ARM_R
        bodies.append(_body(CAPSULE, (ARM_R, hl, 0.0), (0.0, 0.0, cz), mass=m, mu=0.5))
        qf = _Q_Z if i % 2 == 0 else _Q_Y
        if i == 0:
            fp = (0.0, 0.0, zj) + qf
            parent = -1
        else:
            fp = (0.0, 0.0, prev_hl + ARM_R) + qf
            parent = base_index + i - 1
        fc = (0.0, 0.0, -(hl + ARM_R)) + qf
        joints.append(_joint(parent, base_index + i, fp, fc, ARM_KP, ARM_KD, 0.0))
        zj = zj + L + 2 * ARM_R
        prev_hl = hl
    return bodies, joints


def arm_targets(seed: int, env_ids, redraw: int) -> np.ndarray:
    """Drive targets U[-1, 1] rad for the 7 arm joints of each env, redraw number `redraw`."""
    return (2.0 * uniforms(seed, env_ids, P_TARGET, 7, sub=redraw) - 1.0).astype(np.float32)


def arm_cube(n_envs: int = 1024, seed: int = 0, first_env: int = 0) -> Scene:
    """Fixed-base 7-link capsule arm (r = 0.04 m, cylinder length U[0.1, 0.3] m, mass U[1, 3] kg,
    PD drives kp = 1000, kd = 100 toward targets U[-1, 1] rad) plus a 0.04 m cube (density 1000)
    resting at (U[0.2, 0.5], U[-0.3, 0.3]); dt = 0.01 s, 8 iterations."""
    ids = np.arange(first_env, first_env + n_envs)
    ul = uniforms(seed, ids, P_LINK, 14)
    uc = uniforms(seed, ids, P_CUBE, 2)
    tg = arm_targets(seed, ids, 0)
    env_b, env_j = [], []
    for k in range(n_envs):
        b, j = arm_bodies_joints(ul[k, :7], ul[k, 7:])
        b.append(_body(BOX, (0.02, 0.02, 0.02), (0.2 + 0.3 * uc[k, 0], -0.3 + 0.6 * uc[k, 1], 0.02), mu=0.5))
        jj = np.concatenate(j)
        jj["target"] = tg[k]
        env_b.append(np.concatenate(b))
        env_j.append(jj)
    return concat_envs("arm_cube", make_params(dt=0.01, pos_iters=8), env_b, env_j,
                       dict(seed=seed, steps=1000, redraw_every=50))


# ----------------------------------------------------------------------------- cartpole
# A cart on a horizontal rail (prismatic joint to the world along x, 1 m above the ground, limits
# +-CART_LIMIT, PD position drive) and a pole hinged on the cart's top (revolute about y, free).
# Geometry and masses are this project's choice (the paper's benchmark uses a cart-pole robot
# description that is not available here).
CART_HALF = (0.1, 0.075, 0.05)
CART_MASS, CART_KP, CART_KD, CART_LIMIT, RAIL_Z = 1.0, 200.0, 20.0, 1.5, 1.0
POLE_R, POLE_HL, POLE_MASS = 0.03, 0.25, 0.1
_Q_X = (math.sqrt(0.5), 0.0, math.sqrt(0.5), 0.0)   # joint frame whose z is the world x


def cartpole_bodies_joints(theta0: float, x0: float = 0.0, cart_target: float = 0.0):
    """One cart-pole: the pole tilted by theta0 (rad, about y) from upright, the cart at x0."""
    hx, hy, hz = CART_HALF
    cart = _body(BOX, CART_HALF, (x0, 0.0, RAIL_Z), mass=CART_MASS, mu=0.5)
    d = POLE_HL + POLE_R                                  # hinge to pole centre
    c, s_ = math.cos(theta0), math.sin(theta0)
    pq = (math.cos(0.5 * theta0), 0.0, math.sin(0.5 * theta0), 0.0)   # rotation about y by theta0
    pole = _body(CAPSULE, (POLE_R, POLE_HL, 0.0), (x0 + d * s_, 0.0, RAIL_Z + hz + d * c), pq,
                 mass=POLE_MASS, mu=0.5)
    rail = _joint(-1, 0, (0.0, 0.0, RAIL_Z) + _Q_X, (0.0, 0.0, 0.0) + _Q_X, CART_KP, CART_KD, cart_target,
                  type=PRISMATIC, limits=(-CART_LIMIT, CART_LIMIT))
    hinge = _joint(0, 1, (0.0, 0.0, hz) + _Q_Y, (0.0, 0.0, -d) + _Q_Y, type=REVOLUTE)
    return [cart, pole], [rail, hinge]


def cartpole(n_envs: int = 4096, seed: int = 0, first_env: int = 0) -> Scene:
    """The paper's simulation-only benchmark workload: a cart-pole per env at 120 Hz simulation
    with 4 position and 0 velocity solver iterations (control at 60 Hz: 2 steps per control
    step).  Pole angle U[-0.1, 0.1] rad from upright, cart at U[-0.5, 0.5] m; no ground contact."""
    ids = np.arange(first_env, first_env + n_envs)
    u = uniforms(seed, ids, P_POLE, 2)
    env_b, env_j = [], []
    for k in range(n_envs):
        b, j = cartpole_bodies_joints(-0.1 + 0.2 * u[k, 0], -0.5 + u[k, 1])
        env_b.append(np.concatenate(b))
        env_j.append(np.concatenate(j))
    return concat_envs("cartpole", make_params(dt=1.0 / 120.0, pos_iters=4, vel_iters=0, plane_enabled=0), env_b, env_j,
                       dict(seed=seed, steps=500, control_every=2))


def cartpole_targets(seed: int, env_ids, draw: int) -> np.ndarray:
    """Cart drive targets (m) of control step `draw`: U[-1, 1]; the pole joint's target is 0."""
    t = np.zeros((len(env_ids), 2), np.float32)
    t[:, 0] = 2.0 * uniforms(seed, env_ids, P_CART, 1, sub=draw)[:, 0] - 1.0
    return t.reshape(-1)


# ----------------------------------------------------------------------------- random primitives
def _random_shapes(seed, ids, n, slot0=0):
    """Shapes uniform over {box, sphere, capsule}; sizes U[0.02, 0.08] m (box full sides, sphere
    diameter, capsule diameter and cylinder length); mu U[0.3, 1.0]; density 1000 kg/m^3."""
    E = len(ids)
    us = uniforms(seed, ids, P_SHAPE, n, sub=slot0)
    uz = uniforms(seed, ids, P_SIZE, 3 * n, sub=slot0).reshape(E, n, 3)
    um = uniforms(seed, ids, P_MU, n, sub=slot0)
    shape = np.minimum((us * 3).astype(np.int32), 2)
    size = 0.02 + 0.06 * uz
    dims = np.zeros((E, n, 3))
    # box: half of each full side
    dims[shape == BOX] = 0.5 * size[shape == BOX]
    # sphere: radius = half the diameter
    dims[shape == SPHERE, 0] = 0.5 * size[shape == SPHERE, 0]
    # capsule: radius, half cylinder length
    dims[shape == CAPSULE, 0] = 0.5 * size[shape == CAPSULE, 0]
    dims[shape == CAPSULE, 1] = 0.5 * size[shape == CAPSULE, 1]
    bound = np.where(shape == BOX, np.linalg.norm(dims, axis=2),
                     np.where(shape == SPHERE, dims[..., 0], dims[..., 0] + dims[..., 1]))
    mu = 0.3 + 0.7 * um
    return shape, dims, bound, mu


def _prims_to_bodies(shape, dims, pos, q, mu):
    E, n = shape.shape
    b = np.zeros((E, n), dtype=BODY_DTYPE)
    b["shape"], b["dims"], b["pos"], b["quat"], b["friction"] = shape, dims, pos, q, mu
    b["mass"], b["density"] = 0.0, 1000.0
    return b


TRAY_INNER, TRAY_H, TRAY_T = 0.40, 0.10, 0.01


def tray_walls():
    """Four static boxes forming a tray of inner size 0.40 x 0.40 m, height 0.10 m, wall
    thickness 0.01 m, standing on the ground."""
    a, h, t = TRAY_INNER / 2, TRAY_H / 2, TRAY_T / 2
    walls = [((0.0, a + t, h), (a + 2 * t, t, h)), ((0.0, -a - t, h), (a + 2 * t, t, h)),
             ((a + t, 0.0, h), (t, a, h)), ((-a - t, 0.0, h), (t, a, h))]
    return np.concatenate([_body(BOX, d, p, mu=0.5, flags=STATIC) for p, d in walls])


def tray(n_envs: int = 4096, seed: int = 0, n_objects: int = 20, first_env: int = 0) -> Scene:
    """A static tray (4 walls) holding 20 random primitives dropped from random poses, centres in
    [-0.15, 0.15]^2 x [0.05, 0.6] m (kept clear of the walls), bounding spheres disjoint;
    dt = 0.005 s, 8 iterations.  Bodies 0..19 are the objects, 20..23 the walls."""
    ids = np.arange(first_env, first_env + n_envs)
    shape, dims, bound, mu = _random_shapes(seed, ids, n_objects)
    pos = _place_subset(seed, ids, bound, np.full(n_envs, n_objects), 0.15, TRAY_INNER / 2, 0.05, 0.6,
                        np.zeros(n_envs))
    q = shoemake_quat(uniforms(seed, ids, P_QUAT, 3 * n_objects).reshape(n_envs, n_objects, 3))
    objs = _prims_to_bodies(shape, dims, pos, q, mu)
    walls = tray_walls()
    bodies = np.concatenate([objs, np.broadcast_to(walls, (n_envs, 4))], axis=1).reshape(-1)
    nb = n_objects + 4
    return Scene("tray", make_params(dt=0.005, pos_iters=8), np.arange(n_envs + 1, dtype=np.int32) * nb,
                 bodies, np.zeros(n_envs + 1, dtype=np.int32), np.zeros(0, JOINT_DTYPE),
                 dict(seed=seed, steps=500, n_objects=n_objects))


# ----------------------------------------------------------------------------- heterogeneous
def hetero_counts(seed, ids, p=1.0 / 8.0, nmax=64):
    """Body counts from Geom(p) truncated to 1..nmax (inverse CDF of the truncated law)."""
    u = uniforms(seed, ids, P_COUNT, 1)[:, 0]
    tail = 1.0 - (1.0 - p) ** nmax
    n = 1 + np.floor(np.log1p(-u * tail) / np.log1p(-p)).astype(np.int64)
    return np.clip(n, 1, nmax)


def hetero(n_envs: int = 4096, seed: int = 0, pad_to: int = 0, first_env: int = 0) -> Scene:
    """Per-env body count n ~ Geom(1/8) on 1..64; when n >= 8 the 7-link arm is present with
    probability 1/2 and uses 7 of the n bodies.  Free bodies follow the tray's size / mu laws,
    centres in [-0.5, 0.5]^2 x [0.05, 0.6] m, clear of the arm.  pad_to = 64 pads every env
    with far-away static spheres (the padded baseline).  dt = 0.005 s, 8 iterations."""
    ids = np.arange(first_env, first_env + n_envs)
    counts = hetero_counts(seed, ids)
    has_arm = (counts >= 8) & (uniforms(seed, ids, P_ARM, 1)[:, 0] < 0.5)
    nfree = counts - 7 * has_arm
    nmax = int(nfree.max())
    shape, dims, bound, mu = _random_shapes(seed, ids, nmax)
    pos = _place_subset(seed, ids, bound, nfree, 0.5, np.inf, 0.05, 0.6, np.where(has_arm, ARM_R + 0.03, 0.0))
    q = shoemake_quat(uniforms(seed, ids, P_QUAT, 3 * nmax).reshape(n_envs, nmax, 3))
    objs = _prims_to_bodies(shape, dims, pos, q, mu)
    ul = uniforms(seed, ids, P_LINK, 14)
    env_b, env_j = [], []
    pad_body = _body(SPHERE, (0.01, 0, 0), (0.0, 0.0, 0.0), flags=STATIC)
    tg = arm_targets(seed, ids, 0)
    for k in range(n_envs):
        parts, js = [], []
        if has_arm[k]:
            b, j = arm_bodies_joints(ul[k, :7], ul[k, 7:])
            parts.append(np.concatenate(b))
            jj = np.concatenate(j)
            jj["target"] = tg[k]
            js.append(jj)
        parts.append(objs[k, :nfree[k]])
        eb = np.concatenate(parts)
        if pad_to and len(eb) < pad_to:
            npad = pad_to - len(eb)
            pads = np.repeat(pad_body, npad)
            pads["pos"][:, 0] = 100.0 + 0.5 * np.arange(npad)
            pads["pos"][:, 2] = 50.0
            eb = np.concatenate([eb, pads])
        env_b.append(eb)
        env_j.append(np.concatenate(js) if js else np.zeros(0, JOINT_DTYPE))
    return concat_envs("hetero_padded" if pad_to else "hetero", make_params(dt=0.005, pos_iters=8),
                       env_b, env_j, dict(seed=seed, steps=500, counts=counts, has_arm=has_arm))


def _place_subset(seed, ids, bound, nfree, centre_half, wall_half, lo_z, hi_z, avoid):
    """Rejection-sample centres slot by slot so that bounding spheres are disjoint (vectorised
    over envs; env e fills its first nfree[e] slots).  A centre lies in
    [max(-centre_half, -wall_half + R), min(centre_half, wall_half - R)]^2 x [max(lo_z, R), hi_z];
    avoid[e] > 0 keeps it at least avoid + R from the vertical line through the origin."""
    E, n = bound.shape
    pos = np.zeros((E, n, 3))
    for k in range(n):
        need = nfree > k
        if not need.any():
            break
        sel0 = np.nonzero(need)[0]
        pos[sel0, k] = _place_slot(seed, ids[sel0], bound[sel0, :k + 1], pos[sel0, :k], centre_half, wall_half,
                                   lo_z, hi_z, avoid[sel0], k)
    return pos


def _place_slot(seed, ids, bound, prev, centre_half, wall_half, lo_z, hi_z, avoid, k, max_tries=1000):
    E = len(ids)
    R = bound[:, k]
    out = np.zeros((E, 3))
    todo = np.ones(E, dtype=bool)
    for t in range(max_tries):
        if not todo.any():
            return out
        sel = np.nonzero(todo)[0]
        u = uniforms(seed, ids[sel], P_POS, 3, sub=k * 1024 + t)
        lo = np.maximum(-centre_half, -wall_half + R[sel])
        hi = np.minimum(centre_half, wall_half - R[sel])
        x = lo + (hi - lo) * u[:, 0]
        y = lo + (hi - lo) * u[:, 1]
        zl = np.maximum(lo_z, R[sel])
        z = zl + (hi_z - zl) * u[:, 2]
        c = np.stack([x, y, z], axis=1)
        ok = np.ones(len(sel), dtype=bool)
        if k:
            d = np.linalg.norm(prev[sel] - c[:, None, :], axis=2)
            ok &= (d > bound[sel, :k] + R[sel, None]).all(axis=1)
        a = avoid[sel]
        ok &= (a <= 0) | (np.hypot(x, y) > a + R[sel])
        acc = sel[ok]
        out[acc] = c[ok]
        todo[acc] = False
    raise RuntimeError(f"placement failed for slot {k} in {int(todo.sum())} envs")


# ----------------------------------------------------------------------------- compound bodies
_QID = (1.0, 0.0, 0.0, 0.0)


def compound_record(parts):
    """A compound record from [(shape, dims, pos, quat)] (at most 4 parts, body-frame poses)."""
    c = np.zeros((), dtype=COMPOUND_DTYPE)
    c["n_children"] = len(parts)
    for k, (sh, d, pos, q) in enumerate(parts):
        c["shape"][k] = sh
        c["dims"][k] = list(d) + [0.0] * (3 - len(d))
        c["pose"][k] = list(pos) + list(q)
    return c


def dumbbell(r_end, half_bar, r_bar):
    """Two spheres joined by a capsule bar along z (symmetric: centre of mass at the origin,
    principal axes along x, y, z)."""
    return compound_record([(CAPSULE, (r_bar, half_bar), (0.0, 0.0, 0.0), _QID),
                            (SPHERE, (r_end,), (0.0, 0.0, half_bar), _QID),
                            (SPHERE, (r_end,), (0.0, 0.0, -half_bar), _QID)])


def bench(ha, hb, ht, leg, hl):
    """A box top (half sizes ha, hb, ht) on two slab legs (half sizes leg, hb, hl) under its
    ends, shifted so that the centre of mass is the origin (mirror symmetry in x and y makes x,
    y, z principal)."""
    zt, zl = hl + ht, 0.0          # top above the legs' centres
    vt, vl = 8 * ha * hb * ht, 8 * leg * hb * hl
    zc = (vt * zt + 2 * vl * zl) / (vt + 2 * vl)
    return compound_record([(BOX, (ha, hb, ht), (0.0, 0.0, zt - zc), _QID),
                            (BOX, (leg, hb, hl), (ha - leg, 0.0, zl - zc), _QID),
                            (BOX, (leg, hb, hl), (-(ha - leg), 0.0, zl - zc), _QID)])


def jack(h, t):
    """Three crossed boxes along x, y and z (half length h, half thickness t)."""
    return compound_record([(BOX, (h, t, t), (0.0, 0.0, 0.0), _QID), (BOX, (t, h, t), (0.0, 0.0, 0.0), _QID),
                            (BOX, (t, t, h), (0.0, 0.0, 0.0), _QID)])


def compound_bound(rec):
    """Bounding-sphere radius of a compound about its origin."""
    r = 0.0
    for k in range(int(rec["n_children"])):
        d, c = rec["dims"][k], rec["pose"][k][:3]
        sh = int(rec["shape"][k])
        pr = np.linalg.norm(d) if sh == BOX else (d[0] if sh == SPHERE else d[0] + d[1])
        r = max(r, float(np.linalg.norm(c)) + float(pr))
    return r


def compound_library(seed: int, n: int = 32) -> np.ndarray:
    """n compound templates: dumbbells, benches and jacks with extents of 0.04-0.1 m (the tray
    objects' scale), drawn from the seed's own stream (purpose P_COMP)."""
    u = uniforms(seed, np.arange(n), P_COMP, 5)
    recs = []
    for k in range(n):
        kind = min(int(u[k, 0] * 3), 2)
        if kind == 0:
            recs.append(dumbbell(0.01 + 0.01 * u[k, 1], 0.015 + 0.02 * u[k, 2], 0.004 + 0.004 * u[k, 3]))
        elif kind == 1:
            ha, hb = 0.02 + 0.02 * u[k, 1], 0.02 + 0.02 * u[k, 2]
            recs.append(bench(ha, hb, 0.004 + 0.003 * u[k, 3], 0.004, 0.01 + 0.01 * u[k, 4]))
        else:
            recs.append(jack(0.02 + 0.02 * u[k, 1], 0.004 + 0.004 * u[k, 2]))
    return np.array(recs, dtype=COMPOUND_DTYPE)


def compound_tray(n_envs: int = 4096, seed: int = 0, n_objects: int = 12, first_env: int = 0) -> Scene:
    """The tray holding 12 objects dropped from random poses: each a compound body (a template
    of `compound_library`, U{0..31}) with probability 1/2, else a primitive with the tray laws;
    density 1000 kg/m^3, mu U[0.3, 1.0]; dt = 0.005 s, 8 iterations.  Bodies 0..11 are the
    objects, 12..15 the walls."""
    ids = np.arange(first_env, first_env + n_envs)
    lib = compound_library(seed)
    shape, dims, bound, mu = _random_shapes(seed, ids, n_objects)
    uc = uniforms(seed, ids, P_COMP, 2 * n_objects, sub=1).reshape(n_envs, n_objects, 2)
    is_c = uc[..., 0] < 0.5
    tmpl = np.minimum((uc[..., 1] * len(lib)).astype(np.int32), len(lib) - 1)
    lib_bound = np.array([compound_bound(r) for r in lib])
    shape = np.where(is_c, COMPOUND, shape)
    dims = np.where(is_c[..., None], np.stack([tmpl, np.zeros_like(tmpl), np.zeros_like(tmpl)], -1), dims)
    bound = np.where(is_c, lib_bound[tmpl], bound)
    pos = _place_subset(seed, ids, bound, np.full(n_envs, n_objects), 0.15, TRAY_INNER / 2, 0.05, 0.6,
                        np.zeros(n_envs))
    q = shoemake_quat(uniforms(seed, ids, P_QUAT, 3 * n_objects).reshape(n_envs, n_objects, 3))
    objs = _prims_to_bodies(shape, dims, pos, q, mu)
    bodies = np.concatenate([objs, np.broadcast_to(tray_walls(), (n_envs, 4))], axis=1).reshape(-1)
    nb = n_objects + 4
    # a pair of compounds yields up to 9 manifolds (one per pair of parts): capacities above the
    # defaults for 12 dynamic bodies (80 points, 40 manifolds), at the most that keeps an env
    # within 20,480 bytes of LDS (8 envs per CU)
    params = make_params(dt=0.005, pos_iters=8, max_contacts_per_env=164, max_manifolds_per_env=64)
    return Scene("compound_tray", params, np.arange(n_envs + 1, dtype=np.int32) * nb,
                 bodies, np.zeros(n_envs + 1, dtype=np.int32), np.zeros(0, JOINT_DTYPE),
                 dict(seed=seed, steps=500, n_objects=n_objects), lib)


# ----------------------------------------------------------------------------- named workloads
def by_name(name: str, n_envs: int, seed: int = 0, first_env: int = 0) -> Scene:
    if name == "drop_boxes":
        return drop_boxes(n_envs, seed, first_env)
    if name == "arm_cube":
        return arm_cube(n_envs, seed, first_env)
    if name == "tray":
        return tray(n_envs, seed, first_env=first_env)
    if name == "hetero":
        return hetero(n_envs, seed, first_env=first_env)
    if name == "hetero_padded":
        return hetero(n_envs, seed, pad_to=64, first_env=first_env)
    if name == "cartpole":
        return cartpole(n_envs, seed, first_env=first_env)
    if name == "compound_tray":
        return compound_tray(n_envs, seed, first_env=first_env)
    raise ValueError(name)


def single(bodies, joints=None, **params) -> Scene:
    """A one-env scene from explicit body / joint records (hand-built closed-form cases)."""
    b = np.concatenate(bodies) if isinstance(bodies, list) else bodies
    j = np.concatenate(joints) if joints else np.zeros(0, JOINT_DTYPE)
    return Scene("single", make_params(**params), np.array([0, len(b)], np.int32), b,
                 np.array([0, len(j)], np.int32), j, {})


def replicate(scene: Scene, n: int) -> Scene:
    """n copies of a one-env scene."""
    assert scene.n_envs == 1
    out = concat_envs(scene.name, scene.params.copy(), [scene.bodies] * n, [scene.joints] * n, dict(scene.meta))
    out.compounds = scene.compounds.copy()
    return out


body = _body
joint = _joint
