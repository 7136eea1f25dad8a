"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use this module.  It
loads ``liboracle.so`` built from ``ms_oracle.cpp`` with g++ (no GPU code, no shared source with
the GPU library).  Descriptor arrays are the records produced by the input generators: the
oracle reads them by byte layout (88-byte bodies, 92-byte joints, 96-byte parameters).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ms_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

BODY_BYTES, JOINT_BYTES, PARAMS_BYTES, COMPOUND_BYTES = 88, 92, 96, 180
N_COUNTERS = 20
COUNTER_NAMES = ["pairs_tested", "candidates", "points", "manifolds", "colours", "dynamic", "static",
                 "joints"] + [f"kind{k}" for k in range(12)]


def build(force: bool = False, out: str = _LIB, extra=()) -> str:
    """Compile the oracle with g++ (-O2, no FP contraction); `extra` adds flags (sanitizers)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
                               "-pthread", *extra, "-o", tmp, _SRC])
        os.replace(tmp, out)
    return out


def lib():
    global _lib
    if _lib is None:
        # MS_ORACLE_LIB names an alternative build of the same source (the sanitizer test)
        path = os.environ.get("MS_ORACLE_LIB") or build()
        L = C.CDLL(path)
        P = C.c_void_p
        L.or_create.restype = P
        L.or_create.argtypes = [P, C.c_int, P, P, P, P, C.c_int, C.c_int, P]
        L.or_destroy.argtypes = [P]
        L.or_set_targets.argtypes = [P, P]
        L.or_step.argtypes = [P, C.c_int, C.c_int, C.c_int]
        L.or_get_state.argtypes = [P, P, P, P, P, P]
        L.or_set_state.argtypes = [P, P, P, P, P]
        L.or_record_sizes.argtypes = [P, P, P, P]
        L.or_record_pairs.argtypes = [P, P, P]
        L.or_record_points.argtypes = [P, P, P]
        L.or_record_blocks.argtypes = [P, P]
        L.or_n_counters.restype = C.c_int
        L.or_env_counters.argtypes = [P, P, P]
        L.or_mass_props.argtypes = [C.c_int, P, C.c_double, P, P]
        L.or_compound_props.argtypes = [P, C.c_double, P, P]
        L.or_narrow.restype = C.c_int
        L.or_narrow.argtypes = [C.c_int, P, P, C.c_int, P, P, C.c_double, P, P]
        L.or_box_box_sat.argtypes = [P, P, P, P, P, P]
        L.or_reduce4.restype = C.c_int
        L.or_reduce4.argtypes = [P, C.c_int, P]
        L.or_reset_random.restype = C.c_int
        L.or_reset_random.argtypes = [P, P, C.c_int, P, C.c_int, C.c_uint64, C.c_uint32]
        L.or_apply_actions.argtypes = [P, P, P, P, C.c_float, C.c_float]
        L.or_get_targets.argtypes = [P, P]
        L.or_joint_positions.argtypes = [P, P]
        L.or_contact_forces.argtypes = [P, P]
        L.or_philox4x32_10.argtypes = [P, P, P]
        L.or_sin_series.restype = C.c_double
        L.or_sin_series.argtypes = [C.c_double, C.c_int]
        L.or_cos_series.restype = C.c_double
        L.or_cos_series.argtypes = [C.c_double, C.c_int]
        L.or_normal12.restype = C.c_double
        L.or_normal12.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int]
        assert L.or_n_counters() == N_COUNTERS
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Oracle:
    """The step model on the CPU for a whole batch, in float32 (precision=32) or float64."""

    def __init__(self, scene, precision: int = 32, params=None):
        L = lib()
        p = np.ascontiguousarray(scene.params if params is None else params)
        assert p.dtype.itemsize == PARAMS_BYTES
        self._keep = [p, np.ascontiguousarray(scene.body_off, np.int32), np.ascontiguousarray(scene.bodies),
                      np.ascontiguousarray(scene.joint_off, np.int32), np.ascontiguousarray(scene.joints)]
        assert self._keep[2].dtype.itemsize == BODY_BYTES and self._keep[4].dtype.itemsize == JOINT_BYTES
        comps = np.ascontiguousarray(getattr(scene, "compounds", np.zeros(0, np.uint8)))
        assert len(comps) == 0 or comps.dtype.itemsize == COMPOUND_BYTES
        self._keep.append(comps)
        self.n_envs = scene.n_envs
        self.n_bodies = scene.n_bodies
        self.n_joints = scene.n_joints
        self.precision = precision
        self._h = L.or_create(_ptr(p), self.n_envs, _ptr(self._keep[1]), _ptr(self._keep[2]),
                              _ptr(self._keep[3]), _ptr(self._keep[4]), precision, len(comps),
                              _ptr(comps) if len(comps) else None)

    def close(self):
        if self._h:
            lib().or_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_targets(self, targets):
        t = np.ascontiguousarray(targets, dtype=np.float32)
        assert t.shape == (self.n_joints,)
        lib().or_set_targets(self._h, _ptr(t))

    def step(self, n_steps: int = 1, n_threads: int = 1, record: bool = False):
        lib().or_step(self._h, n_steps, n_threads, 1 if record else 0)

    def state(self):
        B, E = self.n_bodies, self.n_envs
        pos, quat = np.zeros((3, B)), np.zeros((4, B))
        v, w = np.zeros((3, B)), np.zeros((3, B))
        st = np.zeros(E, np.int32)
        lib().or_get_state(self._h, _ptr(pos), _ptr(quat), _ptr(v), _ptr(w), _ptr(st))
        return dict(pos=pos, quat=quat, linvel=v, angvel=w, status=st)

    def set_state(self, pos, quat, linvel, angvel):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (pos, quat, linvel, angvel)]
        assert arrs[0].shape == (3, self.n_bodies) and arrs[1].shape == (4, self.n_bodies)
        lib().or_set_state(self._h, *[_ptr(a) for a in arrs])

    def record(self):
        """The last recorded step: candidate pairs (env, a, b, n_points, decision, kind) with their
        decision margin and friction patch (lambda_t1, lambda_t2, lambda_twist, mu, torsional
        radius) in ``patch``; contact points (env, pair) + (p, n, s0, lambda_n, lambda_n at the
        step start: the cross-step warm start's, else 0); solver blocks (env, kind, index, colour)."""
        L = lib()
        n = [C.c_int64(), C.c_int64(), C.c_int64()]
        L.or_record_sizes(self._h, *[C.byref(x) for x in n])
        npair, npt, nblk = (x.value for x in n)
        pairs = np.zeros((npair, 6), np.int32)
        pm = np.zeros((npair, 6))
        ids = np.zeros((npt, 2), np.int32)
        pts = np.zeros((npt, 9))
        blocks = np.zeros((nblk, 4), np.int32)
        L.or_record_pairs(self._h, _ptr(pairs), _ptr(pm))
        L.or_record_points(self._h, _ptr(ids), _ptr(pts))
        L.or_record_blocks(self._h, _ptr(blocks))
        return dict(pairs=pairs, margin=pm[:, 0].copy(), patch=pm[:, 1:].copy(), point_ids=ids, points=pts,
                    blocks=blocks)

    def reset_random(self, env_ids, joint_sigma=0.0, xy_half=0.0, yaw_half=0.0, targets_follow=True, seed=0, count=0):
        """Randomised reset of the listed envs (see reset_env_random in ms_oracle.cpp)."""
        ids = np.ascontiguousarray(env_ids, dtype=np.int32)
        nz = np.array([joint_sigma, xy_half, yaw_half], np.float32)
        r = lib().or_reset_random(self._h, _ptr(ids), len(ids), _ptr(nz), 1 if targets_follow else 0, int(seed),
                                  int(count))
        if r != 0:
            raise ValueError("joints are not ordered parents first")

    def apply_actions(self, actions, low=None, high=None, lo=-1.0, hi=1.0):
        """Target delta controller: targets += clip(a, -1, 1) (high - low) / 2."""
        a = np.ascontiguousarray(actions, dtype=np.float32)
        assert a.shape == (self.n_joints,)
        lw = None if low is None else np.ascontiguousarray(low, dtype=np.float32)
        hg = None if high is None else np.ascontiguousarray(high, dtype=np.float32)
        lib().or_apply_actions(self._h, _ptr(a), _ptr(lw) if lw is not None else None,
                               _ptr(hg) if hg is not None else None, float(lo), float(hi))

    def targets(self):
        out = np.zeros(self.n_joints, np.float32)
        lib().or_get_targets(self._h, _ptr(out))
        return out

    def joint_positions(self):
        out = np.zeros(self.n_joints)
        lib().or_joint_positions(self._h, _ptr(out))
        return out

    def contact_forces(self):
        """Net contact force on every body over the last step's last substep, [3, B]."""
        out = np.zeros((3, self.n_bodies))
        lib().or_contact_forces(self._h, _ptr(out))
        return out

    def counters(self):
        """Per-env work counters of the last step (int64 [E, N_COUNTERS]) and minimum margins."""
        out = np.zeros((self.n_envs, N_COUNTERS), np.int64)
        mm = np.zeros(self.n_envs)
        lib().or_env_counters(self._h, _ptr(out), _ptr(mm))
        return out, mm


def mass_props(shape: int, dims, mass: float):
    d = np.ascontiguousarray(dims, dtype=np.float64)
    vol = C.c_double()
    inertia = np.zeros(3)
    lib().or_mass_props(shape, _ptr(d), mass, C.byref(vol), _ptr(inertia))
    return vol.value, inertia


def compound_mass_props(record, mass: float):
    """Volume and principal moments (float64) of a compound record (the scenes' COMPOUND_DTYPE)."""
    rec = np.ascontiguousarray(np.asarray(record).reshape(1))
    assert rec.dtype.itemsize == COMPOUND_BYTES
    vol = C.c_double()
    inertia = np.zeros(3)
    lib().or_compound_props(_ptr(rec), mass, C.byref(vol), _ptr(inertia))
    return vol.value, inertia


def narrow(shape_a, dims_a, pose_a, shape_b, dims_b, pose_b, delta=0.01):
    """Contact points of one pair of shapes in float64: array [k, 7] = p(3), n(3), s, and the
    branch code.  shape_a = -1 is the ground plane z = 0."""
    da = np.ascontiguousarray(dims_a if dims_a is not None else np.zeros(3), dtype=np.float64)
    pa = np.ascontiguousarray(pose_a if pose_a is not None else [0, 0, 0, 1, 0, 0, 0], dtype=np.float64)
    db = np.ascontiguousarray(dims_b, dtype=np.float64)
    pb = np.ascontiguousarray(pose_b, dtype=np.float64)
    out = np.zeros((16, 7))
    dec = C.c_int32()
    k = lib().or_narrow(shape_a, _ptr(da), _ptr(pa), shape_b, _ptr(db), _ptr(pb), delta, _ptr(out), C.byref(dec))
    return out[:k].copy(), dec.value


def box_box_sat(dims_a, pose_a, dims_b, pose_b):
    """The 15 separating-axis gaps of two boxes (float64) and their validity flags."""
    arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (dims_a, pose_a, dims_b, pose_b)]
    sep = np.zeros(15)
    valid = np.zeros(15, np.int32)
    lib().or_box_box_sat(*[_ptr(a) for a in arrs], _ptr(sep), _ptr(valid))
    return sep, valid.astype(bool)


def reduce4(points, s):
    """Manifold reduction of a point list (float64 [n, 3] positions, [n] separations, normal +z):
    the indices picked in selection order (deepest, farthest from it, largest triangle, largest
    added area; [-1] * 4 when n <= 4) and the number of points kept."""
    p = np.ascontiguousarray(np.column_stack([np.asarray(points, np.float64), np.asarray(s, np.float64)]))
    picked = np.zeros(4, np.int32)
    n = lib().or_reduce4(_ptr(p), len(p), _ptr(picked))
    return [int(x) for x in picked], n


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def sin_series(x, precision=64):
    return lib().or_sin_series(float(x), precision)


def cos_series(x, precision=64):
    return lib().or_cos_series(float(x), precision)


def normal12(seed, env, count, purpose, first_block, precision=64):
    return lib().or_normal12(int(seed), int(env), int(count), int(purpose), int(first_block), precision)
