"""Python binding of libms (argument marshalling only).

Every step of the simulation runs in the HIP kernels of ``libms.so``; this module converts numpy
descriptors and torch device tensors into the C ABI's plain pointers.  torch provides the
device memory (the caller-owned workspace and state buffers) and the stream.  Importing it
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import scenes

_HERE = os.path.dirname(os.path.abspath(__file__))
# MS_LIBRARY may name another build of the same library (the per-phase clock build)
LIB_PATH = os.environ.get("MS_LIBRARY") or os.path.join(_HERE, "libms.so")

# torch first: its HIP runtime is then the one libms binds to (loading libms first would bring in
# a second copy of the runtime, and torch's device calls and the library's would not share a device)
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2410_00425_amd.build` "
                      "(hipcc, gfx950) before using the GPU step")

_lib = C.CDLL(LIB_PATH)

MS_OK, MS_E_INVALID_ARG, MS_E_NO_WORKSPACE, MS_E_BUDGET, MS_E_DEVICE, MS_E_CAPACITY, MS_E_STATE = range(7)
STATUS_NONFINITE, STATUS_CONTACT_OVERFLOW, STATUS_COLOR_OVERFLOW = 1, 2, 4
PLANE = 0xFFFF
STEP_MANY_NOALLOC_BYTES = 4 << 20   # MS_STEP_MANY_NOALLOC_BYTES


class MsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libms error {code}: {msg}")
        self.code = code


class ms_scene_desc(C.Structure):
    _fields_ = [("n_envs", C.c_int32), ("env_body_off", C.c_void_p), ("bodies", C.c_void_p),
                ("env_joint_off", C.c_void_p), ("joints", C.c_void_p), ("n_compounds", C.c_int32),
                ("compounds", C.c_void_p)]


class ms_state_view(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("quat", C.c_void_p), ("linvel", C.c_void_p), ("angvel", C.c_void_p),
                ("status", C.c_void_p)]


class ms_reset_noise(C.Structure):
    _fields_ = [("joint_sigma", C.c_float), ("xy_half", C.c_float), ("yaw_half", C.c_float),
                ("targets_follow", C.c_int32)]


class ms_plan(C.Structure):
    _fields_ = [("lanes_per_env", C.c_int32), ("pack", C.c_int32), ("max_resident_groups", C.c_int32),
                ("launch_mode", C.c_int32)]


_P = C.c_void_p
_I = C.c_int32
_sig = {
    "ms_query_batch_bytes": [_P, _P, _P, C.POINTER(C.c_size_t)],
    "ms_create_batch": [_P, _P, _P, _P, C.c_size_t, _P, C.POINTER(_P)],
    "ms_step": [_P, _P, _I, _P],
    "ms_reset_envs": [_P, _P, _I, _P, _P],
    "ms_get_state": [_P, _P, _P],
    "ms_get_layout": [_P, _P, _P],
    "ms_get_sizes": [_P, _P, _P, _P],
    "ms_get_plan": [_P, _P, _P, _P, _P],
    "ms_get_contacts": [_P, _P, _I, _P, _I, _P, _I, _P, _P, _P, _P],
    "ms_get_stats": [_P, _P, _I, _P],
    "ms_get_classes": [_P, _P, _P],
    "ms_tune_batch": [_P, _I, _P],
    "ms_destroy_batch": [_P],
    "ms_graph_create": [_P, _P, _I, _I, C.POINTER(_P)],
    "ms_graph_launch": [_P, _P],
    "ms_graph_destroy": [_P],
    "ms_server_create": [_P, C.c_size_t, C.c_size_t, C.POINTER(_P)],
    "ms_server_open": [_P, _P, _P, _P, C.POINTER(C.c_int64)],
    "ms_server_submit": [_P, C.c_int64, _I, _P, C.POINTER(C.c_int64)],
    "ms_server_wait": [_P, C.c_int64, _P],
    "ms_server_close": [_P, C.c_int64],
    "ms_server_get_state": [_P, C.c_int64, _P, _P],
    "ms_server_drain": [_P],
    "ms_server_stats": [_P, _P],
    "ms_server_destroy": [_P],
    "ms_peak_fp32": [_P, _I, _I, _P],
    "ms_query_step_many_bytes": [_P, _I, C.POINTER(C.c_size_t)],
    "ms_step_many": [_P, _P, _I, _I, _P, C.c_size_t, _P],
    "ms_step_many_noalloc": [_P, _P, _I, _I, _P],
    "ms_reset_envs_random": [_P, _P, _I, _P, C.c_uint64, C.c_uint32, _P],
    "ms_apply_actions": [_P, _P, _P, _P, C.c_float, C.c_float, _P],
    "ms_get_targets": [_P, _P, _P],
    "ms_get_joint_positions": [_P, _P, _P],
    "ms_set_contact_forces": [_P, _I, _P],
    "ms_get_contact_forces": [_P, _P, _P],
    "ms_get_invalid_ids": [_P, C.POINTER(C.c_int32), _I, _P],
    "ms_get_phase_clocks": [_P, _P, _I, _P],
}
for _name, _args in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.ms_server_clock.restype = C.c_double
_lib.ms_last_error.restype = C.c_char_p
_lib.ms_version.restype = C.c_char_p


def _check(code):
    if code != MS_OK:
        raise MsError(code, _lib.ms_last_error().decode())


def ms_version() -> str:
    return _lib.ms_version().decode()


def _scene_struct(scene):
    arrs = [np.ascontiguousarray(scene.body_off, np.int32), np.ascontiguousarray(scene.bodies),
            np.ascontiguousarray(scene.joint_off, np.int32), np.ascontiguousarray(scene.joints)]
    assert arrs[1].dtype == scenes.BODY_DTYPE and arrs[3].dtype == scenes.JOINT_DTYPE
    comps = np.ascontiguousarray(getattr(scene, "compounds", np.zeros(0, scenes.COMPOUND_DTYPE)))
    assert len(comps) == 0 or comps.dtype == scenes.COMPOUND_DTYPE
    arrs.append(comps)
    sd = ms_scene_desc(scene.n_envs, arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data,
                       arrs[3].ctypes.data if len(arrs[3]) else None, len(comps),
                       comps.ctypes.data if len(comps) else None)
    return sd, arrs


def _params(scene, params):
    p = np.ascontiguousarray(scene.params if params is None else params)
    assert p.dtype == scenes.PARAMS_DTYPE
    return p


def _plan(lanes_per_env=0, pack=1, max_resident_groups=0, launch_mode=0):
    return ms_plan(int(lanes_per_env), int(pack), int(max_resident_groups), int(launch_mode))


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def ms_query_batch_bytes(scene, params=None, plan=None) -> int:
    p = _params(scene, params)
    sd, keep = _scene_struct(scene)
    pl = plan or _plan()
    out = C.c_size_t()
    _check(_lib.ms_query_batch_bytes(p.ctypes.data, C.byref(sd), C.byref(pl), C.byref(out)))
    return out.value


class Batch:
    """A batch of envs resident on one GPU: owns its torch workspace and the C handle."""

    def __init__(self, scene, params=None, device="cuda:0", lanes_per_env=0, pack=1, max_resident_groups=0,
                 stream=None, launch_mode=0):
        import torch
        self.device = torch.device(device)
        self.scene = scene
        self.params = _params(scene, params)
        self.n_envs, self.n_bodies, self.n_joints = scene.n_envs, scene.n_bodies, scene.n_joints
        self._plan = _plan(lanes_per_env, pack, max_resident_groups, launch_mode)
        sd, keep = _scene_struct(scene)
        nbytes = C.c_size_t()
        _check(_lib.ms_query_batch_bytes(self.params.ctypes.data, C.byref(sd), C.byref(self._plan),
                                         C.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        with torch.cuda.device(self.device):
            # 256-byte alignment: over-allocate and offset
            self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
            base = self._ws.data_ptr()
            self._ws_ptr = (base + 255) & ~255
            h = C.c_void_p()
            _check(_lib.ms_create_batch(self.params.ctypes.data, C.byref(sd), C.byref(self._plan),
                                        C.c_void_p(self._ws_ptr), self.workspace_bytes, _stream(stream),
                                        C.byref(h)))
        self._h = h

    # ------------------------------------------------------------------ ABI wrappers
    def step(self, n_steps: int = 1, targets=None, stream=None):
        """ms_step: advance every env by n_steps steps; targets is a float32 device tensor [J]."""
        tp = None
        if targets is not None:
            assert targets.dtype.is_floating_point and targets.numel() == self.n_joints and targets.is_cuda
            assert targets.is_contiguous()
            tp = C.c_void_p(targets.data_ptr())
        _check(_lib.ms_step(self._h, tp, int(n_steps), _stream(stream)))

    def reset_envs(self, env_ids, src=None, stream=None):
        """ms_reset_envs: env_ids an int32 device tensor; src None (initial state) or a dict of
        full-batch SoA device tensors pos [3, B], quat [4, B], linvel [3, B], angvel [3, B]."""
        import torch
        assert env_ids.dtype == torch.int32 and env_ids.is_cuda and env_ids.is_contiguous()
        view = None
        if src is not None:
            for k, rows in (("pos", 3), ("quat", 4), ("linvel", 3), ("angvel", 3)):
                t = src[k]
                assert t.dtype == torch.float32 and t.is_cuda and t.is_contiguous() and tuple(t.shape) == (rows, self.n_bodies)
            view = ms_state_view(src["pos"].data_ptr(), src["quat"].data_ptr(), src["linvel"].data_ptr(),
                                 src["angvel"].data_ptr(), None)
        _check(_lib.ms_reset_envs(self._h, C.c_void_p(env_ids.data_ptr()), int(env_ids.numel()),
                                  C.byref(view) if view is not None else None, _stream(stream)))

    def reset_envs_random(self, env_ids, joint_sigma=0.0, xy_half=0.0, yaw_half=0.0, targets_follow=True, seed=0,
                          count=0, stream=None):
        """ms_reset_envs_random: seeded randomised reset of the listed envs (int32 device tensor)."""
        import torch
        assert env_ids.dtype == torch.int32 and env_ids.is_cuda and env_ids.is_contiguous()
        nz = ms_reset_noise(float(joint_sigma), float(xy_half), float(yaw_half), 1 if targets_follow else 0)
        _check(_lib.ms_reset_envs_random(self._h, C.c_void_p(env_ids.data_ptr()), int(env_ids.numel()), C.byref(nz),
                                         int(seed), int(count), _stream(stream)))

    def apply_actions(self, actions, low=None, high=None, lo=-1.0, hi=1.0, stream=None):
        """ms_apply_actions: targets += clip(a, -1, 1) (high - low) / 2 (float32 device tensors [J])."""
        def ptr(t):
            if t is None:
                return None
            assert t.is_cuda and t.is_contiguous() and t.numel() == self.n_joints
            return C.c_void_p(t.data_ptr())
        _check(_lib.ms_apply_actions(self._h, ptr(actions), ptr(low), ptr(high), float(lo), float(hi), _stream(stream)))

    def targets(self, stream=None):
        """ms_get_targets: the current drive targets, float32 device tensor [J]."""
        import torch
        out = torch.empty(self.n_joints, dtype=torch.float32, device=self.device)
        _check(_lib.ms_get_targets(self._h, C.c_void_p(out.data_ptr()) if self.n_joints else None, _stream(stream)))
        return out

    def joint_positions(self, stream=None):
        """ms_get_joint_positions: float32 device tensor [J]."""
        import torch
        out = torch.empty(self.n_joints, dtype=torch.float32, device=self.device)
        _check(_lib.ms_get_joint_positions(self._h, C.c_void_p(out.data_ptr()) if self.n_joints else None,
                                           _stream(stream)))
        return out

    def set_contact_forces(self, enable=True, stream=None):
        _check(_lib.ms_set_contact_forces(self._h, 1 if enable else 0, _stream(stream)))

    def contact_forces(self, stream=None):
        """ms_get_contact_forces: float32 device tensor [3, B] (net contact force of the last step)."""
        import torch
        out = torch.empty(3, self.n_bodies, dtype=torch.float32, device=self.device)
        _check(_lib.ms_get_contact_forces(self._h, C.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def phase_clocks(self, reset=False, stream=None):
        """ms_get_phase_clocks (per-phase clock build only): int64 [16] wave-cycles per phase."""
        out = np.zeros(16, np.int64)
        _check(_lib.ms_get_phase_clocks(self._h, out.ctypes.data, 1 if reset else 0, _stream(stream)))
        return out

    def invalid_ids(self, clear=False, stream=None) -> int:
        v = C.c_int32()
        _check(_lib.ms_get_invalid_ids(self._h, C.byref(v), 1 if clear else 0, _stream(stream)))
        return v.value

    def get_state(self, out=None, stream=None):
        """ms_get_state into (new or given) device tensors; returns the dict."""
        import torch
        B, E = self.n_bodies, self.n_envs
        if out is None:
            f = dict(dtype=torch.float32, device=self.device)
            out = dict(pos=torch.empty(3, B, **f), quat=torch.empty(4, B, **f), linvel=torch.empty(3, B, **f),
                       angvel=torch.empty(3, B, **f), status=torch.empty(E, dtype=torch.int32, device=self.device))
        view = ms_state_view(out["pos"].data_ptr(), out["quat"].data_ptr(), out["linvel"].data_ptr(),
                             out["angvel"].data_ptr(), out["status"].data_ptr())
        _check(_lib.ms_get_state(self._h, C.byref(view), _stream(stream)))
        return out

    def state_numpy(self):
        import torch
        st = self.get_state()
        torch.cuda.current_stream().synchronize()
        return {k: v.cpu().numpy() for k, v in st.items()}

    def layout(self):
        bo = np.zeros(self.n_envs + 1, np.int32)
        jo = np.zeros(self.n_envs + 1, np.int32)
        _check(_lib.ms_get_layout(self._h, bo.ctypes.data, jo.ctypes.data))
        return bo, jo

    def plan(self):
        nt, grid, lds = C.c_int32(), C.c_int32(), C.c_int32()
        lanes = np.zeros(self.n_envs, np.int32)
        _check(_lib.ms_get_plan(self._h, C.byref(nt), C.byref(grid), C.byref(lds), lanes.ctypes.data))
        return dict(n_tiles=nt.value, grid=grid.value, lds_bytes=lds.value, lanes=lanes)

    def contacts(self, stream=None):
        """ms_get_contacts (needs debug_export): pairs int32 [n, 5], points float32 [n, 8],
        manifolds float32 [n, 8]."""
        n = [C.c_int32(), C.c_int32(), C.c_int32()]
        _check(_lib.ms_get_contacts(self._h, None, 0, None, 0, None, 0, *[C.byref(x) for x in n], _stream(stream)))
        np_, npt, nm = (x.value for x in n)
        pairs = np.zeros((np_, 5), np.int32)
        pts = np.zeros((npt, 8), np.float32)
        mans = np.zeros((nm, 8), np.float32)
        _check(_lib.ms_get_contacts(self._h, pairs.ctypes.data, np_, pts.ctypes.data, npt, mans.ctypes.data, nm,
                                    *[C.byref(x) for x in n], _stream(stream)))
        return dict(pairs=pairs, points=pts, manifolds=mans)

    def classes(self):
        """ms_get_classes: per LDS class {tiles, lds_bytes, variant, lanes, first_tile}."""
        n = C.c_int32()
        _check(_lib.ms_get_classes(self._h, C.byref(n), None))
        out = np.zeros((n.value, 5), np.int32)
        _check(_lib.ms_get_classes(self._h, C.byref(n), out.ctypes.data))
        return [dict(tiles=int(r[0]), lds_bytes=int(r[1]), variant=int(r[2]), lanes=int(r[3])) for r in out]

    def tune(self, trial_steps=3, stream=None):
        """ms_tune_batch: pick the fastest kernel variant per LDS class (state is restored)."""
        _check(_lib.ms_tune_batch(self._h, int(trial_steps), _stream(stream)))
        return self.classes()

    def stats(self, reset=False, stream=None):
        """ms_get_stats: int64 [E, 16] work counters accumulated since the last reset."""
        out = np.zeros((self.n_envs, 16), np.int64)
        _check(_lib.ms_get_stats(self._h, out.ctypes.data, 1 if reset else 0, _stream(stream)))
        return out

    def graph(self, steps_per_launch=1, n_launches=1, targets=None):
        """ms_graph_create: n_launches ms_step calls captured into a replayable HIP graph."""
        return Graph(self, steps_per_launch, n_launches, targets)

    def close(self):
        if getattr(self, "_h", None):
            _lib.ms_destroy_batch(self._h)
            self._h = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A captured sequence of steps of one batch (ms_graph_*); replay with launch()."""

    def __init__(self, batch, steps_per_launch, n_launches, targets=None):
        self.batch = batch
        self.steps = int(steps_per_launch) * int(n_launches)
        self._targets = targets   # the graph reads this buffer at replay: keep it alive
        tp = None
        if targets is not None:
            assert targets.is_cuda and targets.is_contiguous() and targets.numel() == batch.n_joints
            tp = C.c_void_p(targets.data_ptr())
        h = C.c_void_p()
        _check(_lib.ms_graph_create(batch._h, tp, int(steps_per_launch), int(n_launches), C.byref(h)))
        self._g = h

    def launch(self, stream=None):
        _check(_lib.ms_graph_launch(self._g, _stream(stream)))

    def close(self):
        if getattr(self, "_g", None):
            _lib.ms_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _batch_lists(batches, targets):
    hs = (C.c_void_p * len(batches))(*[b._h for b in batches])
    tp = None
    if targets is not None:
        assert len(targets) == len(batches)
        for b, t in zip(batches, targets):
            assert t is None or (t.is_cuda and t.is_contiguous() and t.numel() == b.n_joints)
        tp = (C.c_void_p * len(batches))(*[None if t is None else t.data_ptr() for t in targets])
    return hs, tp


def query_step_many_bytes(batches) -> int:
    hs, _ = _batch_lists(batches, None)
    out = C.c_size_t()
    _check(_lib.ms_query_step_many_bytes(hs, len(batches), C.byref(out)))
    return out.value


def step_many(batches, n_steps: int = 1, targets=None, scratch=None, stream=None):
    """ms_step_many: one fused launch over several batches; scratch is a uint8 device tensor of
    at least query_step_many_bytes() bytes (allocated here when None)."""
    import torch
    need = query_step_many_bytes(batches)
    if scratch is None:
        scratch = torch.empty(need + 256, dtype=torch.uint8, device=batches[0].device)
    ptr = (scratch.data_ptr() + 255) & ~255
    avail = scratch.numel() - (ptr - scratch.data_ptr())
    hs, tp = _batch_lists(batches, targets)
    _check(_lib.ms_step_many(hs, tp, len(batches), int(n_steps), C.c_void_p(ptr), avail, _stream(stream)))
    return scratch


def step_many_noalloc(batches, n_steps: int = 1, targets=None, stream=None):
    """ms_step_many_noalloc: the same fused launch with the library's static work-list scratch
    (nothing is allocated)."""
    hs, tp = _batch_lists(batches, targets)
    _check(_lib.ms_step_many_noalloc(hs, tp, len(batches), int(n_steps), _stream(stream)))


class ms_request_info(C.Structure):
    _fields_ = [("request", C.c_int64), ("session", C.c_int64), ("status", C.c_int32), ("n_steps", C.c_int32),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
                ("fused_batches", C.c_int32), ("pad", C.c_int32)]


def server_clock() -> float:
    return _lib.ms_server_clock()


def peak_fp32(out, n_waves: int, iters: int, stream=None):
    """Launch the FP32 issue-rate kernel (ms_peak_fp32) writing into the float32 CUDA tensor `out`
    (at least n_waves * 64 elements); returns the FLOP count of the launch."""
    if out.dtype.itemsize != 4 or not out.is_cuda or out.numel() < n_waves * 64:
        raise ValueError("out must be a float32 CUDA tensor of at least n_waves * 64 elements")
    _check(_lib.ms_peak_fp32(C.c_void_p(out.data_ptr()), int(n_waves), int(iters), _stream(stream)))
    return 16 * int(iters) * 64 * int(n_waves)


class Server:
    """ms_server_*: sessions admitted against an HBM arena and continuous batching of their step
    requests.  The arena is a torch uint8 tensor owned by this object; every call is thread safe
    (ctypes releases the GIL while the library waits)."""

    def __init__(self, arena_bytes: int, scratch_bytes: int = 0, device="cuda:0"):
        import torch
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self._arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=self.device)
            ptr = (self._arena.data_ptr() + 255) & ~255
            h = C.c_void_p()
            _check(_lib.ms_server_create(C.c_void_p(ptr), int(arena_bytes), int(scratch_bytes), C.byref(h)))
        self._h = h
        self._scenes = {}

    def open(self, scene, params=None, lanes_per_env=0, pack=1) -> int:
        p = _params(scene, params)
        sd, keep = _scene_struct(scene)
        pl = _plan(lanes_per_env, pack, 0)
        sid = C.c_int64()
        _check(_lib.ms_server_open(self._h, p.ctypes.data, C.byref(sd), C.byref(pl), C.byref(sid)))
        self._scenes[sid.value] = scene
        return sid.value

    def submit(self, session: int, n_steps: int, targets=None) -> int:
        rid = C.c_int64()
        tp = None
        if targets is not None:
            t = np.ascontiguousarray(targets, dtype=np.float32)
            assert t.size == self._scenes[session].n_joints
            tp = t.ctypes.data
        _check(_lib.ms_server_submit(self._h, int(session), int(n_steps), tp, C.byref(rid)))
        return rid.value

    def wait(self, request: int) -> dict:
        info = ms_request_info()
        _check(_lib.ms_server_wait(self._h, int(request), C.byref(info)))
        return dict(request=info.request, session=info.session, status=info.status, n_steps=info.n_steps,
                    t_submit=info.t_submit, t_start=info.t_start, t_done=info.t_done, fused=info.fused_batches)

    def close_session(self, session: int):
        _check(_lib.ms_server_close(self._h, int(session)))

    def get_state(self, session: int) -> dict:
        import torch
        sc = self._scenes[session]
        B, E = sc.n_bodies, sc.n_envs
        f = dict(dtype=torch.float32, device=self.device)
        out = dict(pos=torch.empty(3, B, **f), quat=torch.empty(4, B, **f), linvel=torch.empty(3, B, **f),
                   angvel=torch.empty(3, B, **f), status=torch.empty(E, dtype=torch.int32, device=self.device))
        view = ms_state_view(out["pos"].data_ptr(), out["quat"].data_ptr(), out["linvel"].data_ptr(),
                             out["angvel"].data_ptr(), out["status"].data_ptr())
        s = torch.cuda.current_stream(self.device)
        _check(_lib.ms_server_get_state(self._h, int(session), C.byref(view), C.c_void_p(s.cuda_stream)))
        s.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}

    def drain(self):
        _check(_lib.ms_server_drain(self._h))

    def stats(self) -> dict:
        out = np.zeros(8, np.int64)
        _check(_lib.ms_server_stats(self._h, out.ctypes.data))
        keys = ("launches", "fused_batches", "env_steps", "requests_done", "sessions_admitted", "busy_us",
                "peak_arena_bytes", "sessions_rejected")
        return dict(zip(keys, (int(x) for x in out)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.ms_server_destroy(self._h)
            self._h = None
            self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# The C names, for callers that prefer the flat ABI.
def ms_create_batch(scene, params=None, device="cuda:0", **plan) -> Batch:
    return Batch(scene, params, device, **plan)


def ms_step(batch: Batch, targets=None, n_steps: int = 1, stream=None):
    batch.step(n_steps, targets, stream)


def ms_reset_envs(batch: Batch, env_ids, src=None, stream=None):
    batch.reset_envs(env_ids, src, stream)


def ms_get_state(batch: Batch, out=None, stream=None):
    return batch.get_state(out, stream)


def ms_get_contacts(batch: Batch, stream=None):
    return batch.contacts(stream)


def ms_destroy_batch(batch: Batch):
    batch.close()
