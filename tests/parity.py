"""Shared helpers of the parity tests: the one-step parity rule and GPU-vs-oracle comparison.

The rule (float32 arithmetic on both sides): per component |a - b| <= 1e-4 max(|b|, floor), with
floors x 0.01 m, v 0.1 m/s, q 1 and w 0.1 m/s / r_body, r_body the body's smallest half-size, so
that every point of every body is held to 1e-4 relative velocity.  Candidate pair lists must be
bit-identical (exact AABB arithmetic on both sides).  An env whose oracle record shows a discrete
decision within MARGIN of its threshold may take the other branch (excused) and is only checked
for validity; at most MAX_EXCUSED of the envs may be excused.
"""
import numpy as np

from paper_2410_00425_amd import scenes as S

MARGIN = 1e-5
REL = 1e-4


def part_scale(shape, dims):
    d = np.asarray(dims, np.float64)
    return d.min() if shape == S.BOX else d[0]


def body_scale(bodies, compounds=None):
    """Smallest half-size of each body (of its smallest part for a compound)."""
    d = bodies["dims"].astype(np.float64)
    out = np.where(bodies["shape"] == S.BOX, d.min(axis=1), d[:, 0])
    for i in np.nonzero(bodies["shape"] == S.COMPOUND)[0]:
        rec = compounds[int(d[i, 0])]
        out[i] = min(part_scale(int(rec["shape"][k]), rec["dims"][k][:3 if rec["shape"][k] == S.BOX else 1])
                     for k in range(int(rec["n_children"])))
    return out


def env_ok(sa, sb, bodies, sl, rel=REL, compounds=None):
    wf = 0.1 / body_scale(bodies[sl], compounds)
    for k, fl in (("pos", 0.01), ("linvel", 0.1), ("angvel", wf), ("quat", 1.0)):
        x, y = np.asarray(sa[k][:, sl], np.float64), np.asarray(sb[k][:, sl], np.float64)
        if k == "quat":
            x = x * np.where(np.sum(x * y, axis=0) < 0, -1.0, 1.0)
        if not np.all(np.abs(x - y) <= rel * np.maximum(np.abs(y), fl)):
            return False
    return True


def compare_states(scene, sa, sb, margins, envs=None, max_excused_frac=0.001, min_excused=1):
    """Check the parity rule env by env; returns (bad envs, excused envs)."""
    bo = scene.body_off
    envs = range(scene.n_envs) if envs is None else envs
    comps = getattr(scene, "compounds", None)
    bad = [e for e in envs if not env_ok(sa, sb, scene.bodies, slice(bo[e], bo[e + 1]), compounds=comps)]
    excused = [e for e in bad if margins[e] < MARGIN]
    return [e for e in bad if e not in excused], excused


def compare_pairs(gpu_pairs, orc_pairs, margins):
    """Candidate lists (env, a, b) must be identical; per-pair kept points and branch must match
    unless the env is excused.  Returns the set of envs whose decisions differ."""
    g = gpu_pairs[:, :3]
    o = orc_pairs[:, :3]
    assert g.shape == o.shape, (g.shape, o.shape)
    assert np.array_equal(g, o)
    diff = np.nonzero((gpu_pairs[:, 3] != orc_pairs[:, 3]) | (gpu_pairs[:, 4] != orc_pairs[:, 4]))[0]
    envs = set(int(gpu_pairs[k, 0]) for k in diff)
    for e in envs:
        assert margins[e] < MARGIN, f"env {e}: decision differs with margin {margins[e]}"
    return envs
