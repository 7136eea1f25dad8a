"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU, host code only).

A sanitized build of ms_oracle.cpp (-fsanitize=address,undefined, no recovery) runs every
workload generator's scenes, both precisions, the test record, multi-threaded stepping and the
narrowphase / reduction entry points in a child process with the sanitizer runtimes preloaded.
Any out-of-bounds access, use after free, signed overflow or invalid shift aborts the child.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import numpy as np
from oracle.oracle import Oracle, narrow, reduce4
from paper_2410_00425_amd import scenes as S
rng = np.random.default_rng(0)
for name, n, steps in (("drop_boxes", 4, 60), ("arm_cube", 2, 40), ("tray", 2, 60), ("hetero", 12, 30)):
    sc = S.by_name(name, n, seed=3)
    for prec in (32, 64):
        o = Oracle(sc, prec)
        o.step(steps - 1, n_threads=2)
        o.step(1, record=True)
        rec = o.record()
        cnt, mm = o.counters()
        assert np.all(o.state()["status"] & 1 == 0)
        o.close()
# a 64-body env at the size limit with tight capacities (overflow paths)
sc = S.by_name("hetero", 64, seed=1)
big = [e for e in range(sc.n_envs) if sc.body_off[e + 1] - sc.body_off[e] >= 20][:2]
sub = sc.subset(big)
sub.params["max_contacts_per_env"] = 8
sub.params["max_manifolds_per_env"] = 4
o = Oracle(sub, 32)
o.step(40, record=True)
o.record()
for _ in range(200):
    sa, sb = int(rng.integers(-1, 3)), int(rng.integers(0, 3))
    q = rng.normal(size=4); q /= np.linalg.norm(q)
    pa = [0, 0, 0, 1, 0, 0, 0]
    pb = list(rng.uniform(-0.05, 0.05, 3)) + list(q)
    narrow(sa, rng.uniform(0.01, 0.04, 3), pa, sb, rng.uniform(0.01, 0.04, 3), pb)
for n in range(1, 17):
    reduce4(rng.uniform(-0.05, 0.05, (n, 3)), rng.uniform(-0.01, 0.01, n))
print("sanitized oracle ok")
'''


def _runtime(name):
    p = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.slow
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("sanitizer runtimes not installed")
    from oracle import oracle
    lib = oracle.build(force=True, out=str(tmp_path / "liboracle_san.so"),
                       extra=("-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"))
    env = dict(os.environ, MS_ORACLE_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}", ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0 and "sanitized oracle ok" in r.stdout, (r.stdout[-2000:] + r.stderr[-4000:])
