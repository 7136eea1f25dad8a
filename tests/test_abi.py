"""C ABI checks that need no GPU: the library loads, exports every function include/ms.h
declares, passes its host self-check, and rejects invalid descriptors with the documented codes
in the host-only ms_query_batch_bytes."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2410_00425_amd import scenes as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2410_00425_amd", "libms.so")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ms.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ms_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert "ms_step" in names and "ms_create_batch" in names and len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_selfcheck():
    assert ctypes.CDLL(LIB).ms_selfcheck() == 0


def test_query_bytes_and_validation():
    from paper_2410_00425_amd import ms
    sc = S.tray(8, seed=0)
    nb = ms.ms_query_batch_bytes(sc)
    assert nb > 8 * 24 * 13 * 4
    bad = S.tray(2, seed=0)
    bad.bodies["shape"][3] = 7
    with pytest.raises(ms.MsError) as e:
        ms.ms_query_batch_bytes(bad)
    assert e.value.code == ms.MS_E_INVALID_ARG
    arm = S.arm_cube(2, seed=0)
    arm.joints["child"][2] = 99
    with pytest.raises(ms.MsError) as e:
        ms.ms_query_batch_bytes(arm)
    assert e.value.code == ms.MS_E_INVALID_ARG
    big = S.single([S.body(S.SPHERE, (0.01,), (0.1 * i, 0, 0.5), mass=1.0) for i in range(65)])
    with pytest.raises(ms.MsError) as e:
        ms.ms_query_batch_bytes(big)
    assert e.value.code == ms.MS_E_CAPACITY
    p = sc.params.copy()
    p["dt"] = -1
    with pytest.raises(ms.MsError):
        ms.ms_query_batch_bytes(sc, p)
    with pytest.raises(ms.MsError):
        ms.ms_query_batch_bytes(sc, plan=ms.ms_plan(3, 1, 0))
    nan_t = S.arm_cube(1, seed=0)
    nan_t.joints["target"][0] = np.nan
    with pytest.raises(ms.MsError):
        ms.ms_query_batch_bytes(nan_t)


def test_empty_batch_and_size_limits_are_rejected():
    """An empty batch, and an env above 64 bodies or 64 joints, are invalid arguments / capacity
    errors from the host-only query (nothing is enqueued)."""
    from paper_2410_00425_amd import ms
    empty = S.tray(4, seed=0).subset([])
    with pytest.raises(ms.MsError) as e:
        ms.ms_query_batch_bytes(empty)
    assert e.value.code == ms.MS_E_INVALID_ARG
    # exactly 64 bodies is accepted
    sixty_four = S.single([S.body(S.SPHERE, (0.01,), (0.03 * i, 0, 0.5), mass=1.0) for i in range(64)])
    assert ms.ms_query_batch_bytes(sixty_four) > 0


def test_compound_table_validation():
    """The compound table is checked by the host-only query: index in range and integral, 1..4
    parts of primitive shape, unit part quaternions, centre of mass at the body origin and body
    axes principal."""
    from paper_2410_00425_amd import ms
    sc = S.compound_tray(4, seed=0)
    assert ms.ms_query_batch_bytes(sc) > 0

    def rejected(mutate, code=ms.MS_E_INVALID_ARG):
        bad = S.compound_tray(4, seed=0)
        mutate(bad)
        with pytest.raises(ms.MsError) as e:
            ms.ms_query_batch_bytes(bad)
        assert e.value.code == code

    comp = np.nonzero(sc.bodies["shape"] == S.COMPOUND)[0][0]

    def index(v):
        def f(s):
            s.bodies["dims"][comp, 0] = v
        return f
    rejected(index(float(len(sc.compounds))))
    rejected(index(-1.0))
    rejected(index(1.5))

    def table(f):
        def g(s):
            s.compounds = s.compounds.copy()
            f(s.compounds)
        return g
    rejected(table(lambda c: c["n_children"].__setitem__(0, 5)))
    rejected(table(lambda c: c["n_children"].__setitem__(0, 0)))
    rejected(table(lambda c: c["shape"].__setitem__((0, 0), 3)))
    rejected(table(lambda c: c["pose"].__setitem__((0, 0, 3), 0.9)))       # quaternion not unit

    def off_centre(c):
        c["pose"][0, 0, 0] += 0.01                                          # centre of mass moves
    rejected(table(off_centre))

    def tilted(c):
        # two boxes on a diagonal: centre at the origin, products of inertia nonzero
        c[0] = S.compound_record([(S.BOX, (0.02, 0.01, 0.01), (0.03, 0.03, 0.0), (1.0, 0.0, 0.0, 0.0)),
                                  (S.BOX, (0.02, 0.01, 0.01), (-0.03, -0.03, 0.0), (1.0, 0.0, 0.0, 0.0))])
    rejected(table(tilted))
    # a compound body in a scene without a table
    nt = S.compound_tray(4, seed=0)
    nt.compounds = nt.compounds[:0]
    with pytest.raises(ms.MsError):
        ms.ms_query_batch_bytes(nt)
