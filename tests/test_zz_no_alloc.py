"""ms_step_many_noalloc (the fused multi-batch step that allocates nothing, its work list in the
library's static device scratch) against ms_step_many with caller scratch: the same bits for
every batch, on two calls in a row, the second with a smaller input; a work list beyond the
static maximum is rejected with MS_E_CAPACITY before anything is enqueued."""
import numpy as np
import pytest

from paper_2410_00425_amd import scenes as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def ms():
    from paper_2410_00425_amd import ms as m
    return m


def twins(scs):
    m = ms()
    return [m.Batch(sc) for sc in scs], [m.Batch(sc) for sc in scs]


def assert_same(ref, got, what):
    for b_ref, b_got in zip(ref, got):
        a, b = b_ref.state_numpy(), b_got.state_numpy()
        for k in ("pos", "quat", "linvel", "angvel", "status"):
            assert np.array_equal(a[k], b[k]), (what, b_ref.scene.name, k)


def test_noalloc_equals_step_many_on_two_calls():
    m = ms()
    print("no-alloc: call 1 = tray 64 + hetero 96 + arm 24 (several LDS sizes, bins launch)", flush=True)
    scs = [S.tray(64, seed=31), S.hetero(96, seed=32), S.arm_cube(24, seed=33)]
    ref, got = twins(scs)
    tg = [None, None, torch.from_numpy(S.arm_targets(33, np.arange(24), 1).reshape(-1)).cuda()]
    assert m.query_step_many_bytes(ref) <= m.STEP_MANY_NOALLOC_BYTES
    for _ in range(2):
        m.step_many(ref, 3, targets=tg)
        m.step_many_noalloc(got, 3, targets=tg)
    torch.cuda.synchronize()
    assert_same(ref, got, "call 1")
    # the batches moved: the steps did something
    assert not np.array_equal(ref[0].state_numpy()["pos"], scs[0].bodies["pos"].T)

    print("no-alloc: call 2 = one-box batch of 16 envs (one LDS class) and the tray batch alone", flush=True)
    small = [S.drop_boxes(16, seed=34)]
    ref2, got2 = twins(small)
    m.step_many(ref2, 2)
    m.step_many_noalloc(got2, 2)
    m.step_many(ref[:1], 1)
    m.step_many_noalloc(got[:1], 1)
    torch.cuda.synchronize()
    assert_same(ref2, got2, "call 2")
    assert_same(ref[:1], got[:1], "call 3")
    for b in ref + got + ref2 + got2:
        b.close()


def test_noalloc_rejects_oversized_work_list():
    m = ms()
    print("no-alloc: oversized work list", flush=True)
    b = m.Batch(S.drop_boxes(4096, seed=35))
    before = b.state_numpy()
    k = m.STEP_MANY_NOALLOC_BYTES // m.query_step_many_bytes([b]) + 1
    assert m.query_step_many_bytes([b] * k) > m.STEP_MANY_NOALLOC_BYTES
    with pytest.raises(m.MsError) as e:
        m.step_many_noalloc([b] * k, 1)
    assert e.value.code == m.MS_E_CAPACITY
    torch.cuda.synchronize()
    after = b.state_numpy()
    for key in before:
        assert np.array_equal(before[key], after[key]), key
    b.close()
