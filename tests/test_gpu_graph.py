"""Captured step sequences (ms_graph_*) against eager ms_step calls, on the GPU.

A graph of k launches replayed r times must leave every env in the bits that r * k eager
launches give, for a batch with several LDS classes (side-stream fork / join inside the graph)
and for an arm batch whose target buffer the caller rewrites between replays.  Each replay is
checked on its own, with eager work and host synchronisation between the replays.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2410_00425_amd import scenes as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def ms():
    from paper_2410_00425_amd import ms as m
    return m


def start_state(sc, warm):
    o = Oracle(sc, 64)
    if warm:
        o.step(warm, n_threads=8)
    st = o.state()
    return {k: torch.from_numpy(np.float32(st[k])).cuda() for k in ("pos", "quat", "linvel", "angvel")}


def fresh(sc, st):
    b = ms().Batch(sc)
    b.reset_envs(torch.arange(sc.n_envs, dtype=torch.int32, device="cuda"), st)
    return b


@pytest.mark.parametrize("name,n,spl,nl", [("hetero", 96, 2, 3), ("tray", 32, 1, 4), ("drop_boxes", 64, 3, 2)])
def test_graph_replays_match_eager(name, n, spl, nl):
    sc = S.by_name(name, n, seed=11)
    st = start_state(sc, 20)
    eager, cap = fresh(sc, st), fresh(sc, st)
    if name == "hetero":
        assert len(cap.classes()) > 1
    g = cap.graph(spl, nl)
    for r in range(3):
        g.launch()
        for _ in range(nl):
            eager.step(spl)
        # eager work of the program between replays
        junk = torch.randn(1 << 16, device="cuda").sum()
        a, b = eager.state_numpy(), cap.state_numpy()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for k in a:
            assert np.array_equal(a[k], b[k]), (r, k)
    g.close()
    eager.close()
    cap.close()


def test_graph_reads_targets_at_replay():
    sc = S.arm_cube(16, seed=12)
    st = start_state(sc, 10)
    eager, cap = fresh(sc, st), fresh(sc, st)
    tbuf = torch.zeros(sc.n_joints, dtype=torch.float32, device="cuda")
    g = cap.graph(2, 2, targets=tbuf)
    for r in range(3):
        t = torch.from_numpy(S.arm_targets(12, np.arange(16), r).reshape(-1).astype(np.float32)).cuda()
        tbuf.copy_(t)
        g.launch()
        eager.step(2, t)
        eager.step(2, t)
        a, b = eager.state_numpy(), cap.state_numpy()
        for k in a:
            assert np.array_equal(a[k], b[k]), (r, k)
    g.close()
    eager.close()
    cap.close()


def test_graph_argument_errors():
    m = ms()
    sc = S.drop_boxes(4, seed=0)
    b = m.Batch(sc)
    with pytest.raises(m.MsError) as e:
        b.graph(0, 1)
    assert e.value.code == m.MS_E_INVALID_ARG
    b.close()
