"""The allocation-free repair entry point, mf_apply_batch_device_noalloc,
through the C ABI: on the same graph and the same device-resident batches its
values equal mf_apply_batch_device's (and the oracle's), call after call, the
second call with a smaller batch; its limits are errors that change nothing.
"""
import numpy as np
import pytest

import oracle
import paper_2511_01235_amd as mf
from paper_2511_01235_amd import gen

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)


@pytest.mark.parametrize("name", ["er2000", "rmat12", "grid64"])
def test_noalloc_matches_allocating_repair(name):
    import torch
    assert torch.cuda.is_available()
    g, stream, k, _ = gen.workload(name)
    say("noalloc", name, "batch", k)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    sizes = [k, max(1, k // 3), k, 7, max(1, k // 2)]   # the second call smaller than the first
    batches = []
    for kk in sizes:
        u, v, c = stream.next_batch(kk)
        batches.append(torch.from_numpy(np.ascontiguousarray(np.stack([u, v, c], 1).astype(np.int32))).cuda())
    cur = torch.cuda.current_stream()
    # rows keep enough free slots for every insert of these batches (the
    # allocation-free path cannot re-lay rows; that case is tested below)
    opt = dict(stream=cur, device=0, insert_slack_min=24)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, **opt) as A, \
            mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, **opt) as B:
        want = o.static()
        assert A.maxflow() == B.maxflow() == want
        for i, b in enumerate(batches):
            a_val = A.apply_batch_device(b)
            b_val = B.apply_batch_device_noalloc(b)
            want = o.apply(*[x.cpu().numpy() for x in b.unbind(1)])
            assert a_val == b_val == want, (i, a_val, b_val, want)
            side, cut = B.min_cut()
            assert cut == want and side[g.s] == 1 and side[g.t] == 0


def test_noalloc_limits_change_nothing():
    import torch
    g, stream, k, _ = gen.workload("er2000")
    cur = torch.cuda.current_stream()
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, stream=cur, device=0) as B:
        big = torch.zeros((mf.NOALLOC_MAX_UPDATES + 1, 3), dtype=torch.int32, device="cuda")
        # before the first solve
        with pytest.raises(mf.MFError) as ei:
            B.apply_batch_device_noalloc(big[:4])
        assert ei.value.status == mf.MF_ERR_STATE
        want = B.maxflow()
        with pytest.raises(mf.MFError) as ei:
            B.apply_batch_device_noalloc(big)
        assert ei.value.status == mf.MF_ERR_INVALID
        assert B.min_cut()[1] == want
    # a batch that inserts more pairs than a row's free slots: nothing applied
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, stream=cur, device=0,
                         insert_slack_min=1, insert_slack_pct=1) as B:
        o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
        want = o.static()
        assert B.maxflow() == want
        u = np.zeros(40, np.int32)
        v = np.arange(1000, 1040, dtype=np.int32)
        c = np.full(40, 5, np.int32)
        keep = ~np.isin(v, g.dst[g.src == 0])
        u, v, c = u[keep], v[keep], c[keep]
        upd = torch.from_numpy(np.ascontiguousarray(np.stack([u, v, c], 1))).cuda()
        with pytest.raises(mf.MFError) as ei:
            B.apply_batch_device_noalloc(upd)
        assert ei.value.status == mf.MF_ERR_OUT_OF_MEMORY
        assert B.min_cut()[1] == want
        # the allocating entry point re-lays the rows and applies it
        assert B.apply_batch_device(upd) == o.apply(u, v, c)
