"""GPU checks of the residual-state invariants and of the failure paths.

Invariants (Section 3.1): between kernels every residual is >= 0, the two
residuals of a pair sum to its two capacities, every excess is its vertex's
net inflow and the excesses sum to zero; after a remove-invalid-edges round
(Algorithm 3) or a fresh relabel no residual slot is steep.  They are counted
on the device over every slot (mf_debug_check_invariants) after single
push-relabel and remove-invalid-edges rounds, after solves and after repairs.

Failure paths: an allocator that returns NULL gives MF_ERR_OUT_OF_MEMORY and
a handle that still solves exactly; an iteration cap of one global relabel
gives MF_ERR_NOT_CONVERGED.
"""
import ctypes as C

import numpy as np
import pytest

import oracle
import paper_2511_01235_amd as mf
from paper_2511_01235_amd import gen

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def device_ready():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"


SAFETY = ("negative_residuals", "pair_sums", "pair_links", "excess_mismatches", "excess_total",
          "heights_out_of_range")


def _safe(inv):
    bad = {k: inv[k] for k in SAFETY if inv[k] != 0}
    assert not bad, bad


@pytest.mark.parametrize("cap", [0, -1])
@pytest.mark.parametrize("name", ["er2000", "rmat12", "grid64"])
def test_invariants_between_kernels(name, cap):
    g, stream, k, _ = gen.workload(name)
    say("invariants", name, "cap", cap)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, bfs_cap=cap) as G:
        # zero flow as loaded
        inv = G.invariants()
        _safe(inv)
        assert inv["active"] == 0 and inv["steep_slots"] == 0
        # the preflow after source saturation and a fresh relabel (Algorithm 1)
        _, _, active = G.initial_labels()
        inv = G.invariants()
        _safe(inv)
        assert inv["steep_slots"] == 0
        assert inv["active"] == active.size > 0
        # rounds of push-relabel plus remove-invalid-edges over one worklist
        for r in range(6):
            G.debug_round(3)
            inv = G.invariants()
            _safe(inv)
            assert inv["steep_slots"] == 0, (r, inv)
        # a push-relabel round alone keeps the conservation invariants
        G.debug_round(1)
        _safe(G.invariants())
        # solve and repairs: no active vertex and no steep slot at the end
        assert G.maxflow() == o.static()
        inv = G.invariants()
        _safe(inv)
        assert inv["active"] == 0 and inv["steep_slots"] == 0
        for _ in range(3):
            u, v, c = stream.next_batch(k)
            want = o.apply(u, v, c)
            assert G.apply_batch(u, v, c) == want
            inv = G.invariants()
            _safe(inv)
            assert inv["active"] == 0 and inv["steep_slots"] == 0
            # the cut (after a relabel of its own when the repair ended after a round)
            side, cut = G.min_cut()
            assert cut == want and side[g.s] == 1 and side[g.t] == 0
            _safe(G.invariants())


class FailingAllocator:
    """Device memory from torch's caching allocator; returns NULL while
    `fail` is set, or at the allocation numbered `fail_at`."""

    def __init__(self):
        import torch
        self.torch = torch
        self.live = {}
        self.calls = 0
        self.fail = False
        self.fail_at = None

        def _alloc(nbytes, ctx):
            n = self.calls
            self.calls += 1
            if self.fail or n == self.fail_at:
                return None
            p = torch.cuda.caching_allocator_alloc(int(nbytes), 0)
            self.live[p] = nbytes
            return p

        def _free(ptr, ctx):
            self.live.pop(ptr)
            torch.cuda.caching_allocator_delete(ptr)

        self.alloc_fn = mf.ALLOC_FN(_alloc)
        self.free_fn = mf.FREE_FN(_free)


def test_allocation_failure_leaves_handle_usable():
    import torch
    g, stream, _, _ = gen.workload("er2000")
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    A = FailingAllocator()
    # a load whose k-th allocation fails returns OUT_OF_MEMORY and gives back the rest
    for k in (0, 1, 5, 12):
        A.fail_at, A.calls = k, 0
        with pytest.raises(mf.MFError) as ei:
            mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, allocator=A, device=0)
        assert ei.value.status == mf.MF_ERR_OUT_OF_MEMORY, k
        assert not A.live, (k, len(A.live))
    A.fail_at = None
    stream_t = torch.cuda.current_stream()
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, allocator=A, device=0, stream=stream_t) as G:
        # the first solve's loop buffers cannot be had: nothing changes
        A.fail = True
        with pytest.raises(mf.MFError) as ei:
            G.maxflow()
        assert ei.value.status == mf.MF_ERR_OUT_OF_MEMORY
        A.fail = False
        assert G.maxflow() == o.static()
        # a batch larger than the update buffers: their growth fails, nothing is applied
        u, v, c = stream.next_batch(3000)
        A.fail = True
        with pytest.raises(mf.MFError) as ei:
            G.apply_batch(u, v, c)
        assert ei.value.status == mf.MF_ERR_OUT_OF_MEMORY
        A.fail = False
        side, cut = G.min_cut()
        assert cut == o.static()
        want = o.apply(u, v, c)
        assert G.apply_batch(u, v, c) == want
        side, cut = G.min_cut()
        assert cut == want
    assert not A.live


def test_iteration_cap_not_converged():
    g, stream, k, _ = gen.workload("grid64")
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, max_iterations=1) as G:
        with pytest.raises(mf.MFError) as ei:
            G.maxflow()
        assert ei.value.status == mf.MF_ERR_NOT_CONVERGED
        # no repair, cut or flow without a finished solve
        u, v, c = stream.next_batch(k)
        with pytest.raises(mf.MFError) as ei:
            G.apply_batch(u, v, c)
        assert ei.value.status == mf.MF_ERR_STATE
        with pytest.raises(mf.MFError) as ei:
            G.min_cut()
        assert ei.value.status == mf.MF_ERR_STATE
        # the same handle with the default cap solves exactly
        G.tune(max_iterations=0)
        assert G.maxflow() == o.static()
        assert G.apply_batch(u, v, c) == o.apply(u, v, c)
