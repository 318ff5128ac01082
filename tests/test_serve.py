"""The serving loop (paper_2511_01235_amd.serve).

CPU tests drive the scheduler with handles that wrap the oracle, so that
admission, least-recently-used eviction, re-admission from read-back
capacities and per-graph ordering are checked without a GPU.  The GPU test
serves a Poisson trace over real library handles under an HBM budget that
forces evictions, and checks every answer against the oracle applying each
graph's batches in arrival order.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2511_01235_amd import gen
from paper_2511_01235_amd.serve import Server, estimate_device_bytes


class OracleHandle:
    """Stands in for a device handle: the oracle solves, a dict keeps the
    merged capacities for get_edges, and a short sleep lets slots overlap."""

    def __init__(self, n, src, dst, cap, s, t):
        self.caps = {}
        for a, b, c in zip(np.asarray(src).tolist(), np.asarray(dst).tolist(), np.asarray(cap).tolist()):
            self.caps[(a, b)] = self.caps.get((a, b), 0) + c
        self.o = oracle.DynOracle(n, src, dst, cap, s, t)
        self.n = n
        self.closed = False
        self.offloaded = False

    def offload(self):
        assert not self.offloaded
        self.offloaded = True

    def restore(self):
        assert self.offloaded
        self.offloaded = False

    def maxflow(self):
        return self.o.static()

    def apply_batch(self, u, v, c):
        assert not self.closed and not self.offloaded
        time.sleep(0.002)
        for a, b, x in zip(u.tolist(), v.tolist(), c.tolist()):
            self.caps[(a, b)] = x
        return self.o.apply(u, v, c)

    def get_edges(self):
        items = sorted((k, c) for k, c in self.caps.items() if c > 0)
        src = np.array([k[0] for k, _ in items], np.int32)
        dst = np.array([k[1] for k, _ in items], np.int32)
        cap = np.array([c for _, c in items], np.int32)
        return src, dst, cap

    def stats(self):
        return {"device_bytes": estimate_device_bytes(self.n, len(self.caps))}

    def close(self):
        self.closed = True
        self.o.close()


def _fleet(count, seed, n_lo=40, n_hi=160):
    rng = gen.rng_for(seed)
    graphs = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi))
        graphs.append(gen.erdos_renyi(n, 5 * n, 50, seed=seed + 1 + i, name=f"er_{i}"))
    return graphs


def _trace(graphs, seed, count, rate, k_hi):
    streams = [gen.BatchStream(g, seed + 100 * i, inc_max=30, new_cap_max=50) for i, g in enumerate(graphs)]
    return gen.serving_trace(streams, rate=rate, count=count, seed=seed, k_lo=1, k_hi=k_hi)


def _expected(graphs, trace):
    """Each graph's batches applied in arrival order by a fresh oracle."""
    orc = [oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t) for g in graphs]
    for o in orc:
        o.static()
    want = [orc[gi].apply(u, v, c) for gi, _, u, v, c in trace]
    for o in orc:
        o.close()
    return want


def _check_order(server):
    by_graph = {}
    for r in server.requests:
        by_graph.setdefault(r.graph, []).append(r)
    for rs in by_graph.values():
        rs.sort(key=lambda r: r.arrival)
        for a, b in zip(rs, rs[1:]):
            assert a.done <= b.start, "a graph's requests overlapped or ran out of order"


@pytest.mark.parametrize("evict", ["offload", "rebuild"])
@pytest.mark.parametrize("slots,budget_graphs", [(1, 2), (3, 2), (4, 100)])
def test_serving_matches_sequential_oracle(slots, budget_graphs, evict):
    graphs = _fleet(6, 7100)
    trace = _trace(graphs, 7200, count=50, rate=2000.0, k_hi=40)
    want = _expected(graphs, trace)
    biggest = max(estimate_device_bytes(g.n, g.m) for g in graphs)
    budget = budget_graphs * biggest + biggest // 2
    with Server(graphs, budget, slots=slots, factory=OracleHandle, evict=evict) as srv:
        res = srv.run(trace)
        got = [r.value for r in srv.requests]
        assert got == want
        _check_order(srv)
        assert res["peak_resident_bytes"] <= budget
        touched = len({t[0] for t in trace})
        if budget_graphs < len(graphs):
            assert res["evictions"] > 0
            if evict == "offload":
                assert res["loads"] == touched     # every re-admission is a restore
            else:
                assert res["loads"] >= touched and res["restores"] == 0
        else:
            assert res["evictions"] == 0 and res["loads"] == touched


@pytest.mark.parametrize("evict", ["offload", "rebuild"])
def test_serving_after_preload(evict):
    graphs = _fleet(5, 7050)
    trace = _trace(graphs, 7060, count=30, rate=3000.0, k_hi=30)
    want = _expected(graphs, trace)
    biggest = max(estimate_device_bytes(g.n, g.m) for g in graphs)
    with Server(graphs, 2 * biggest, slots=3, factory=OracleHandle, evict=evict) as srv:
        loaded = srv.preload(threads=2)
        assert loaded == len(graphs) if evict == "offload" else 1 <= loaded < len(graphs)
        assert srv.resident_bytes <= srv.budget
        res = srv.run(trace)
        assert [r.value for r in srv.requests] == want
        assert res["peak_resident_bytes"] <= srv.budget
        _check_order(srv)


@pytest.mark.parametrize("max_wait", [0.0, 10.0])
def test_residency_first_with_aging(max_wait):
    """Room for one graph: graph 0 is resident, graph 1's request came first.
    With no aging allowance it is admitted first; with a long one the
    resident graph's requests go first and graph 1 waits for them."""
    graphs = _fleet(2, 7900)
    streams = [gen.BatchStream(g, 7950 + i, inc_max=30, new_cap_max=50) for i, g in enumerate(graphs)]
    sizes = [estimate_device_bytes(g.n, g.m) for g in graphs]
    with Server(graphs, max(sizes) + min(sizes) // 2, slots=1, factory=OracleHandle, max_wait=max_wait) as srv:
        srv.preload(threads=1)
        res = [i for i in range(2) if srv.g[i].resident]
        assert len(res) == 1
        res, other = res[0], 1 - res[0]
        trace = [(other, 0.0, *streams[other].next_batch(5))] + \
                [(res, 0.0, *streams[res].next_batch(5)) for _ in range(6)]
        want = _expected(graphs, trace)
        srv.run(trace)
        assert [r.value for r in srv.requests] == want
        first = min(srv.requests, key=lambda r: r.start)
        assert first.graph == (other if max_wait == 0.0 else res)
        _check_order(srv)


def test_fifo_policy_serves_in_arrival_order():
    """policy="fifo": with room for one graph and one slot, requests that
    alternate between two graphs run in arrival order (each one evicting the
    other graph), where residency-first would group them by graph."""
    graphs = _fleet(2, 7960)
    streams = [gen.BatchStream(g, 7970 + i, inc_max=30, new_cap_max=50) for i, g in enumerate(graphs)]
    sizes = [estimate_device_bytes(g.n, g.m) for g in graphs]
    trace = [(i % 2, 0.0, *streams[i % 2].next_batch(5)) for i in range(6)]
    want = _expected(graphs, trace)
    with Server(graphs, max(sizes) + min(sizes) // 2, slots=1, factory=OracleHandle, policy="fifo") as srv:
        srv.run(trace)
        assert [r.value for r in srv.requests] == want
        order = sorted(range(len(srv.requests)), key=lambda i: srv.requests[i].start)
        assert order == list(range(6))
    with pytest.raises(ValueError):
        Server(graphs, 1 << 40, factory=OracleHandle, policy="lifo")


def test_serving_honours_arrival_times():
    graphs = _fleet(2, 7300)
    trace = _trace(graphs, 7400, count=6, rate=50.0, k_hi=10)
    with Server(graphs, 1 << 40, slots=2, factory=OracleHandle) as srv:
        srv.run(trace)
        for r in srv.requests:
            assert r.start >= r.arrival


def test_serving_rejects_graph_above_budget():
    graphs = _fleet(2, 7500)
    with pytest.raises(MemoryError):
        Server(graphs, 1000, factory=OracleHandle)


def test_serving_surfaces_errors():
    graphs = _fleet(2, 7600)
    bad = [(0, 0.0, np.array([0], np.int32), np.array([0], np.int32), np.array([5], np.int32))]
    with Server(graphs, 1 << 40, slots=2, factory=OracleHandle) as srv:
        with pytest.raises(ValueError):
            srv.run(bad)


@pytest.mark.gpu
@pytest.mark.parametrize("evict", ["offload", "rebuild"])
def test_serving_gpu_matches_oracle(evict):
    import torch
    assert torch.cuda.is_available()
    graphs = gen.batched_graphs(8, seed=7700, n_lo=500, n_hi=20000, degree=8)
    trace = _trace(graphs, 7800, count=80, rate=5000.0, k_hi=400)
    want = _expected(graphs, trace)
    sizes = sorted(estimate_device_bytes(g.n, g.m) for g in graphs)
    budget = sum(sizes[-3:])          # room for about three graphs at a time
    print("[gpu] serving", len(graphs), "graphs", len(trace), "requests budget", budget, flush=True)
    with Server(graphs, budget, slots=4, evict=evict) as srv:
        res = srv.run(trace)
        print("[gpu] serving", res, flush=True)
        assert [r.value for r in srv.requests] == want
        _check_order(srv)
        assert res["evictions"] > 0
