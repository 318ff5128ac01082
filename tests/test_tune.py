"""The autotuner (paper_2511_01235_amd.tune): its search and its repeatable
trials.  CPU tests drive it with an oracle-backed stand-in for a handle; the
GPU tests tune real handles and check that values stay the oracle's."""
import numpy as np
import pytest

import oracle
from paper_2511_01235_amd import gen, tune


class OracleGraph:
    """Quacks like MaxFlowGraph for the tuner: apply_batch / get_edges / stats
    / tune, answers from the oracle; records every tuning it is given."""

    def __init__(self, g):
        self.n, self.s, self.t = g.n, g.s, g.t
        self.o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
        self.value = self.o.static()
        self.caps = {}
        for a, b, c in zip(g.src.tolist(), g.dst.tolist(), g.cap.tolist()):
            self.caps[(a, b)] = self.caps.get((a, b), 0) + c
        self.tunings = []

    def apply_batch(self, u, v, c):
        if len(u):
            for a, b, x in zip(u.tolist(), v.tolist(), c.tolist()):
                self.caps[(a, b)] = x
            self.value = self.o.apply(u, v, c)
        return self.value

    def get_edges(self):
        items = sorted((k, c) for k, c in self.caps.items() if c > 0)
        return (np.array([k[0] for k, _ in items], np.int32), np.array([k[1] for k, _ in items], np.int32),
                np.array([c for _, c in items], np.int32))

    def stats(self):
        return {"kernel_cycles": 8}

    def tune(self, **kw):
        self.tunings.append(kw)


def test_configs_start_with_defaults_and_respect_bins():
    cs = tune._configs(tune.GRAPH_SPACE, 20, 3)
    assert len(cs) == 20 and cs[0] == {k: tune.DEFAULTS[k] for k in tune.GRAPH_SPACE}
    assert all(c["bin_wave_max"] >= c["bin_thread_max"] for c in cs)
    assert len({tuple(sorted(c.items())) for c in cs}) == len(cs)


def test_halving_keeps_the_fastest():
    cfgs = [{"x": i} for i in range(27)]
    best, ms, table, trials = tune._halving(cfgs, lambda c, t: abs(c["x"] - 11) + 0.01 * t, rounds=4)
    assert best == {"x": 11}
    assert trials == 27 + 9 * 2 + 3 * 4 + 1 * 8


def test_pairs_restore_capacities():
    g, _, k, _ = gen.workload("er2000")
    mk = tune._PairMaker(g.n, g.src, g.dst, g.cap, g.s, g.t)
    (u, v, c), (u2, v2, old) = mk.draw(k, 5)
    model = {}
    for a, b, x in zip(g.src.tolist(), g.dst.tolist(), g.cap.tolist()):
        model[(a, b)] = model.get((a, b), 0) + x
    before = dict(model)
    for a, b, x in zip(u.tolist(), v.tolist(), c.tolist()):
        model[(a, b)] = x
    assert model != before
    for a, b, x in zip(u2.tolist(), v2.tolist(), old.tolist()):
        model[(a, b)] = x
    assert {k: x for k, x in model.items() if x} == {k: x for k, x in before.items() if x}
    # a second draw starts again from the same capacities
    (u3, _, _), _ = mk.draw(k, 5)
    assert np.array_equal(u3, u)


def test_tune_graph_on_oracle_stand_in():
    g, _, k, _ = gen.workload("er2000")
    G = OracleGraph(g)
    v0 = G.value
    res = tune.tune_graph(G, k, sample=9, rounds=3)
    assert res["trials"] == 9 + 3 * 2 + 1 * 4
    assert G.tunings[-1] == res["options"] and res["options"]["kernel_cycles"] >= 1
    assert G.value == v0


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["rmat12", "grid64"])
def test_tune_graph_gpu_keeps_values(name):
    import paper_2511_01235_amd as mf
    g, stream, k, _ = gen.workload(name)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t) as G:
        assert G.maxflow() == o.static()
        res = tune.tune_graph(G, k, sample=12, rounds=2)
        print("[gpu] tuned", name, res, flush=True)
        for _ in range(3):
            b = stream.next_batch(k)
            assert G.apply_batch(*b) == o.apply(*b)


@pytest.mark.gpu
def test_tune_batch_gpu_keeps_values():
    import paper_2511_01235_amd as mf
    graphs = gen.batched_graphs(8, seed=79500, n_lo=500, n_hi=5e3)
    want = [oracle.max_flow(g.n, g.src, g.dst, g.cap, g.s, g.t) for g in graphs]
    with mf.MaxFlowBatch(graphs) as B:
        assert B.maxflow().tolist() == want
        res = tune.tune_batch(B, graphs, sample=12, rounds=2)
        print("[gpu] tuned batch", res, flush=True)
        assert B.maxflow().tolist() == want
