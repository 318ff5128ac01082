"""Pins for the CPU oracle against facts fixed outside it.

Every check here compares the oracle with something it does not compute
itself: hand-derived values (tests/golden), the min-cut definition by
enumeration, closed forms, third-party solvers (scipy's Dinic and
Edmonds-Karp, networkx's Hopcroft-Karp), and the flow/cut certificate of the
paper's correctness proofs (Sections 3.1 and 4.3).
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2511_01235_amd import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def _arrays(edges):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 3)
    return e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), e[:, 2].astype(np.int32)


def _scipy_value(n, src, dst, cap, s, t, method):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import maximum_flow
    key = src.astype(np.int64) * n + dst
    uk, inv = np.unique(key, return_inverse=True)
    c = np.bincount(inv, weights=cap.astype(np.float64)).astype(np.int32)
    mat = csr_matrix((c, ((uk // n).astype(np.int32), (uk % n).astype(np.int32))), shape=(n, n))
    return int(maximum_flow(mat, s, t, method=method).flow_value)


def _random_small(rng, n, m, cap_max, zero_frac=0.1):
    u = rng.integers(0, n, size=m)
    v = rng.integers(0, n, size=m)
    keep = u != v
    u, v = u[keep], v[keep]
    c = rng.integers(1, cap_max + 1, size=u.size)
    c[rng.random(u.size) < zero_frac] = 0
    return u.astype(np.int32), v.astype(np.int32), c.astype(np.int32)


def _all_values(n, src, dst, cap, s, t):
    ek, flow, side = oracle.edmonds_karp(n, src, dst, cap, s, t)
    fifo = oracle.max_flow(n, src, dst, cap, s, t)
    return ek, fifo, flow, side


# --- golden, hand-derived ----------------------------------------------------

def test_golden_static():
    data = json.load(open(GOLDEN))
    for case in data["static"]:
        src, dst, cap = _arrays(case["edges"])
        n, s, t = case["n"], case["s"], case["t"]
        ek, fifo, flow, side = _all_values(n, src, dst, cap, s, t)
        assert oracle.brute_min_cut(n, src, dst, cap, s, t) == case["expected"], case["name"]
        assert ek == case["expected"] and fifo == case["expected"], case["name"]
        assert oracle.cert_check(n, src, dst, cap, s, t, flow, side, ek) == (0, "")


def test_golden_dynamic():
    data = json.load(open(GOLDEN))
    for case in data["dynamic"]:
        src, dst, cap = _arrays(case["edges"])
        n, s, t = case["n"], case["s"], case["t"]
        o = oracle.DynOracle(n, src, dst, cap, s, t)
        assert o.static() == case["initial"]
        for batch, want in zip(case["batches"], case["expected"]):
            u, v, c = _arrays(batch)
            assert o.apply(u, v, c) == want, case["name"]


# --- the min-cut definition, by enumeration -----------------------------------

@pytest.mark.parametrize("seed", range(40))
def test_brute_force_small(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(2, 11))
    m = int(rng.integers(0, 4 * n))
    src, dst, cap = _random_small(rng, n, m, 20)
    s = int(rng.integers(0, n))
    t = int((s + 1 + rng.integers(0, n - 1)) % n)
    want = oracle.brute_min_cut(n, src, dst, cap, s, t)
    ek, fifo, flow, side = _all_values(n, src, dst, cap, s, t)
    assert ek == want and fifo == want
    assert oracle.cert_check(n, src, dst, cap, s, t, flow, side, want) == (0, "")
    o = oracle.DynOracle(n, src, dst, cap, s, t)
    assert o.static() == want
    cut_side, cut_cap = o.min_cut()
    assert cut_cap == want
    assert oracle.cert_check(n, src, dst, cap, s, t, None, cut_side, want)[0] == 0


def test_brute_force_sixteen_vertices():
    rng = np.random.default_rng(77)
    for _ in range(3):
        src, dst, cap = _random_small(rng, 16, 60, 30)
        want = oracle.brute_min_cut(16, src, dst, cap, 0, 15)
        assert oracle.max_flow(16, src, dst, cap, 0, 15) == want
        assert oracle.edmonds_karp(16, src, dst, cap, 0, 15)[0] == want


# --- closed forms ------------------------------------------------------------

def test_single_edge_and_parallel_edges():
    for c in (0, 1, 7, 2**31 - 1):
        src, dst, cap = _arrays([[0, 1, c]])
        assert oracle.max_flow(2, src, dst, cap, 0, 1) == c
    src, dst, cap = _arrays([[0, 1, 3], [0, 1, 4], [0, 1, 5], [1, 0, 100]])
    assert oracle.max_flow(2, src, dst, cap, 0, 1) == 12


def test_path_is_its_minimum():
    rng = np.random.default_rng(5)
    for L in (1, 2, 5, 30):
        caps = rng.integers(1, 1000, size=L)
        edges = [[i, i + 1, int(caps[i])] for i in range(L)]
        src, dst, cap = _arrays(edges)
        assert oracle.max_flow(L + 1, src, dst, cap, 0, L) == int(caps.min())


def test_disjoint_paths_sum_of_minima():
    rng = np.random.default_rng(6)
    k, L = 7, 5
    n = 2 + k * L
    edges, total = [], 0
    for p in range(k):
        ids = [0] + [2 + p * L + i for i in range(L)] + [1]
        caps = rng.integers(1, 100, size=len(ids) - 1)
        total += int(caps.min())
        edges += [[ids[i], ids[i + 1], int(caps[i])] for i in range(len(ids) - 1)]
    src, dst, cap = _arrays(edges)
    assert oracle.max_flow(n, src, dst, cap, 0, 1) == total
    assert oracle.edmonds_karp(n, src, dst, cap, 0, 1)[0] == total


@pytest.mark.parametrize("W,c", [(4, 5), (16, 37), (32, 100)])
def test_uniform_grid_is_width_times_capacity(W, c):
    g = gen.grid(W, 100, seed=1)
    cap = np.where(g.cap == 1000, 1000, c).astype(np.int32)
    assert oracle.max_flow(g.n, g.src, g.dst, cap, g.s, g.t) == W * c


def test_bipartite_matching_networkx():
    nx = pytest.importorskip("networkx")
    rng = np.random.default_rng(9)
    L, R = 40, 35
    B = nx.Graph()
    B.add_nodes_from(range(L), bipartite=0)
    B.add_nodes_from(range(L, L + R), bipartite=1)
    pairs = {(int(a), int(L + b)) for a, b in zip(rng.integers(0, L, 120), rng.integers(0, R, 120))}
    B.add_edges_from(pairs)
    match = nx.bipartite.hopcroft_karp_matching(B, top_nodes=range(L))
    size = len(match) // 2
    s, t = L + R, L + R + 1
    edges = [[s, a, 1] for a in range(L)] + [[a, b, 1] for a, b in pairs] + \
            [[L + b, t, 1] for b in range(R)]
    src, dst, cap = _arrays(edges)
    assert oracle.max_flow(L + R + 2, src, dst, cap, s, t) == size


def test_bounds_out_of_source_into_sink():
    rng = np.random.default_rng(12)
    for _ in range(20):
        src, dst, cap = _random_small(rng, 30, 150, 50)
        v = oracle.max_flow(30, src, dst, cap, 0, 29)
        assert v <= cap[src == 0].sum() and v <= cap[dst == 29].sum()


# --- third-party solvers -----------------------------------------------------

@pytest.mark.parametrize("name", ["er2000", "rmat12", "grid64"])
def test_scipy_agrees(name):
    g, _, _, _ = gen.workload(name)
    fifo = oracle.max_flow(g.n, g.src, g.dst, g.cap, g.s, g.t)
    assert fifo == _scipy_value(g.n, g.src, g.dst, g.cap, g.s, g.t, "dinic")
    assert fifo == _scipy_value(g.n, g.src, g.dst, g.cap, g.s, g.t, "edmonds_karp")
    if name != "rmat12":
        ek, flow, side = oracle.edmonds_karp(g.n, g.src, g.dst, g.cap, g.s, g.t)
        assert ek == fifo
        assert oracle.cert_check(g.n, g.src, g.dst, g.cap, g.s, g.t, flow, side, ek) == (0, "")


# --- certificate checker catches planted mistakes ------------------------------

def test_cert_check_rejects_broken_flows():
    data = json.load(open(GOLDEN))
    case = data["static"][0]
    src, dst, cap = _arrays(case["edges"])
    n, s, t = case["n"], case["s"], case["t"]
    ek, flow, side = oracle.edmonds_karp(n, src, dst, cap, s, t)
    assert oracle.cert_check(n, src, dst, cap, s, t, flow, side, ek)[0] == 0
    internal = np.flatnonzero((src != s) & (dst != t) & (src != t) & (dst != s) & (flow < cap))
    bad = flow.copy()
    bad[internal[0]] += 1                # conservation breaks at both ends, value unchanged
    assert oracle.cert_check(n, src, dst, cap, s, t, bad, side, ek)[0] == 2
    over = flow.copy()
    i = int(np.argmax(cap - flow == 0))  # a saturated edge
    over[i] = cap[i] + 1
    assert oracle.cert_check(n, src, dst, cap, s, t, over, None, ek)[0] == 1
    assert oracle.cert_check(n, src, dst, cap, s, t, flow, None, ek + 1)[0] == 3
    wrong = side.copy()
    wrong[t] = 1
    assert oracle.cert_check(n, src, dst, cap, s, t, None, wrong, ek)[0] == 4
    other = np.zeros(n, np.uint8)
    other[s] = 1                          # cut {s} has capacity 20 != 19
    assert oracle.cert_check(n, src, dst, cap, s, t, None, other, ek)[0] == 4


# --- dynamic: repair == from scratch, after every batch -------------------------

class _CapModel:
    """Independent bookkeeping of the current capacity function."""

    def __init__(self, n, src, dst, cap):
        self.n = n
        self.c = {}
        for a, b, x in zip(src.tolist(), dst.tolist(), cap.tolist()):
            self.c[(a, b)] = self.c.get((a, b), 0) + x

    def apply(self, u, v, c):
        for a, b, x in zip(u.tolist(), v.tolist(), c.tolist()):
            self.c[(a, b)] = x

    def arrays(self):
        items = sorted(self.c.items())
        if not items:
            return (np.zeros(0, np.int32),) * 3
        e = np.array([[a, b, x] for (a, b), x in items], dtype=np.int64)
        return e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), e[:, 2].astype(np.int32)


@pytest.mark.parametrize("seed", range(25))
def test_dynamic_equals_from_scratch_small(seed):
    rng = np.random.default_rng(5000 + seed)
    n = int(rng.integers(3, 12))
    src, dst, cap = _random_small(rng, n, 3 * n, 15)
    s, t = 0, n - 1
    o = oracle.DynOracle(n, src, dst, cap, s, t)
    model = _CapModel(n, src, dst, cap)
    prev = o.static()
    assert prev == oracle.brute_min_cut(n, src, dst, cap, s, t)
    for b in range(6):
        k = int(rng.integers(1, 10))
        pairs = np.array(list(model.c.keys()), dtype=np.int64).reshape(-1, 2)
        u, v, c = gen.random_batch(n, k, 15, seed=seed * 100 + b, pairs=pairs)
        if b % 3 == 1:   # s and t edges in the batch
            u[0], v[-1] = s, t
            v[0] = v[0] if v[0] != s else (s + 1) % n
            u[-1] = u[-1] if u[-1] != t else (t + 1) % n
        old = dict(model.c)
        model.apply(u, v, c)
        ms, md, mc = model.arrays()
        want = oracle.brute_min_cut(n, ms, md, mc, s, t)
        got = o.apply(u, v, c)
        assert got == want
        assert oracle.edmonds_karp(n, ms, md, mc, s, t)[0] == want
        side, cut = o.min_cut()
        assert cut == want
        assert oracle.cert_check(n, ms, md, mc, s, t, None, side, want)[0] == 0
        delta = sum(abs(model.c[p] - old.get(p, 0)) for p in model.c)
        assert abs(got - prev) <= delta
        prev = got


@pytest.mark.parametrize("direction", ["increase", "decrease"])
def test_dynamic_monotone(direction):
    g, _, _, _ = gen.workload("rmat12")
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    model = _CapModel(g.n, g.src, g.dst, g.cap)
    prev = o.static()
    rng = np.random.default_rng(3)
    for b in range(4):
        pairs = [p for p, x in model.c.items() if x > 0]
        pick = rng.choice(len(pairs), size=200, replace=False)
        u = np.array([pairs[i][0] for i in pick], np.int32)
        v = np.array([pairs[i][1] for i in pick], np.int32)
        old = np.array([model.c[pairs[i]] for i in pick], np.int64)
        if direction == "increase":
            c = old + rng.integers(1, 50, size=old.size)
        else:
            c = rng.integers(0, old)
        c = c.astype(np.int32)
        model.apply(u, v, c)
        got = o.apply(u, v, c)
        assert (got >= prev) if direction == "increase" else (got <= prev)
        ms, md, mc = model.arrays()
        assert got == oracle.max_flow(g.n, ms, md, mc, g.s, g.t)
        assert got == _scipy_value(g.n, ms, md, mc, g.s, g.t, "dinic")
        prev = got


@pytest.mark.parametrize("name", ["er2000", "rmat12", "grid64"])
def test_dynamic_workload_streams(name):
    g, stream, k, nb = gen.workload(name)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    o.static()
    for b in range(min(nb, 5)):
        u, v, c = stream.next_batch(k)
        got = o.apply(u, v, c)
        cs, cd, cc = stream.current_edges()
        assert got == _scipy_value(g.n, cs, cd, cc, g.s, g.t, "dinic")
        e, h = o.state()
        side, cut = o.min_cut()
        assert cut == got


def test_state_invariants_after_static():
    g, _, _, _ = gen.workload("rmat12")
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    val = o.static()
    u, v, c, f = o.pairs()
    assert (f >= 0).all() and (f <= c).all()
    e, h = o.state()
    inflow = np.bincount(v, weights=f, minlength=g.n) - np.bincount(u, weights=f, minlength=g.n)
    assert np.array_equal(inflow.astype(np.int64), e)
    others = np.ones(g.n, bool)
    others[[g.s, g.t]] = False
    assert (e[others] >= 0).all()
    assert e[g.t] == val


def test_initial_labels_are_bfs_distances():
    """Heights after saturation = hop distance to t over residual arcs,
    checked against scipy's unweighted shortest paths on the reversed graph."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    g, _, _, _ = gen.workload("er2000")
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    h, e = o.initial_labels()
    # residual arcs after saturating s: every edge (u,v) not out of s with
    # cap > 0, plus (v,s) for every saturated (s,v)
    keep = (g.src != g.s) & (g.cap > 0)
    ru = np.concatenate([g.src[keep], g.dst[g.src == g.s]])
    rv = np.concatenate([g.dst[keep], g.src[g.src == g.s]])
    mat = csr_matrix((np.ones(ru.size), (rv, ru)), shape=(g.n, g.n))  # reversed
    d = shortest_path(mat, unweighted=True, indices=g.t)
    want = np.where(np.isinf(d), g.n, d).astype(np.int64)
    want[g.s] = g.n
    assert np.array_equal(h.astype(np.int64), want)
    assert e[g.t] == 0 and e[g.s] == -g.cap[g.src == g.s].sum()
