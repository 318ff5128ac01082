"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bit-exact comparisons (integer method): max-flow values after the static
solve and after every update batch; global-relabel heights (BFS distances are
unique); the active-vertex set.  The cut returned by mf_min_cut is checked as
a certificate: it separates s from t and its capacity equals the value.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2511_01235_amd as mf
from paper_2511_01235_amd import gen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
from test_oracle_pins import _CapModel, _arrays, _random_small  # noqa: E402


def say(*a):
    print("[gpu]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def device_ready():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    assert mf.mf_debug_selftest(-1) == mf.MF_OK


def _cut_ok(g_n, s, t, side, cut, value, src, dst, cap):
    assert side[s] == 1 and side[t] == 0
    assert cut == value
    rc, msg = oracle.cert_check(g_n, src, dst, cap, s, t, None, side, value)
    assert rc == 0, msg


def _solve_both(n, src, dst, cap, s, t, **opt):
    want = oracle.max_flow(n, src, dst, cap, s, t)
    with mf.MaxFlowGraph(n, src, dst, cap, s, t, **opt) as g:
        got = g.maxflow()
        side, cut = g.min_cut()
    return want, got, side, cut


def test_selftest():
    assert mf.mf_debug_selftest(0) == mf.MF_OK


def test_atomic_probe_runs():
    for width in (4, 8):
        rate = mf.mf_debug_atomic_probe(1 << 20, width, 0)
        assert rate > 1e8, (width, rate)
    with pytest.raises(mf.MFError):
        mf.mf_debug_atomic_probe(0, 4, 0)


# --- global relabel and worklist, bit-exact -------------------------------------

@pytest.mark.parametrize("name", ["er2000", "rmat12", "grid64"])
def test_initial_labels_bit_exact(name):
    g, _, _, _ = gen.workload(name)
    say("initial labels", name, g.n, g.m)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    h_want, e_want = o.initial_labels()
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t) as G:
        h, e, active = G.initial_labels()
    assert np.array_equal(h, h_want)
    assert np.array_equal(e, e_want)
    others = np.ones(g.n, bool)
    others[[g.s, g.t]] = False
    want_active = np.flatnonzero(others & (e_want > 0) & (h_want < g.n))
    assert np.array_equal(np.sort(active), want_active)
    assert np.unique(active).size == active.size


@pytest.mark.parametrize("name", ["grid2048", "rmat20"])
def test_full_size_initial_labels_bit_exact(name):
    """Algorithm 1's initialisation and the first global relabel (Algorithms
    4 and 6) at the benchmark shapes: the 2,049-level grid BFS runs through
    the one-workgroup, cooperative and multi-block level kernels, the RMAT
    one through top-down and bottom-up levels.  Every height and excess
    equals the oracle's, and so does the active set."""
    g, _, _, _ = gen.workload(name)
    say("full-size initial labels", name, g.n, g.m)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    h_want, e_want = o.initial_labels()
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t) as G:
        h, e, active = G.initial_labels()
    bad = np.flatnonzero(h != h_want)
    assert bad.size == 0, (name, bad[:8], h[bad[:8]], h_want[bad[:8]])
    assert np.array_equal(e, e_want)
    others = np.ones(g.n, bool)
    others[[g.s, g.t]] = False
    want_active = np.flatnonzero(others & (e_want > 0) & (h_want < g.n))
    assert np.array_equal(np.sort(active), want_active)


@pytest.mark.parametrize("variant", ["rows4", "rows8", "slots"])
@pytest.mark.parametrize("name", ["er2000", "rmat12", "grid64"])
def test_bottom_up_levels_bit_exact(name, variant):
    """Every BFS level bottom-up (per-row early exit with four or eight loads
    in flight, or slot-parallel rows): heights bit-exact to the oracle's BFS,
    and the dynamic values too."""
    opts = dict(bfs_alpha=1000000, bfs_beta=1000000,
                bfs_bottom_up={"rows4": 0, "rows8": 1, "slots": 2}[variant],
                bfs_narrow_slots=-1, bfs_medium_slots=-1)   # every level through the multi-block kernels
    g, stream, k, _ = gen.workload(name)
    say("bottom-up levels", name, variant)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    h_want, _ = o.initial_labels()
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, **opts) as G:
        h, _, _ = G.initial_labels()
        assert np.array_equal(h, h_want)
        assert G.maxflow() == o.static()
        for _ in range(3):
            u, v, c = stream.next_batch(k)
            assert G.apply_batch(u, v, c) == o.apply(u, v, c)


@pytest.mark.parametrize("narrow", [0, -1, 16])
@pytest.mark.parametrize("scan", [0, 1])
@pytest.mark.parametrize("div", [1, 8, 1000000])
@pytest.mark.parametrize("name", ["grid64", "rmat12"])
def test_push_rounds_between_relabels(name, div, scan, narrow):
    """Push-relabel rounds on the current heights between global relabels
    (one per relabel up to one per BFS level), their worklists built from the
    previous one plus the activated vertices or by scanning every vertex,
    short lists run many rounds per launch in one workgroup (up to 2048 or 16
    vertices, or never): values equal the oracle's in the single-graph and
    the batched loops."""
    g, stream, k, _ = gen.workload(name)
    say("push rounds", name, "div", div, "scan", scan, "narrow", narrow)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    want = [o.static()]
    batches = [stream.next_batch(k) for _ in range(3)]
    want += [o.apply(*b) for b in batches]
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, round_div=div, round_scan=scan,
                         round_narrow=narrow) as G:
        got = [G.maxflow()] + [G.apply_batch(*b) for b in batches]
        if div == 1 and name == "grid64":
            assert G.stats()["last_rounds"] > G.stats()["last_iterations"]
    assert got == want
    if narrow:
        return  # the batched loop has no one-workgroup rounds
    with mf.MaxFlowBatch([g], round_div=div) as B:
        got_b = [int(B.maxflow()[0])] + [int(B.apply([b])[0]) for b in batches]
    assert got_b == want


@pytest.mark.parametrize("narrow", [0, 16, 4096, 1 << 30])
@pytest.mark.parametrize("name", ["er2000", "rmat12", "rmat14", "grid64", "grid256"])
def test_thin_frontier_levels_bit_exact(name, narrow):
    """BFS levels with frontiers of up to `narrow` slots run in one workgroup
    (0: never, 1 << 30: every level), handing larger ones to the multi-block
    kernels and taking them back: heights bit-exact, values equal."""
    g, stream, k, _ = gen.workload(name)
    say("thin frontiers", name, narrow)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    h_want, _ = o.initial_labels()
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, bfs_narrow_slots=narrow or -1) as G:
        h, _, _ = G.initial_labels()
        assert np.array_equal(h, h_want)
        assert G.maxflow() == o.static()
        for _ in range(3):
            u, v, c = stream.next_batch(k)
            assert G.apply_batch(u, v, c) == o.apply(u, v, c)


@pytest.mark.parametrize("cycles", [1, 2, 1000])
@pytest.mark.parametrize("name", ["rmat12", "er2000"])
def test_long_row_cycles_same_values(name, cycles):
    """Rows above bin_wave_max slots run `cycles` push/relabel cycles per
    launch (1000: capped at kernel_cycles); with bins of 4 and 8 slots most
    rows take that path.  Static value and repairs equal the oracle's."""
    g, stream, k, _ = gen.workload(name)
    say("long-row cycles", name, cycles)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, long_row_cycles=cycles,
                         bin_thread_max=4, bin_wave_max=8) as G:
        assert G.maxflow() == o.static()
        for _ in range(3):
            u, v, c = stream.next_batch(k)
            assert G.apply_batch(u, v, c) == o.apply(u, v, c)


@pytest.mark.parametrize("mode", ["ordinary", "queued", "pipelined"])
@pytest.mark.parametrize("name", ["er2000", "rmat12", "grid64"])
def test_queued_rounds_same_values(name, mode):
    """The worklist build and first two rounds queued behind the relabel's
    first chunk of levels (device-sized, guarded on the BFS having ended;
    grid64's BFS outlasts the first chunk, so its queued launches must do
    nothing), also with the next iteration queued before the host reads the
    last one's counters (shallow graphs), or everything launched after the
    host read the counters: static value and repairs equal the oracle's in
    every mode, cut certified."""
    opts = dict(queue_rounds=-1 if mode == "ordinary" else 1,
                pipeline=1 if mode == "pipelined" else -1)
    g, stream, k, _ = gen.workload(name)
    say("queued rounds", name, mode)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, **opts) as G:
        assert G.maxflow() == o.static()
        for _ in range(4):
            u, v, c = stream.next_batch(k)
            want = o.apply(u, v, c)
            assert G.apply_batch(u, v, c) == want
            side, cut = G.min_cut()
            assert cut == want


@pytest.mark.parametrize("capture", [1, -1])
@pytest.mark.parametrize("name", ["er2000", "rmat12"])
def test_pipelined_surplus_iteration_leaves_exact_cut(name, capture):
    """Pipelined iterations with a first chunk of one BFS level: the surplus
    iteration queued behind the last one must still finish its BFS (every
    pipelined iteration launches at least as many levels as the pipeline's
    depth limit), so the cut read after each call is the certified one:
    capacity equal to the value and a valid certificate, after the static
    solve and after every repair, replayed from a captured graph or launched
    kernel by kernel."""
    g, stream, k, _ = gen.workload(name)
    say("pipelined surplus", name, "capture", capture)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    cur = _CapModel(g.n, g.src, g.dst, g.cap)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, bfs_first_chunk=1, pipeline=1,
                         graph_capture=capture) as G:
        val = G.maxflow()
        assert val == o.static()
        for i in range(6):
            side, cut = G.min_cut()
            assert cut == val
            src, dst, cap = cur.arrays()
            _cut_ok(g.n, g.s, g.t, side, cut, val, src, dst, cap)
            u, v, c = stream.next_batch(k)
            cur.apply(u, v, c)
            val = G.apply_batch(u, v, c)
            assert val == o.apply(u, v, c), i


@pytest.mark.parametrize("medium", [-1, 65536, 1 << 30])
@pytest.mark.parametrize("name", ["er2000", "rmat12", "grid64"])
def test_mid_frontier_levels_bit_exact(name, medium):
    """Frontiers above the one-workgroup threshold and up to bfs_medium_slots
    slots run in one cooperative launch of a few workgroups with grid
    barriers (-1: never; 1 << 30: every level that is not thin), handing
    larger frontiers to the multi-block levels: heights bit-exact, static
    value and repairs equal the oracle's."""
    g, stream, k, _ = gen.workload(name)
    say("mid-size frontiers", name, medium)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    h_want, _ = o.initial_labels()
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, bfs_medium_slots=medium) as G:
        h, _, _ = G.initial_labels()
        assert np.array_equal(h, h_want)
        assert G.maxflow() == o.static()
        for _ in range(3):
            u, v, c = stream.next_batch(k)
            assert G.apply_batch(u, v, c) == o.apply(u, v, c)


# --- static value ---------------------------------------------------------------

def test_golden_static_gpu():
    import json
    data = json.load(open(os.path.join(HERE, "golden", "hand_examples.json")))
    for case in data["static"]:
        src, dst, cap = _arrays(case["edges"])
        say("golden", case["name"])
        want, got, side, cut = _solve_both(case["n"], src, dst, cap, case["s"], case["t"])
        assert got == want == case["expected"]
        _cut_ok(case["n"], case["s"], case["t"], side, cut, got, src, dst, cap)


@pytest.mark.parametrize("seed", range(30))
def test_static_tiny_vs_brute_force(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(2, 11))
    src, dst, cap = _random_small(rng, n, int(rng.integers(0, 4 * n)), 20)
    s = int(rng.integers(0, n))
    t = int((s + 1 + rng.integers(0, n - 1)) % n)
    say("tiny", seed, n, src.size)
    want = oracle.brute_min_cut(n, src, dst, cap, s, t)
    with mf.MaxFlowGraph(n, src, dst, cap, s, t) as G:
        got = G.maxflow()
        side, cut = G.min_cut()
    assert got == want
    _cut_ok(n, s, t, side, cut, got, src, dst, cap)


# every graph with the defaults; the option sweep on the smaller ones
_STATIC_CASES = [(name, {}) for name in ("er2000", "rmat12", "rmat16", "grid64", "grid256")] + [
    (name, opts) for opts in ({"kernel_cycles": 1}, {"kernel_cycles": 64}, {"topology_driven": True})
    for name in ("er2000", "rmat12", "grid64")]


@pytest.mark.parametrize("name,opts", _STATIC_CASES,
                         ids=[f"{n}-{'-'.join(f'{k}={v}' for k, v in o.items()) or 'defaults'}"
                              for n, o in _STATIC_CASES])
def test_static_workloads(name, opts):
    g, _, _, _ = gen.workload(name)
    say("static", name, opts)
    want, got, side, cut = _solve_both(g.n, g.src, g.dst, g.cap, g.s, g.t, **opts)
    assert got == want
    _cut_ok(g.n, g.s, g.t, side, cut, got, g.src, g.dst, g.cap)


@pytest.mark.parametrize("name", ["er2000", "rmat14", "grid64"])
def test_persistent_relabel_mode(name):
    """The cooperative single-launch global relabel gives the same values."""
    g, stream, k, nb = gen.workload(name)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, relabel_mode=1) as G:
        assert G.maxflow() == o.static()
        h, e, active = G.initial_labels()
        h_want, e_want = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t).initial_labels()
        assert np.array_equal(h, h_want)
        G.maxflow()
        for b in range(3):
            u, v, c = stream.next_batch(k)
            say("persistent", name, b)
            assert G.apply_batch(u, v, c) == o.apply(u, v, c)


def test_static_repeatable():
    g, _, _, _ = gen.workload("rmat14")
    want = oracle.max_flow(g.n, g.src, g.dst, g.cap, g.s, g.t)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t) as G:
        for r in range(5):
            say("repeat", r)
            assert G.maxflow() == want


def test_closed_forms_gpu():
    W, c = 32, 37
    g = gen.grid(W, 100, seed=1)
    cap = np.where(g.cap == 1000, 1000, c).astype(np.int32)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, cap, g.s, g.t) as G:
        assert G.maxflow() == W * c
    src, dst, cap = _arrays([[0, 1, 5], [1, 2, 3], [2, 3, 9]])
    with mf.MaxFlowGraph(4, src, dst, cap, 0, 3) as G:
        assert G.maxflow() == 3
    src, dst, cap = _arrays([[0, 1, 5], [2, 3, 3]])
    with mf.MaxFlowGraph(4, src, dst, cap, 0, 3) as G:
        assert G.maxflow() == 0
    with mf.MaxFlowGraph(4, np.zeros(0), np.zeros(0), np.zeros(0), 0, 3) as G:
        assert G.maxflow() == 0


# --- dynamic ---------------------------------------------------------------------

def test_golden_dynamic_gpu():
    import json
    data = json.load(open(os.path.join(HERE, "golden", "hand_examples.json")))
    for case in data["dynamic"]:
        src, dst, cap = _arrays(case["edges"])
        with mf.MaxFlowGraph(case["n"], src, dst, cap, case["s"], case["t"]) as G:
            assert G.maxflow() == case["initial"]
            for batch, want in zip(case["batches"], case["expected"]):
                u, v, c = _arrays(batch)
                assert G.apply_batch(u, v, c) == want


@pytest.mark.parametrize("seed", range(12))
def test_dynamic_tiny_adversarial(seed):
    rng = np.random.default_rng(5000 + seed)
    n = int(rng.integers(3, 12))
    src, dst, cap = _random_small(rng, n, 3 * n, 15)
    s, t = 0, n - 1
    model = _CapModel(n, src, dst, cap)
    say("dyn tiny", seed, n)
    with mf.MaxFlowGraph(n, src, dst, cap, s, t, insert_slack_min=1, insert_slack_pct=1) as G:
        assert G.maxflow() == oracle.brute_min_cut(n, src, dst, cap, s, t)
        for b in range(6):
            pairs = np.array(list(model.c.keys()), dtype=np.int64).reshape(-1, 2)
            u, v, c = gen.random_batch(n, int(rng.integers(1, 12)), 15, seed=seed * 100 + b,
                                       pairs=pairs)
            model.apply(u, v, c)
            ms, md, mc = model.arrays()
            want = oracle.brute_min_cut(n, ms, md, mc, s, t)
            got = G.apply_batch(u, v, c)
            assert got == want, (seed, b)
            side, cut = G.min_cut()
            _cut_ok(n, s, t, side, cut, got, ms, md, mc)


@pytest.mark.parametrize("cap", [0, -1])
@pytest.mark.parametrize("warm", [False, True])
@pytest.mark.parametrize("name,batches", [("er2000", 10), ("rmat12", 8), ("rmat14", 5),
                                          ("grid64", 5), ("grid256", 3)])
def test_dynamic_workloads(name, batches, warm, cap):
    """Repairs against the oracle after every batch, cut certificates, with
    relabels that stop once every vertex with excess has its height (cap 0,
    the default) or run to the end (-1)."""
    g, stream, k, nb = gen.workload(name)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, warm_start=warm, bfs_cap=cap) as G:
        assert G.maxflow() == o.static()
        for b in range(min(batches, nb)):
            u, v, c = stream.next_batch(k)
            say("dyn", name, "batch", b, k)
            want = o.apply(u, v, c)
            got = G.apply_batch(u, v, c)
            assert got == want, (name, b)
            cs, cd, cc = stream.current_edges()
            side, cut = G.min_cut()
            _cut_ok(g.n, g.s, g.t, side, cut, got, cs, cd, cc)


def _comb_graph(side=64):
    """A side x side grid (4-connected, capacity 1000 both ways) drained into
    the sink t through one corner, and three vertices fed by the source at 10
    that each reach the grid at 5, about 80 hops from t: the excess needs more
    push-relabel rounds than one relabel's share (depth / 4), and every vertex
    with excess sits well short of the grid's far corner (127 hops)."""
    s, t, xs, base = 0, 1, [2, 3, 4], 5
    gid = lambda r, c: base + r * side + c
    src, dst, cap = [], [], []
    for r in range(side):
        for c in range(side):
            for dr, dc in ((0, 1), (1, 0)):
                if r + dr < side and c + dc < side:
                    src += [gid(r, c), gid(r + dr, c + dc)]
                    dst += [gid(r + dr, c + dc), gid(r, c)]
                    cap += [1000, 1000]
    src.append(gid(0, 0)); dst.append(t); cap.append(1000)
    for i, x in enumerate(xs):
        src += [s, x]; dst += [x, gid(40 + 5 * i, 40)]; cap += [10, 5]
    n = base + side * side
    feeds = np.array([gid(40 + 5 * i, 40) for i in range(3)], np.int32)
    return (n, s, t, xs, feeds, np.array(src, np.int32), np.array(dst, np.int32),
            np.array(cap, np.int32))


@pytest.mark.parametrize("narrow,medium", [(0, 0), (-1, 1 << 30), (-1, -1)])
def test_capped_relabel_stops_early(narrow, medium):
    """By default (bfs_cap) the relabels of a solve that follow a round stop once
    every vertex with excess below |V| has its height: on a graph whose
    excess sits well short of the BFS's far end some relabel stops early (in
    the one-workgroup levels, the cooperative mid-size levels or the
    multi-block levels), the value and the cut match the oracle's, and
    with bfs_cap = -1 no relabel stops."""
    n, s, t, xs, feeds, src, dst, cap = _comb_graph()
    o = oracle.DynOracle(n, src, dst, cap, s, t)
    want = o.static()
    assert want == 15
    for on in (0, -1):
        say("capped relabel", narrow, medium, on)
        with mf.MaxFlowGraph(n, src, dst, cap, s, t, bfs_cap=on, bfs_narrow_slots=narrow,
                             bfs_medium_slots=medium) as G:
            assert G.maxflow() == want
            capped = G.stats()["last_capped_relabels"]
            assert (capped >= 1) if on == 0 else (capped == 0), capped
            side, cut = G.min_cut()
            _cut_ok(n, s, t, side, cut, want, src, dst, cap)
    # a repair that raises the feeds: the graph handle and the oracle agree
    u, v = np.array(xs, np.int32), feeds
    c = np.array([10, 10, 10], np.int32)
    want = o.apply(u, v, c)
    assert want == 30
    with mf.MaxFlowGraph(n, src, dst, cap, s, t, bfs_narrow_slots=narrow,
                         bfs_medium_slots=medium) as G:
        G.maxflow()
        assert G.apply_batch(u, v, c) == want
        src2 = np.concatenate([src[:-6], np.array([s, xs[0], s, xs[1], s, xs[2]], np.int32)])
        dst2 = np.concatenate([dst[:-6], np.array([xs[0], v[0], xs[1], v[1], xs[2], v[2]], np.int32)])
        cap2 = np.concatenate([cap[:-6], np.array([10, 10, 10, 10, 10, 10], np.int32)])
        side, cut = G.min_cut()
        _cut_ok(n, s, t, side, cut, want, src2, dst2, cap2)


def test_dynamic_device_batches_match_host():
    import torch
    g, stream, k, nb = gen.workload("rmat12")
    batches = [stream.next_batch(k) for _ in range(4)]
    vals_host, vals_dev = [], []
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t) as G:
        G.maxflow()
        for u, v, c in batches:
            vals_host.append(G.apply_batch(u, v, c))
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t) as G:
        G.maxflow()
        for u, v, c in batches:
            t = torch.from_numpy(np.stack([u, v, c], 1).astype(np.int32)).cuda().contiguous()
            vals_dev.append(G.apply_batch_device(t))
            torch.cuda.synchronize()
    assert vals_host == vals_dev


def test_batch_errors_leave_graph_unchanged():
    g, stream, k, nb = gen.workload("er2000")
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t) as G:
        v0 = G.maxflow()
        bad = [([0, 5], [1, 5], [3, 3]),          # u == v
               ([0, g.n], [1, 2], [3, 3]),        # out of range
               ([0, 1], [1, 2], [3, -1])]         # negative capacity
        for u, v, c in bad:
            with pytest.raises(mf.MFError) as ei:
                G.apply_batch(u, v, c)
            assert ei.value.status == mf.MF_ERR_INVALID
        with pytest.raises(mf.MFError) as ei:
            G.apply_batch([0, 1], [1, 0], [2**31 - 1, 5])
        assert ei.value.status == mf.MF_ERR_OVERFLOW
        assert G.apply_batch([], [], []) == v0
        u, v, c = stream.next_batch(k)
        want = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
        want.static()
        assert G.apply_batch(u, v, c) == want.apply(u, v, c)


def test_state_errors():
    g, _, _, _ = gen.workload("er2000")
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t) as G:
        with pytest.raises(mf.MFError) as ei:
            G.apply_batch([0], [1], [5])
        assert ei.value.status == mf.MF_ERR_STATE
        with pytest.raises(mf.MFError) as ei:
            G.min_cut()
        assert ei.value.status == mf.MF_ERR_STATE


def test_relayout_when_slack_runs_out():
    """Many inserts into rows with one slot of slack force re-layouts."""
    g = gen.erdos_renyi(300, 1200, 100, seed=4)
    model = _CapModel(g.n, g.src, g.dst, g.cap)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, insert_slack_min=1,
                         insert_slack_pct=1) as G:
        assert G.maxflow() == o.static()
        for b in range(5):
            u, v, c = gen.random_batch(g.n, 400, 100, seed=77 + b)
            model.apply(u, v, c)
            say("relayout batch", b)
            val = G.apply_batch(u, v, c)
            assert val == o.apply(u, v, c)
        assert G.stats()["relayouts"] >= 1
        # slots, capacities and pair links survived the moves
        es, ed, ec = G.get_edges()
        ms, md, mc = model.arrays()
        live = mc > 0
        assert np.array_equal(es, ms[live]) and np.array_equal(ed, md[live]) and np.array_equal(ec, mc[live])
        _flow_cert(G, g.n, g.s, g.t, val, model)


def test_relayout_keeps_long_unsorted_rows():
    """RMAT scale 16 has rows longer than the in-block sort takes: their
    inserted tails stay unsorted after a re-layout and must still be found."""
    g, stream, k, _ = gen.workload("rmat16")
    model = _CapModel(g.n, g.src, g.dst, g.cap)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, insert_slack_min=1,
                         insert_slack_pct=1) as G:
        assert G.maxflow() == o.static()
        for b in range(4):
            u, v, c = stream.next_batch(4 * k)
            model.apply(u, v, c)
            say("long-row relayout batch", b)
            assert G.apply_batch(u, v, c) == o.apply(u, v, c)
        assert G.stats()["relayouts"] >= 1
        es, ed, ec = G.get_edges()
        ms, md, mc = model.arrays()
        live = mc > 0
        assert np.array_equal(es, ms[live]) and np.array_equal(ed, md[live]) and np.array_equal(ec, mc[live])


def test_offload_restore_resumes_exactly():
    """Offload the retained state to host memory and back between batches
    (also across a re-layout that grows the slot arrays): every value still
    matches the oracle and calls on an offloaded handle are refused."""
    g, stream, k, _ = gen.workload("rmat12")
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, insert_slack_min=1,
                         insert_slack_pct=1) as G:
        assert G.maxflow() == o.static()
        full = G.stats()["device_bytes"]
        for b in range(4):
            G.offload()
            assert G.stats()["device_bytes"] < full // 100
            with pytest.raises(mf.MFError) as ei:
                G.apply_batch(np.array([0]), np.array([1]), np.array([1]))
            assert ei.value.status == mf.MF_ERR_STATE
            with pytest.raises(mf.MFError) as ei:
                G.offload()
            assert ei.value.status == mf.MF_ERR_STATE
            G.restore()
            u, v, c = stream.next_batch(4 * k)
            say("offload/restore batch", b)
            assert G.apply_batch(u, v, c) == o.apply(u, v, c)
        assert G.stats()["relayouts"] >= 1
        with pytest.raises(mf.MFError) as ei:
            G.restore()
        assert ei.value.status == mf.MF_ERR_STATE


# --- flow output (certificate) --------------------------------------------------

def _flow_cert(G, n, s, t, value, model):
    fs, fd, ff = G.get_flow()
    ms, md, mc = model.arrays()
    live = mc > 0
    assert np.array_equal(fs, ms[live]) and np.array_equal(fd, md[live])
    side, cut = G.min_cut()
    rc, msg = oracle.cert_check(n, fs, fd, mc[live], s, t, ff.astype(np.int64), side, value)
    assert rc == 0, msg


@pytest.mark.parametrize("name", ["er2000", "rmat12", "grid64", "rmat16", "grid256"])
def test_get_flow_is_a_max_flow(name):
    g, stream, k, nb = gen.workload(name)
    model = _CapModel(g.n, g.src, g.dst, g.cap)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t) as G:
        v = G.maxflow()
        say("flow static", name)
        _flow_cert(G, g.n, g.s, g.t, v, model)
        for b in range(3):
            u, vv, c = stream.next_batch(k)
            model.apply(u, vv, c)
            v = G.apply_batch(u, vv, c)
            say("flow batch", name, b)
            _flow_cert(G, g.n, g.s, g.t, v, model)
            # the completion ran on a copy: the next repair still matches
        u, vv, c = stream.next_batch(k)
        model.apply(u, vv, c)
        ms, md, mc = model.arrays()
        assert G.apply_batch(u, vv, c) == oracle.max_flow(g.n, ms, md, mc, g.s, g.t)


@pytest.mark.parametrize("seed", range(8))
def test_get_flow_tiny(seed):
    rng = np.random.default_rng(9000 + seed)
    n = int(rng.integers(3, 11))
    src, dst, cap = _random_small(rng, n, 4 * n, 12)
    model = _CapModel(n, src, dst, cap)
    with mf.MaxFlowGraph(n, src, dst, cap, 0, n - 1) as G:
        v = G.maxflow()
        assert v == oracle.brute_min_cut(n, src, dst, cap, 0, n - 1)
        _flow_cert(G, n, 0, n - 1, v, model)
        for b in range(4):
            pairs = np.array(list(model.c.keys()), dtype=np.int64).reshape(-1, 2)
            u, vv, c = gen.random_batch(n, 6, 12, seed=seed * 10 + b, pairs=pairs)
            model.apply(u, vv, c)
            v = G.apply_batch(u, vv, c)
            _flow_cert(G, n, 0, n - 1, v, model)


# --- full size: the benchmark workload ------------------------------------------

def test_rmat20_full_size():
    g, stream, k, nb = gen.workload("rmat20")
    say("rmat20 oracle static")
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    want = o.static()
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t) as G:
        say("rmat20 gpu static")
        got = G.maxflow()
        assert got == want
        side, cut = G.min_cut()
        _cut_ok(g.n, g.s, g.t, side, cut, got, g.src, g.dst, g.cap)
        for b in range(10):
            u, v, c = stream.next_batch(k)
            say("rmat20 batch", b)
            got = G.apply_batch(u, v, c)
            assert got == o.apply(u, v, c)
            cs, cd, cc = stream.current_edges()
            side, cut = G.min_cut()
            _cut_ok(g.n, g.s, g.t, side, cut, got, cs, cd, cc)


@pytest.mark.parametrize("kind", ["inc", "dec", "mixed"])
@pytest.mark.parametrize("name", ["er2000", "rmat12", "grid64"])
def test_paper_shaped_batches(name, kind):
    """Section 6.2's update files (existing edges, source/sink edges favoured,
    all increases / all decreases / mixed) at 0.1%, 1% and 10% of |E|."""
    g, stream, _, _ = gen.workload(name)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t) as G:
        prev = o.static()
        assert G.maxflow() == prev
        for frac in (0.001, 0.01, 0.1):
            k = max(1, int(round(frac * stream.keys.size)))
            u, v, c = stream.paper_batch(k, kind)
            say("paper batch", name, kind, k)
            want = o.apply(u, v, c)
            assert G.apply_batch(u, v, c) == want
            # raising capacities cannot lower the maximum flow, lowering cannot raise it
            assert want >= prev if kind == "inc" else (want <= prev if kind == "dec" else True)
            prev = want


def test_grid2048_full_size():
    """The 2048 x 2048 grid at full size: the static value and the first
    batches' values equal the oracle's (stored by
    tests/golden/make_full_size_values.py: the CPU oracle takes minutes on
    this graph), and every cut is a certificate."""
    import json
    ref = json.load(open(os.path.join(HERE, "golden", "grid2048_values.json")))
    g, stream, k, _ = gen.workload("grid2048")
    assert ref["batch_size"] == k
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t) as G:
        say("grid2048 gpu static")
        got = G.maxflow()
        assert got == ref["values"][0]
        side, cut = G.min_cut()
        _cut_ok(g.n, g.s, g.t, side, cut, got, g.src, g.dst, g.cap)
        for b, want in enumerate(ref["values"][1:]):
            u, v, c = stream.next_batch(k)
            say("grid2048 batch", b)
            got = G.apply_batch(u, v, c)
            assert got == want
        cs, cd, cc = stream.current_edges()
        side, cut = G.min_cut()
        _cut_ok(g.n, g.s, g.t, side, cut, got, cs, cd, cc)


@pytest.mark.parametrize("relabel_mode", [0, 1])
@pytest.mark.parametrize("name", ["er2000", "rmat12", "grid64", "rmat16"])
def test_push_pull_matches_oracle(name, relabel_mode):
    """Section 5.2's O2: static push-pull (sink in-edges saturated first) and
    the parallel push-pull repair (old min cut saturated again, push inside
    T and pull inside S on two streams, then the ordinary loop) give the
    oracle's values, with cut certificates, on mixed, increase-only and
    decrease-only batches."""
    g, stream, k, _ = gen.workload(name)
    model = _CapModel(g.n, g.src, g.dst, g.cap)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, push_pull=True,
                         relabel_mode=relabel_mode) as G:
        got = G.maxflow()
        assert got == o.static()
        side, cut = G.min_cut()
        _cut_ok(g.n, g.s, g.t, side, cut, got, g.src, g.dst, g.cap)
        for b, kind in enumerate(["mix", "inc", "dec", "mix", "dec"]):
            if kind == "mix":
                u, v, c = stream.next_batch(k)
            else:
                u, v, c = stream.paper_batch(max(1, k // 2), kind)
            model.apply(u, v, c)
            say("push-pull batch", name, b, kind)
            got = G.apply_batch(u, v, c)
            assert got == o.apply(u, v, c)
            ms, md, mc = model.arrays()
            side, cut = G.min_cut()
            _cut_ok(g.n, g.s, g.t, side, cut, got, ms, md, mc)


def test_caller_allocator_torch():
    """Device memory from torch's caching allocator: values unchanged, the
    memory shows up in torch's accounting while the handle lives (also
    across a re-layout) and is given back when it is freed."""
    import torch
    g, stream, k, _ = gen.workload("rmat12")
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    st = torch.cuda.current_stream()
    alloc = mf.TorchAllocator(device=0, stream=st)
    G = mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, stream=st, device=0, allocator=alloc,
                        insert_slack_min=1, insert_slack_pct=1)
    try:
        held = torch.cuda.memory_allocated() - base
        assert held >= G.stats()["slot_capacity"] * 16
        assert G.maxflow() == o.static()
        for _ in range(3):
            b = stream.next_batch(4 * k)
            assert G.apply_batch(*b) == o.apply(*b)
        assert G.stats()["relayouts"] >= 1
    finally:
        G.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
    graphs = gen.batched_graphs(4, seed=79900, n_lo=500, n_hi=3e3)
    want = [oracle.max_flow(x.n, x.src, x.dst, x.cap, x.s, x.t) for x in graphs]
    with mf.MaxFlowBatch(graphs, stream=st, device=0, allocator=alloc) as B:
        assert torch.cuda.memory_allocated() > base
        assert B.maxflow().tolist() == want
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


# --- batched solve: many graphs in one launch -----------------------------------

def _batch_streams(graphs, seed=42000):
    streams = []
    for i, g in enumerate(graphs):
        st = gen.BatchStream(g, seed + i, inc_max=50, new_cap_max=100)
        streams.append(st)
    return streams


@pytest.mark.parametrize("warm", [True, False])
def test_batched_matches_oracle(warm):
    graphs = gen.batched_graphs(24, seed=77000, n_lo=1e3, n_hi=3e4)
    streams = _batch_streams(graphs)
    oracles = [oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t) for g in graphs]
    want = [o.static() for o in oracles]
    say("batched static", len(graphs))
    with mf.MaxFlowBatch(graphs, warm_start=warm) as B:
        got = B.maxflow()
        assert got.tolist() == want
        for rnd in range(2):
            batches = []
            for g, st in zip(graphs, streams):
                k = max(1, int(round(0.01 * st.keys.size)))
                batches.append(st.next_batch(k))
            want = [o.apply(*b) for o, b in zip(oracles, batches)]
            say("batched repair", rnd)
            assert B.apply(batches).tolist() == want


def test_batched_relayout_on_tight_slack():
    """One free slot per row: the first batches' inserts overflow rows, the
    pools are re-laid and the values still match the oracle."""
    graphs = gen.batched_graphs(12, seed=77500, n_lo=500, n_hi=1e4)
    streams = _batch_streams(graphs)
    oracles = [oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t) for g in graphs]
    want = [o.static() for o in oracles]
    with mf.MaxFlowBatch(graphs, insert_slack_min=1, insert_slack_pct=1) as B:
        assert B.maxflow().tolist() == want
        for rnd in range(3):
            batches = []
            for g, st in zip(graphs, streams):
                k = max(1, int(round(0.05 * st.keys.size)))
                batches.append(st.next_batch(k))
            want = [o.apply(*b) for o, b in zip(oracles, batches)]
            say("batched tight-slack repair", rnd)
            assert B.apply(batches).tolist() == want


def test_batched_equals_single_graph_calls():
    graphs = gen.batched_graphs(8, seed=78000, n_lo=500, n_hi=5e3)
    singles = []
    for g in graphs:
        with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t) as G:
            singles.append(G.maxflow())
    with mf.MaxFlowBatch(graphs) as B:
        assert B.maxflow().tolist() == singles
        it, ms = B.info()
        assert (it > 0).all() and ms > 0


def test_batched_errors_change_nothing():
    graphs = gen.batched_graphs(4, seed=79000, n_lo=200, n_hi=2e3)
    with mf.MaxFlowBatch(graphs) as B:
        v0 = B.maxflow().tolist()
        bad = [(np.array([0]), np.array([1]), np.array([5])) for _ in graphs]
        bad[2] = (np.array([0]), np.array([graphs[2].n]), np.array([5]))  # out of range
        with pytest.raises(mf.MFError) as ei:
            B.apply(bad)
        assert ei.value.status == mf.MF_ERR_INVALID
        empty = [(np.zeros(0, np.int32),) * 3 for _ in graphs]
        assert B.apply(empty).tolist() == v0
