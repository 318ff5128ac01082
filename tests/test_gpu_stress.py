"""GPU stress: many small random graphs, each repaired over many batches of
random size, on loop settings drawn per case, against the CPU oracle.

Each case takes an Erdos-Renyi, RMAT or grid graph of random size (so that
BFS frontiers fall into the one-workgroup, cooperative and multi-block level
kernels, and worklists into the one-workgroup and multi-launch rounds), one
of several loop configurations, and a batch stream with random batch sizes
and a random increase/decrease/insert mix.  After the static solve and after
every batch the value must equal the oracle's; the cut returned at the end
is checked as a certificate, and the labelling invariants are checked on
the device after the last batch.  Seeds are fixed, so a failure names its
case (each configuration gets every thirteenth seed).
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
from test_gpu_invariants import SAFETY  # noqa: E402

# loop configurations: defaults, then paths each setting forces
CONFIGS = [
    {},
    {"round_narrow": -1},                                  # every round as separate launches
    {"bfs_cap": -1},                                       # relabels run to the end
    {"bfs_narrow_slots": 16, "bfs_medium_slots": 1 << 30},  # cooperative levels from the start
    {"bfs_narrow_slots": -1, "bfs_medium_slots": -1},      # multi-block levels only
    {"pipeline": -1, "queue_rounds": -1},                  # one read per launch group
    {"warm_start": False},                                 # Algorithm 5 as printed
    {"round_div": 1, "kernel_cycles": 1},                  # many rounds, one cycle each
    {"push_pull": True},                                   # parallel push-pull repairs (O2)
    {"topology_driven": True},                             # every vertex a worker
    {"relabel_mode": 1},                                   # relabel and worklist in one cooperative launch
    {"bfs_bottom_up": 2},                                  # slot-parallel bottom-up levels
    {"graph_capture": 1},                                  # pipelined iterations replayed from HIP graphs
]

N_CASES = 104


def say(*a):
    print("[stress]", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def device_ready():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"


def _case(seed):
    rng = np.random.default_rng(77000 + seed)
    kind = ("er", "rmat", "grid")[seed % 3]
    if kind == "er":
        n = int(rng.integers(300, 4000))
        g = gen.erdos_renyi(n, int(n * rng.integers(3, 10)), int(rng.integers(5, 200)), seed=78000 + seed)
    elif kind == "rmat":
        g = gen.rmat(int(rng.integers(9, 13)), int(rng.integers(4, 12)), int(rng.integers(5, 1000)),
                     seed=79000 + seed)
    else:
        g = gen.grid(int(rng.integers(12, 72)), int(rng.integers(5, 100)), seed=80000 + seed,
                     link_cap=int(rng.integers(50, 2000)))
    config = CONFIGS[seed % len(CONFIGS)]
    frac_inc = float(rng.uniform(0.0, 0.6))
    frac_dec = float(rng.uniform(0.0, 1.0 - frac_inc))
    stream = gen.BatchStream(g, 81000 + 100 * seed, inc_max=int(rng.integers(1, 100)),
                             frac_inc=frac_inc, frac_dec=frac_dec)
    sizes = [int(rng.integers(1, max(2, g.src.size // int(rng.choice([10, 40, 200]))))) for _ in range(8)]
    return kind, g, config, stream, sizes


@pytest.mark.parametrize("seed", range(N_CASES))
def test_random_graph_repairs_match_oracle(seed):
    kind, g, config, stream, sizes = _case(seed)
    say("case", seed, kind, "n", g.n, "m", g.src.size, "config", config, "batches", sizes)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, **config) as G:
        assert G.maxflow() == o.static(), ("static", seed)
        for b, k in enumerate(sizes):
            u, v, c = stream.next_batch(k)
            want = o.apply(u, v, c)
            got = G.apply_batch(u, v, c)
            assert got == want, ("batch", seed, b, k, got, want)
        inv = G.invariants()
        bad = {k: inv[k] for k in SAFETY if inv[k] != 0}
        assert not bad and inv["active"] == 0 and inv["steep_slots"] == 0, ("invariants", seed, inv)
        side, cut = G.min_cut()
        cs, cd, cc = stream.current_edges()
        assert side[g.s] == 1 and side[g.t] == 0
        assert cut == want
        rc, msg = oracle.cert_check(g.n, cs, cd, cc, g.s, g.t, None, side, want)
        assert rc == 0, (seed, msg)
