"""Autotuner for the tuning fields of a live handle (mf_graph_tune,
mf_batch_tune): KC (push-relabel cycles per launch, i.e. how often the global
relabel runs), the BFS direction switch, the number of push-relabel rounds per
global relabel, the worklist degree bins and, for batches, the threads per
graph.  None of these changes a result; the tuner only times.

Trials are repeatable on one handle, so nothing is reloaded:

* a single graph is timed on pairs (batch, inverse batch): the batch is drawn
  from the graph's current capacities (read back with mf_get_edges) and the
  inverse sets every touched pair back, so the graph returns to the same
  capacities after each pair (and to the same value, which the tuner checks);
* a batch of graphs is timed on a from-zero solve (mf_batch_maxflow) plus one
  (batch, inverse) round over all graphs.

The search is successive halving over a sample of the configuration grid
(the defaults always included): every survivor is timed on trials it has not
seen, the best third survive, the trial count doubles, until one remains.
"""
from __future__ import annotations

import itertools
import time

import numpy as np

from . import gen

GRAPH_SPACE = {
    "kc_scale": [0.5, 1.0, 2.0],        # KC as a multiple of round(m/n)
    "bfs_alpha": [14, 40],
    "round_div": [4, 8, 16],
    "bin_thread_max": [8, 16, 32],
    "bin_wave_max": [256, 512, 1024],
    "long_row_cycles": [1, 2, 4],
}
BATCH_SPACE = dict(GRAPH_SPACE, batch_block=[256, 512, 1024])
DEFAULTS = {"kc_scale": 1.0, "bfs_alpha": 14, "round_div": 8, "bin_thread_max": 16, "bin_wave_max": 512,
            "long_row_cycles": 1,
            "batch_block": 1024}


def _configs(space, sample, seed):
    keys = list(space)
    allc = [dict(zip(keys, vals)) for vals in itertools.product(*(space[k] for k in keys))]
    allc = [c for c in allc if c["bin_wave_max"] >= c["bin_thread_max"]]
    default = {k: DEFAULTS[k] for k in keys}
    allc = [c for c in allc if c != default]
    if sample and sample - 1 < len(allc):
        rng = np.random.default_rng(seed)
        allc = [allc[i] for i in rng.choice(len(allc), size=sample - 1, replace=False)]
    return [default] + allc


def _halving(configs, run_trial, rounds):
    """Successive halving; returns (best config, its mean ms, mean ms per
    config index, trials run)."""
    scores = {i: [] for i in range(len(configs))}
    alive = list(range(len(configs)))
    used, per, trials = 0, 1, 0
    for _ in range(rounds):
        for i in alive:
            for t in range(used, used + per):
                scores[i].append(run_trial(configs[i], t))
                trials += 1
        used += per
        alive.sort(key=lambda i: float(np.mean(scores[i])))
        if len(alive) <= 1:
            break
        alive = alive[:max(1, len(alive) // 3)]
        per *= 2
    best = alive[0]
    table = {i: float(np.mean(s)) for i, s in scores.items() if s}
    return configs[best], table[best], table, trials


class _PairMaker:
    """(batch, inverse) pairs drawn from one fixed set of capacities: each
    draw runs the usual update mix on a scratch copy of the capacity table
    and records the old capacity of every pair it touches."""

    def __init__(self, n, src, dst, cap, s, t):
        g = gen.Graph("current", n, src, dst, cap, s, t, {"family": "er", "cap_max": int(cap.max(initial=1))})
        self.st = gen.BatchStream(g, 0)
        self.keys, self.caps = self.st.keys.copy(), self.st.caps.copy()
        self.n = n

    def draw(self, k, seed):
        st = self.st
        st.keys, st.caps = self.keys.copy(), self.caps.copy()
        st.seed_base, st.count = seed, 0
        u, v, c = st.next_batch(k)
        key = u.astype(np.int64) * self.n + v
        pos = np.minimum(np.searchsorted(self.keys, key), self.keys.size - 1)
        old = np.where(self.keys[pos] == key, self.caps[pos], 0).astype(np.int32)
        return (u, v, c), (u, v, old)


def _graph_options(cfg, kc_base):
    o = {k: v for k, v in cfg.items() if k not in ("kc_scale", "batch_block")}
    o["kernel_cycles"] = max(1, int(round(cfg["kc_scale"] * kc_base)))
    return o


def tune_graph(G, k: int, sample: int = 36, rounds: int = 3, seed: int = 0, sync=None) -> dict:
    """Tune a solved MaxFlowGraph for repairs of k-update batches and leave
    the best setting applied.  Returns {"options", "ms" (mean per batch and
    inverse), "default_ms", "configs", "trials", "seconds"}.  sync: called
    before reading the clock when the handle runs on a caller's stream."""
    t0 = time.time()
    empty = np.zeros(0, np.int32)
    value0 = G.apply_batch(empty, empty, empty)
    maker = _PairMaker(G.n, *G.get_edges(), G.s, G.t)
    kc_base = G.stats()["kernel_cycles"]
    pairs = {}

    def trial(cfg, t):
        if t not in pairs:
            pairs[t] = maker.draw(k, 1000 * seed + t)
        b, inv = pairs[t]
        G.tune(**_graph_options(cfg, kc_base))
        a = time.perf_counter()
        G.apply_batch(*b)
        v = G.apply_batch(*inv)
        if sync:
            sync()
        ms = (time.perf_counter() - a) * 1e3
        if v != value0:
            raise RuntimeError("a batch and its inverse did not restore the value")
        return ms

    configs = _configs(GRAPH_SPACE, sample, seed)
    best, ms, table, trials = _halving(configs, trial, rounds)
    G.tune(**_graph_options(best, kc_base))
    return {"options": _graph_options(best, kc_base), "ms": ms, "default_ms": table[0],
            "configs": len(configs), "trials": trials, "seconds": time.time() - t0}


def _batch_options(cfg, graphs):
    o = {k: v for k, v in cfg.items() if k != "kc_scale"}
    if cfg["kc_scale"] != 1.0:
        # one KC for every graph, scaled from the median round(m/n)
        med = float(np.median([g.m / g.n for g in graphs]))
        o["kernel_cycles"] = max(1, int(round(cfg["kc_scale"] * med)))
    return o


def tune_batch(B, graphs, k_frac: float = 0.01, sample: int = 36, rounds: int = 3, seed: int = 0,
               sync=None) -> dict:
    """Tune a MaxFlowBatch holding `graphs` (as loaded, solved) for a
    from-zero solve plus one round of k_frac * m updates per graph, and leave
    the best setting applied.  Returns what tune_graph returns."""
    t0 = time.time()
    vals0 = B.maxflow()
    makers = [_PairMaker(g.n, g.src, g.dst, g.cap, g.s, g.t) for g in graphs]
    cache = {}

    def trial(cfg, t):
        if t not in cache:
            drawn = [mk.draw(max(1, int(round(k_frac * g.m))), 100000 * seed + 1000 * t + i)
                     for i, (mk, g) in enumerate(zip(makers, graphs))]
            cache[t] = ([d[0] for d in drawn], [d[1] for d in drawn])
        b_all, inv_all = cache[t]
        B.tune(**_batch_options(cfg, graphs))
        a = time.perf_counter()
        v = B.maxflow()
        B.apply(b_all)
        v2 = B.apply(inv_all)
        if sync:
            sync()
        ms = (time.perf_counter() - a) * 1e3
        if not (np.array_equal(v, vals0) and np.array_equal(v2, vals0)):
            raise RuntimeError("a tuning trial changed a value")
        return ms

    configs = _configs(BATCH_SPACE, sample, seed)
    best, ms, table, trials = _halving(configs, trial, rounds)
    B.tune(**_batch_options(best, graphs))
    return {"options": _batch_options(best, graphs), "ms": ms, "default_ms": table[0],
            "configs": len(configs), "trials": trials, "seconds": time.time() - t0}
