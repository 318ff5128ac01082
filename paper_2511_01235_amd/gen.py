"""Seeded synthetic workload generators.

This module only produces inputs: capacitated directed graphs with a source
and a sink, and batches of capacity updates.  It holds no max-flow arithmetic
and imports neither the HIP library nor the CPU oracle, so both sides can be
fed from it.

Workload shapes (sizes, capacity ranges, update mix) follow the synthetic
stand-ins for the paper's real-world inputs (Table 1; Section 6.2 describes
how the paper made its update files: randomly chosen existing edges get a
higher or lower capacity).  All randomness comes from numpy's PCG64 seeded
with a fixed integer, so every array is reproducible on any machine with the
same numpy.

Conventions
  * vertices are 0..n-1, edges are (src[i], dst[i], cap[i]) int32 arrays;
  * self-loops are never emitted; the RMAT edge list may contain duplicate
    (u, v) pairs, whose capacities the loader sums;
  * an update (u, v, c) sets the capacity of the directed pair (u, v) to c;
    c = 0 deletes the edge, an absent pair is inserted.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

INT32_MAX = 2**31 - 1


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


@dataclass
class Graph:
    """A capacitated directed s-t graph given as an edge list."""

    name: str
    n: int
    src: np.ndarray  # int32[m]
    dst: np.ndarray  # int32[m]
    cap: np.ndarray  # int32[m]
    s: int
    t: int
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.src.size)


# ----------------------------------------------------------------------------
# graph families
# ----------------------------------------------------------------------------

def _distinct_pairs(rng, n, want, sampler, forbid_keys=None):
    """Draw `want` distinct ordered pairs u != v with `sampler(rng, count)`.

    Pairs already in the sorted int64 array `forbid_keys` (key = u*n+v) are
    rejected.  Order of first appearance is kept."""
    got_keys = np.empty(0, dtype=np.int64)
    while got_keys.size < want:
        need = want - got_keys.size
        u, v = sampler(rng, max(64, int(need * 1.3) + 16))
        keep = u != v
        key = u[keep].astype(np.int64) * n + v[keep].astype(np.int64)
        if forbid_keys is not None and forbid_keys.size:
            pos = np.searchsorted(forbid_keys, key)
            pos = np.minimum(pos, forbid_keys.size - 1)
            key = key[forbid_keys[pos] != key]
        key = np.concatenate([got_keys, key])
        _, first = np.unique(key, return_index=True)
        got_keys = key[np.sort(first)]
    got_keys = got_keys[:want]
    return (got_keys // n).astype(np.int32), (got_keys % n).astype(np.int32)


def _uniform_sampler(n):
    def sample(rng, count):
        u = rng.integers(0, n, size=count, dtype=np.int64)
        v = rng.integers(0, n, size=count, dtype=np.int64)
        return u, v
    return sample


def _rmat_sampler(scale, n, a, b, c):
    """RMAT endpoints: each of `scale` bits picks one of four quadrants with
    probabilities (a, b, c, 1-a-b-c); endpoints >= n are redrawn."""
    def draw(rng, count):
        u = np.zeros(count, dtype=np.int64)
        v = np.zeros(count, dtype=np.int64)
        for bit in range(scale - 1, -1, -1):
            r = rng.random(count)
            ubit = r >= a + b
            vbit = ((r >= a) & (r < a + b)) | (r >= a + b + c)
            u |= ubit.astype(np.int64) << bit
            v |= vbit.astype(np.int64) << bit
        return u, v

    def sample(rng, count):
        u, v = draw(rng, count)
        bad = (u >= n) | (v >= n)
        while bad.any():
            uu, vv = draw(rng, int(bad.sum()))
            u[bad], v[bad] = uu, vv
            bad = (u >= n) | (v >= n)
        return u, v
    return sample


def erdos_renyi(n: int, m: int, cap_max: int, seed: int, s: int = 0, t: int | None = None,
                name: str | None = None) -> Graph:
    """G(n, m): m distinct ordered pairs u != v (antiparallel pairs allowed),
    capacities uniform in [1, cap_max]."""
    rng = rng_for(seed)
    u, v = _distinct_pairs(rng, n, m, _uniform_sampler(n))
    cap = rng.integers(1, cap_max + 1, size=m, dtype=np.int64).astype(np.int32)
    t = n - 1 if t is None else t
    return Graph(name or f"er_n{n}_m{m}", n, u, v, cap, s, t,
                 {"family": "er", "seed": seed, "cap_max": cap_max})


def _pick_source_sink(n, u, v):
    """s = vertex with the most distinct out-neighbours, t = a different vertex
    with the most distinct in-neighbours; ties go to the smallest id."""
    key = np.unique(u.astype(np.int64) * n + v.astype(np.int64))
    uu = key // n
    vv = key % n
    outdeg = np.bincount(uu, minlength=n)
    indeg = np.bincount(vv, minlength=n)
    s = int(np.argmax(outdeg))
    indeg_t = indeg.copy()
    indeg_t[s] = -1
    t = int(np.argmax(indeg_t))
    return s, t


def rmat(scale: int, edge_factor: int, cap_max: int, seed: int, a=0.57, b=0.19, c=0.19,
         n: int | None = None, name: str | None = None) -> Graph:
    """RMAT graph with edge_factor * 2**scale generated edges.  Self-loops are
    dropped; duplicate pairs stay in the list (the loader sums them).  Each
    generated edge draws its own capacity in [1, cap_max]."""
    rng = rng_for(seed)
    n = (1 << scale) if n is None else n
    count = edge_factor * (1 << scale)
    u, v = _rmat_sampler(scale, n, a, b, c)(rng, count)
    cap = rng.integers(1, cap_max + 1, size=count, dtype=np.int64)
    keep = u != v
    u, v, cap = u[keep].astype(np.int32), v[keep].astype(np.int32), cap[keep].astype(np.int32)
    s, t = _pick_source_sink(n, u, v)
    return Graph(name or f"rmat{scale}_ef{edge_factor}", n, u, v, cap, s, t,
                 {"family": "rmat", "scale": scale, "seed": seed, "cap_max": cap_max,
                  "abc": (a, b, c)})


def grid(width: int, cap_max: int, seed: int, link_cap: int = 1000, name: str | None = None) -> Graph:
    """width x width 4-connected grid, both directions present with independent
    capacities in [1, cap_max].  Vertex (r, c) has id r*width + c; the source
    is width**2 (linked to column 0), the sink width**2 + 1 (linked from the
    last column), both links with capacity link_cap."""
    rng = rng_for(seed)
    W = width
    ids = np.arange(W * W, dtype=np.int64).reshape(W, W)
    hu = ids[:, :-1].ravel()
    hv = ids[:, 1:].ravel()
    vu = ids[:-1, :].ravel()
    vv = ids[1:, :].ravel()
    u = np.concatenate([hu, hv, vu, vv])
    v = np.concatenate([hv, hu, vv, vu])
    cap = rng.integers(1, cap_max + 1, size=u.size, dtype=np.int64)
    s, t = W * W, W * W + 1
    left = ids[:, 0].ravel()
    right = ids[:, -1].ravel()
    u = np.concatenate([u, np.full(W, s, np.int64), right])
    v = np.concatenate([v, left, np.full(W, t, np.int64)])
    cap = np.concatenate([cap, np.full(2 * W, link_cap, np.int64)])
    return Graph(name or f"grid{W}", W * W + 2, u.astype(np.int32), v.astype(np.int32),
                 cap.astype(np.int32), s, t, {"family": "grid", "width": W, "seed": seed,
                                              "cap_max": cap_max})


# ----------------------------------------------------------------------------
# update batches
# ----------------------------------------------------------------------------

class BatchStream:
    """Produces seeded update batches for one graph and tracks the capacities
    they leave behind, so that every batch draws from the current edge set.

    Mix per batch of k updates: round(0.4k) increases by U[1, inc_max] and
    round(0.4k) decreases to U[0, cap-1] on distinct existing edges (cap > 0),
    the rest set new edges with capacity U[1, new_cap_max] on absent pairs
    (current capacity 0, u != v).  `patch` restricts every update to one
    random patch x patch square of a grid graph."""

    def __init__(self, g: Graph, seed_base: int, inc_max: int = 50, new_cap_max: int | None = None,
                 patch: int | None = None, frac_inc: float = 0.4, frac_dec: float = 0.4):
        self.g = g
        self.n = g.n
        self.seed_base = seed_base
        self.inc_max = inc_max
        self.new_cap_max = new_cap_max or g.meta.get("cap_max", 100)
        self.patch = patch
        self.frac_inc = frac_inc
        self.frac_dec = frac_dec
        key = g.src.astype(np.int64) * g.n + g.dst.astype(np.int64)
        self.keys, inv = np.unique(key, return_inverse=True)
        self.caps = np.bincount(inv, weights=g.cap.astype(np.float64)).astype(np.int64)
        if g.meta.get("family") == "rmat":
            a, b, c = g.meta["abc"]
            self._sampler = _rmat_sampler(g.meta["scale"], g.n, a, b, c)
        else:
            self._sampler = _uniform_sampler(g.n)
        self.count = 0

    def current_edges(self):
        """(src, dst, cap) of every pair with capacity > 0."""
        live = self.caps > 0
        k = self.keys[live]
        return ((k // self.n).astype(np.int32), (k % self.n).astype(np.int32),
                self.caps[live].astype(np.int32))

    def _lookup(self, key):
        pos = np.searchsorted(self.keys, key)
        posc = np.minimum(pos, self.keys.size - 1)
        found = self.keys[posc] == key
        return posc, found

    def _existing_in(self, cand_idx, want, rng):
        if cand_idx.size < want:
            raise ValueError("not enough existing edges for the requested batch")
        return cand_idx[rng.choice(cand_idx.size, size=want, replace=False)]

    def next_batch(self, k: int):
        rng = rng_for(self.seed_base + self.count)
        self.count += 1
        n_inc = int(round(self.frac_inc * k))
        n_dec = int(round(self.frac_dec * k))
        n_new = k - n_inc - n_dec
        if self.patch is None:
            live_idx = np.flatnonzero(self.caps > 0)
            pick = self._existing_in(live_idx, n_inc + n_dec, rng)
            new_u, new_v = self._new_pairs(rng, n_new, self._sampler)
        else:
            W = self.g.meta["width"]
            P = self.patch
            r0 = int(rng.integers(0, W - P + 1))
            c0 = int(rng.integers(0, W - P + 1))
            ids = (np.arange(r0, r0 + P)[:, None] * W + np.arange(c0, c0 + P)[None, :]).astype(np.int64)
            hu, hv = ids[:, :-1].ravel(), ids[:, 1:].ravel()
            vu, vv = ids[:-1, :].ravel(), ids[1:, :].ravel()
            pu = np.concatenate([hu, hv, vu, vv])
            pv = np.concatenate([hv, hu, vv, vu])
            posc, found = self._lookup(pu * self.n + pv)
            live = found & (self.caps[posc] > 0)
            pick = self._existing_in(posc[live], n_inc + n_dec, rng)

            def patch_sampler(r, count):
                a = r.integers(0, P * P, size=count)
                b = r.integers(0, P * P, size=count)
                ar, ac = a // P, a % P
                br, bc = b // P, b % P
                adj = (np.abs(ar - br) + np.abs(ac - bc)) == 1
                uu = ((r0 + ar) * W + c0 + ac).astype(np.int64)
                vv = ((r0 + br) * W + c0 + bc).astype(np.int64)
                vv[adj] = uu[adj]  # marks adjacent pairs as self-loops: rejected
                return uu, vv
            new_u, new_v = self._new_pairs(rng, n_new, patch_sampler)
        inc_idx, dec_idx = pick[:n_inc], pick[n_inc:]
        inc_cap = self.caps[inc_idx] + rng.integers(1, self.inc_max + 1, size=n_inc)
        dec_cap = rng.integers(0, self.caps[dec_idx]) if n_dec else np.empty(0, np.int64)
        new_cap = rng.integers(1, self.new_cap_max + 1, size=n_new)
        if (inc_cap > INT32_MAX).any():
            raise OverflowError("capacity increase leaves int32 range")
        old_keys = np.concatenate([self.keys[inc_idx], self.keys[dec_idx]])
        self.caps[inc_idx] = inc_cap
        self.caps[dec_idx] = dec_cap
        self._set_new(new_u, new_v, new_cap)   # may shift indices: keys taken above
        u = np.concatenate([old_keys // self.n, new_u])
        v = np.concatenate([old_keys % self.n, new_v])
        c = np.concatenate([inc_cap, dec_cap, new_cap])
        order = rng.permutation(k)
        return (u[order].astype(np.int32), v[order].astype(np.int32), c[order].astype(np.int32))

    def paper_batch(self, k: int, kind: str, st_bias: float = 10.0, inc_max: int | None = None):
        """A batch shaped like the paper's update files (Section 6.2): k
        distinct existing edges (capacity > 0), edges out of s and into t
        drawn st_bias times as likely as the others; kind "inc" raises each
        capacity by U[1, inc_max], "dec" lowers it to U[0, cap - 1], "mixed"
        does one or the other with equal probability.  No new edges."""
        if kind not in ("inc", "dec", "mixed"):
            raise ValueError(kind)
        rng = rng_for(self.seed_base + self.count)
        self.count += 1
        live = np.flatnonzero(self.caps > 0)
        if live.size < k:
            raise ValueError("not enough existing edges for the requested batch")
        src = self.keys[live] // self.n
        dst = self.keys[live] % self.n
        w = np.where((src == self.g.s) | (dst == self.g.t), float(st_bias), 1.0)
        pick = live[rng.choice(live.size, size=k, replace=False, p=w / w.sum())]
        cur = self.caps[pick]
        up = np.ones(k, bool) if kind == "inc" else (np.zeros(k, bool) if kind == "dec"
                                                     else rng.random(k) < 0.5)
        inc = rng.integers(1, (inc_max or self.inc_max) + 1, size=k)
        dec = rng.integers(0, cur)                      # cur >= 1
        new = np.where(up, cur + inc, dec)
        if (new > INT32_MAX).any():
            raise OverflowError("capacity increase leaves int32 range")
        self.caps[pick] = new
        u, v = self.keys[pick] // self.n, self.keys[pick] % self.n
        return u.astype(np.int32), v.astype(np.int32), new.astype(np.int32)

    def _new_pairs(self, rng, want, sampler):
        if want == 0:
            return np.empty(0, np.int32), np.empty(0, np.int32)
        forbid = self.keys[self.caps > 0]
        return _distinct_pairs(rng, self.n, want, sampler, forbid_keys=forbid)

    def _set_new(self, u, v, c):
        if u.size == 0:
            return
        key = u.astype(np.int64) * self.n + v.astype(np.int64)
        posc, found = self._lookup(key)
        self.caps[posc[found]] = c[found]
        fresh = ~found
        if fresh.any():
            fk = key[fresh]
            fc = c[fresh].astype(np.int64)
            order = np.argsort(fk)
            fk, fc = fk[order], fc[order]
            at = np.searchsorted(self.keys, fk)
            self.keys = np.insert(self.keys, at, fk)
            self.caps = np.insert(self.caps, at, fc)


def random_batch(g_n: int, k: int, cap_max: int, seed: int, pairs: np.ndarray | None = None):
    """Adversarial batch for property tests: arbitrary (u, v) with u != v (may
    repeat within the batch, may hit existing, deleted or absent pairs)."""
    rng = rng_for(seed)
    if pairs is not None and pairs.size:
        pick = rng.integers(0, pairs.shape[0], size=k)
        u, v = pairs[pick, 0].astype(np.int64), pairs[pick, 1].astype(np.int64)
        fresh = rng.random(k) < 0.3
        u[fresh] = rng.integers(0, g_n, size=int(fresh.sum()))
        v[fresh] = rng.integers(0, g_n, size=int(fresh.sum()))
    else:
        u = rng.integers(0, g_n, size=k)
        v = rng.integers(0, g_n, size=k)
    clash = u == v
    v[clash] = (v[clash] + 1) % g_n
    c = rng.integers(0, cap_max + 1, size=k)
    c[rng.random(k) < 0.15] = 0
    return u.astype(np.int32), v.astype(np.int32), c.astype(np.int32)


def rmat_n(n: int, edge_factor: int, cap_max: int, seed: int, a=0.57, b=0.19, c=0.19,
           name: str | None = None) -> Graph:
    """RMAT graph on exactly n vertices: scale = ceil(log2 n), edge_factor * n
    generated edges, endpoints >= n redrawn."""
    rng = rng_for(seed)
    scale = max(1, int(np.ceil(np.log2(n))))
    count = edge_factor * n
    u, v = _rmat_sampler(scale, n, a, b, c)(rng, count)
    cap = rng.integers(1, cap_max + 1, size=count, dtype=np.int64)
    keep = u != v
    u, v, cap = u[keep].astype(np.int32), v[keep].astype(np.int32), cap[keep].astype(np.int32)
    s, t = _pick_source_sink(n, u, v)
    return Graph(name or f"rmat_n{n}", n, u, v, cap, s, t,
                 {"family": "rmat", "scale": scale, "seed": seed, "cap_max": cap_max,
                  "abc": (a, b, c)})


def batched_graphs(count: int, seed: int = 41000, n_lo: float = 1e3, n_hi: float = 1e5,
                   degree: int = 8, cap_max: int = 100):
    """Independent graphs for a batched solve: alternately Erdos-Renyi and RMAT,
    n log-uniform in [n_lo, n_hi], average out-degree `degree`, capacities
    U[1, cap_max]; graph i uses seed + i.  Erdos-Renyi graphs take s = 0,
    t = n - 1; RMAT graphs the max out-/in-degree rule."""
    rng = rng_for(seed)
    ns = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=count)).round().astype(np.int64)
    graphs = []
    for i in range(count):
        n = int(max(4, ns[i]))
        if i % 2 == 0:
            graphs.append(erdos_renyi(n, degree * n, cap_max, seed=seed + 1 + i, name=f"er_{i}"))
        else:
            graphs.append(rmat_n(n, degree, cap_max, seed=seed + 1 + i, name=f"rmat_{i}"))
    return graphs


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def workload(name: str):
    """Return (graph, batch_stream, batch_size, n_batches) for a named
    workload.  Full-size names match the configurations the benchmark and the
    large parity tests run; `*_s<k>` variants are scaled-down versions."""
    if name == "er2000":
        g = erdos_renyi(2000, 16000, 100, seed=11)
        return g, BatchStream(g, 11000, inc_max=50, new_cap_max=100), 200, 10
    if name.startswith("rmat"):
        scale = int(name[4:])
        g = rmat(scale, 16, 1000, seed=21 if scale == 20 else 2100 + scale)
        k = 10_000 if scale == 20 else max(50, (16 << scale) // 1600)
        return g, BatchStream(g, 21000 if scale == 20 else 21000 + 100 * scale, inc_max=50,
                              new_cap_max=1000), k, 100 if scale == 20 else 10
    if name.startswith("grid"):
        W = int(name[4:])
        g = grid(W, 100, seed=31 if W == 2048 else 3100 + W)
        P = min(64, W)
        k = 1000 if W >= 64 else max(10, (P * (P - 1) * 4) // 16)
        return g, BatchStream(g, 31000 if W == 2048 else 31000 + W, inc_max=50, new_cap_max=100,
                              patch=P), k, 50 if W == 2048 else 5
    raise KeyError(name)


# ----------------------------------------------------------------------------
# serving traces
# ----------------------------------------------------------------------------

def serving_trace(streams, rate: float, count: int, seed: int, k_lo: int = 10, k_hi: int = 10_000):
    """A request trace for the serving loop: `count` update batches with
    exponential inter-arrival gaps at `rate` per second (a Poisson process),
    each addressed to a graph chosen uniformly among `streams`, of size
    log-uniform in [k_lo, k_hi] but at most half the graph's live edges, and
    drawn from that graph's BatchStream so it follows the capacities the
    graph's earlier batches left.  Returns (graph, arrival_s, u, v, c) tuples
    in arrival order."""
    rng = rng_for(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += float(rng.exponential(1.0 / rate))
        gi = int(rng.integers(0, len(streams)))
        k = int(round(float(np.exp(rng.uniform(np.log(k_lo), np.log(k_hi))))))
        live = int((streams[gi].caps > 0).sum())
        k = max(1, min(k, live // 2))
        u, v, c = streams[gi].next_batch(k)
        out.append((gi, t, u, v, c))
    return out



def _serving_graph(spec):
    """Worker for serving_workload: one graph and its batches, in order."""
    i, scale, seed, stream_seed, ks, cap_max, edge_factor = spec
    g = rmat(scale, edge_factor, cap_max, seed=seed, name=f"rmat{scale}_{i}")
    st = BatchStream(g, stream_seed, inc_max=50, new_cap_max=cap_max)
    return g, [st.next_batch(k) for k in ks]


def serving_workload(graphs: int = 64, requests: int = 2000, seed: int = 51000, arrival_seed: int = 50000,
                     batch_seed: int = 52000, scale_lo: int = 14, scale_hi: int = 20, edge_factor: int = 16,
                     cap_max: int = 1000, k_lo: int = 10, k_hi: int = 10_000, workers: int = 1,
                     scales=None):
    """Graphs and a request trace for the serving loop.

    Graph i is RMAT with scale uniform in [scale_lo, scale_hi] (drawn from
    `seed`), the given edge factor, capacities U[1, cap_max] and seed
    seed + 1 + i.  Request j goes to a graph chosen uniformly, with batch size
    round(exp(U[ln k_lo, ln k_hi])) capped at a quarter of the graph's edge
    count, and a unit-rate exponential gap before it (multiply by 1/rate for a
    Poisson process at that rate); graph, size and gap come from
    `arrival_seed`.  The batches of graph i are drawn in request order from a
    BatchStream seeded with batch_seed + 1000 * i, so they depend only on that
    graph's sizes: graphs are built in `workers` processes.

    `scales` (a list of `graphs` ints) fixes the scales instead of drawing them.

    Returns (graphs, requests) with requests a list of (graph, gap_s, u, v, c)
    in arrival order."""
    rng = rng_for(seed)
    drawn = [int(x) for x in rng.integers(scale_lo, scale_hi + 1, size=graphs)]
    scales = drawn if scales is None else [int(x) for x in scales]
    if len(scales) != graphs:
        raise ValueError("one scale per graph")
    ar = rng_for(arrival_seed)
    target = ar.integers(0, graphs, size=requests)
    size = np.round(np.exp(ar.uniform(np.log(k_lo), np.log(k_hi), size=requests))).astype(np.int64)
    gaps = ar.exponential(1.0, size=requests)
    ks = [[] for _ in range(graphs)]
    for j in range(requests):
        ks[int(target[j])].append(j)
    specs = [(i, scales[i], seed + 1 + i, batch_seed + 1000 * i,
              [int(size[j]) for j in ks[i]], cap_max, edge_factor) for i in range(graphs)]
    for sp in specs:   # at most a quarter of the generated edges
        m_gen = edge_factor << sp[1]
        sp[4][:] = [max(1, min(k, m_gen // 4)) for k in sp[4]]
    if workers > 1:
        import concurrent.futures as cf
        import multiprocessing as mp
        with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
            built = list(ex.map(_serving_graph, specs))
    else:
        built = [_serving_graph(sp) for sp in specs]
    out_graphs = [b[0] for b in built]
    nxt = [0] * graphs
    reqs = []
    for j in range(requests):
        i = int(target[j])
        u, v, c = built[i][1][nxt[i]]
        nxt[i] += 1
        reqs.append((i, float(gaps[j]), u, v, c))
    return out_graphs, reqs
