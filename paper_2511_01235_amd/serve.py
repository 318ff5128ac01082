"""Serving loop: update batches for many graphs held in device memory.

Requests (one batch of capacity updates for one graph) arrive over time.  A
fixed number of slots (host threads) serve them.  A free slot takes the
earliest-arrived request of an idle resident graph, or -- when none waits,
or when a request to a graph that is not resident has waited max_wait
seconds -- one whose graph can be made resident, and runs the repair
(mf_apply_batch) on that graph's own HIP stream: repairs of different graphs
overlap on the device, and each graph sees its requests in arrival order, so
every answer equals that of applying the graph's batches one after another.

A graph is resident while its handle holds device memory.  Admission keeps the
device bytes of the resident graphs within an HBM budget by evicting the
least recently used idle graph.  By default eviction offloads the graph's
retained state to pinned host memory (mf_graph_offload) and re-admission
copies it back (mf_graph_restore), so the repair resumes exactly where it
stopped.  With evict="rebuild" the graph's current capacities are read back
(mf_get_edges), the handle is freed, and re-admission loads those
capacities and solves from zero flow (the same maximum flow value), which
needs no host copy of the state but costs a full solve.

Every step of the computation runs in the HIP library behind the C ABI; this
module only schedules calls into it (ctypes drops the GIL for the length of
each call, so slots run concurrently; the library keeps no state shared
between handles).
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field
from collections import deque

import numpy as np


@dataclass
class Request:
    graph: int
    arrival: float                 # seconds after the start of Server.run
    u: np.ndarray
    v: np.ndarray
    c: np.ndarray
    start: float = -1.0            # when a slot took it (after any admission)
    done: float = -1.0
    value: int | None = None
    slot: int = -1
    loaded: bool = False           # the graph was (re-)admitted for this request
    seq: int = 0                   # position in the trace (breaks ties between equal arrivals)


@dataclass
class _Graph:
    n: int
    s: int
    t: int
    edges: tuple                   # (src, dst, cap) while not resident
    handle: object = None
    resident: bool = False         # handle holds device memory
    device_bytes: int = 0
    busy: bool = False
    last_use: float = 0.0
    loads: int = 0
    pending: deque = field(default_factory=deque)


def estimate_device_bytes(n: int, m: int) -> int:
    """Device bytes a loaded graph is expected to hold before its first load
    reports the real figure: about 24 B per Bi-CSR slot (two per edge plus
    insertion slack) and ~100 B per vertex, plus fixed buffers."""
    slots = int(2.5 * m) + 2 * n
    return 24 * slots + 100 * n + (2 << 20)


class Server:
    """graphs: objects with n, src, dst, cap, s, t.  `factory(n, src, dst, cap,
    s, t)` makes a handle with maxflow(), apply_batch(u, v, c), get_edges(),
    stats()["device_bytes"] and close(); the default builds a MaxFlowGraph with
    `options`."""

    def __init__(self, graphs, hbm_budget: int, slots: int = 4, factory=None, evict: str = "offload",
                 max_wait: float = 0.25, policy: str = "residency", **options):
        if factory is None:
            from . import MaxFlowGraph

            def factory(n, src, dst, cap, s, t):
                return MaxFlowGraph(n, src, dst, cap, s, t, **options)
        if evict not in ("offload", "rebuild"):
            raise ValueError("evict must be 'offload' or 'rebuild'")
        if policy not in ("residency", "fifo"):
            raise ValueError("policy must be 'residency' or 'fifo'")
        self.policy = policy
        self.factory = factory
        self.evict = evict
        self.max_wait = float(max_wait)
        self.restores = 0
        self.budget = int(hbm_budget)
        self.slots = int(slots)
        self.g = [_Graph(int(x.n), int(x.s), int(x.t), (x.src, x.dst, x.cap)) for x in graphs]
        for i in range(len(self.g)):
            if self._need(i) > self.budget:
                raise MemoryError(f"graph {i} needs about {self._need(i)} B, above the HBM budget")
        self.cv = threading.Condition()
        self.resident_bytes = 0
        self.reserved = 0
        self.releasing = 0
        self.now = 0.0
        self.peak_bytes = 0
        self.evictions = 0
        self.errors: list[BaseException] = []

    # -- accounting (lock held) -------------------------------------------------
    def _need(self, gi: int) -> int:
        x = self.g[gi]
        if x.device_bytes:
            return x.device_bytes
        return estimate_device_bytes(x.n, int(np.asarray(x.edges[0]).size))

    def _idle_resident(self, exclude: int):
        return [i for i, x in enumerate(self.g) if x.resident and not x.busy and i != exclude]

    def _committed(self) -> int:
        """Bytes that resident graphs hold or loads have reserved, less what
        graphs claimed for eviction are about to give back."""
        return self.resident_bytes + self.reserved - self.releasing

    def _victim_key(self, i: int):
        """Eviction order: graphs with the fewest requests already waiting,
        then the least recently used (under load the least recently used
        graph is the one whose queue has grown longest)."""
        x = self.g[i]
        waiting = sum(1 for r in x.pending if r.arrival <= self.now)
        return waiting, x.last_use

    def _claim(self, gi: int, need: int):
        """Claim idle resident graphs for eviction (fewest waiting requests
        first, then least recently used) until `need` more bytes fit; they
        stay busy until _release."""
        victims = []
        while self._committed() + need > self.budget:
            idle = self._idle_resident(gi)
            if not idle:
                break
            v = min(idle, key=self._victim_key)
            self.g[v].busy = True
            self.releasing += self.g[v].device_bytes
            victims.append(v)
        return victims

    def _release(self, victims):
        """Evict claimed graphs (outside the lock): read back their current
        capacities, free their device memory, then account for it."""
        for v in victims:
            x = self.g[v]
            if self.evict == "offload":
                x.handle.offload()
                edges, handle = x.edges, x.handle
            else:
                edges, handle = x.handle.get_edges(), None
                x.handle.close()
            with self.cv:
                x.edges, x.handle, x.resident = edges, handle, False
                self.resident_bytes -= x.device_bytes
                self.releasing -= x.device_bytes
                self.evictions += 1
                x.busy = False
                self.cv.notify_all()

    def _evict(self, gi: int):
        with self.cv:
            self.g[gi].busy = True
            self.releasing += self.g[gi].device_bytes
        self._release([gi])

    def _admissible(self, gi: int) -> bool:
        if self.g[gi].resident:
            return True
        free = self.budget - self._committed()
        evictable = sum(self.g[i].device_bytes for i in self._idle_resident(gi))
        return self._need(gi) <= free + evictable

    def _pick(self, now: float):
        """Residency first, with aging: the earliest-arrived request of a
        resident idle graph, unless none waits or the earliest request of a
        graph that must be admitted has waited max_wait seconds; requests to
        a graph coming in meanwhile share its one admission."""
        best_res = best_new = None
        for gi, x in enumerate(self.g):
            if x.busy or not x.pending or x.pending[0].arrival > now:
                continue
            r = x.pending[0]
            if self.policy == "fifo":  # the earliest request of any idle graph that can run
                if (x.resident or self._admissible(gi)) and \
                        (best_res is None or (r.arrival, r.seq) < (best_res.arrival, best_res.seq)):
                    best_res = r
                continue
            if x.resident:
                if best_res is None or r.arrival < best_res.arrival:
                    best_res = r
            elif (best_new is None or r.arrival < best_new.arrival) and self._admissible(gi):
                best_new = r
        if best_new is not None and (best_res is None or now - best_new.arrival >= self.max_wait):
            return best_new
        return best_res

    def _next_arrival(self, now: float) -> float:
        later = [x.pending[0].arrival for x in self.g if x.pending and x.pending[0].arrival > now]
        return min(later) - now if later else 0.005

    # -- slots ----------------------------------------------------------------------
    def _worker(self, slot: int, t0: float):
        while True:
            with self.cv:
                while True:
                    if self.remaining == 0 or self.errors:
                        return
                    now = time.perf_counter() - t0
                    self.now = now
                    r = self._pick(now)
                    if r is not None:
                        break
                    self.cv.wait(timeout=min(max(self._next_arrival(now), 1e-4), 0.005))
                x = self.g[r.graph]
                x.busy = True
                x.pending.popleft()
                reserved, victims = 0, []
                if not x.resident:
                    reserved = self._need(r.graph)
                    victims = self._claim(r.graph, reserved)
                    self.reserved += reserved
            try:
                # device memory is given back before this graph takes its share
                self._release(victims)
                restored = False
                if reserved and x.handle is not None:
                    x.handle.restore()
                    h, dev_bytes, restored = x.handle, x.device_bytes, True
                elif reserved:
                    h = self.factory(x.n, *x.edges, x.s, x.t)
                    h.maxflow()
                    dev_bytes = int(h.stats()["device_bytes"])
                r.start = time.perf_counter() - t0
                r.value = (h if reserved else x.handle).apply_batch(r.u, r.v, r.c)
                r.done = time.perf_counter() - t0
                r.slot, r.loaded = slot, bool(reserved)
            except BaseException as exc:  # re-raised by run()
                with self.cv:
                    self.errors.append(exc)
                    self.cv.notify_all()
                return
            with self.cv:
                if reserved:
                    x.handle, x.resident = h, True
                    x.device_bytes = dev_bytes
                    if restored:
                        self.restores += 1
                    else:
                        x.edges = None
                        x.loads += 1
                    self.reserved -= reserved
                    self.resident_bytes += dev_bytes
                self.peak_bytes = max(self.peak_bytes, self.resident_bytes)
                x.busy = False
                x.last_use = r.done
                self.remaining -= 1
                # the estimate may have been low: give back what is over budget
                over = self._claim(r.graph, 0) if reserved else []
                self.cv.notify_all()
            self._release(over)

    def run(self, requests) -> dict:
        """Serve `requests` (Request objects, or (graph, arrival, u, v, c)
        tuples; arrivals in seconds after the call) and return throughput and
        latency figures.  Each Request gets value, start, done, slot."""
        reqs = [r if isinstance(r, Request) else Request(*r) for r in requests]
        for i, r in enumerate(reqs):
            r.seq = i
        for r in sorted(reqs, key=lambda q: (q.arrival, q.seq)):
            self.g[r.graph].pending.append(r)
        self.remaining = len(reqs)
        t0 = time.perf_counter()
        workers = [threading.Thread(target=self._worker, args=(i, t0), daemon=True)
                   for i in range(self.slots)]
        for w in workers:
            w.start()
        for w in workers:
            w.join()
        if self.errors:
            raise self.errors[0]
        self.requests = reqs
        if not reqs:
            return {"requests": 0}
        lat = np.array([r.done - r.arrival for r in reqs]) * 1e3
        svc = np.array([r.done - r.start for r in reqs]) * 1e3
        span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
        return {"requests": len(reqs), "batches_per_s": len(reqs) / span if span > 0 else float("inf"),
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "service_mean_ms": float(svc.mean()),
                "span_s": span, "evictions": self.evictions,
                "loads": sum(x.loads for x in self.g), "restores": self.restores,
                "peak_resident_bytes": self.peak_bytes}

    def preload(self, threads: int = 8):
        """Load every graph before run (not timed) and solve it, in groups
        that fit the free budget, `threads` loads at a time.  With offload
        eviction every graph ends up loaded (the earlier ones offloaded to host
        memory as later ones need the room); with rebuild eviction loading
        stops when the budget is full.  Returns the number of graphs loaded."""
        import concurrent.futures as cf

        def load(gi):
            x = self.g[gi]
            h = self.factory(x.n, *x.edges, x.s, x.t)
            h.maxflow()
            return gi, h, int(h.stats()["device_bytes"])

        pending = [gi for gi, x in enumerate(self.g) if x.handle is None]
        loaded, order = 0, []
        with cf.ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
            while pending:
                free = self.budget - self.resident_bytes
                group, room = [], free
                for gi in pending:
                    if self._need(gi) <= room:
                        group.append(gi)
                        room -= self._need(gi)
                if not group:
                    if self.evict != "offload" or not order:
                        break
                    self._evict(order.pop(0))
                    continue
                for gi, h, nbytes in ex.map(load, group):
                    x = self.g[gi]
                    x.handle, x.resident, x.edges, x.device_bytes = h, True, None, nbytes
                    self.resident_bytes += nbytes
                    order.append(gi)
                    loaded += 1
                pending = [gi for gi in pending if gi not in set(group)]
                while self.resident_bytes > self.budget and order:
                    self._evict(order.pop(0))
        self.peak_bytes = max(self.peak_bytes, self.resident_bytes)
        self.evictions = 0
        return loaded

    def close(self):
        for x in self.g:
            if x.handle is not None:
                x.handle.close()
                x.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
