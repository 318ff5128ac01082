"""Writes oracle values for the many-graph workloads at their full shapes.

    python tests/golden/make_fleet_values.py batched [rounds]
    python tests/golden/make_fleet_values.py serving

batched: the 512 graphs of the batched benchmark (Erdos-Renyi and RMAT, n
log-uniform in [1e3, 1e5], generator seed 41000) and their update streams
(seed 42000 + i, batches of 1% of the graph's live edges): each graph's
static max-flow value and its value after each of the first `rounds` update
batches, into tests/golden/batched512_values.json.

serving: a fleet of seven RMAT graphs of scales 14 to 20 (edge factor 16,
capacities U[1,1000]) and a 30-request trace drawn by the serving workload
generator: each graph's static value and the value after every request in
arrival order, into tests/golden/serving_fleet_values.json.

Only the seeded generators and the CPU oracle run here; graphs are solved in
parallel worker processes.
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2511_01235_amd import gen  # noqa: E402

SERVING = dict(graphs=7, requests=30, seed=51000, arrival_seed=50000, batch_seed=52000,
               scales=[14, 15, 16, 17, 18, 19, 20])


def batched_inputs(rounds):
    graphs = gen.batched_graphs(512, seed=41000)
    streams = [gen.BatchStream(g, 42000 + i, inc_max=50, new_cap_max=100) for i, g in enumerate(graphs)]
    batches = [[st.next_batch(max(1, int(round(0.01 * st.keys.size)))) for st in streams]
               for _ in range(rounds)]
    return graphs, batches


def _solve_graph(args):
    g, batches = args
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    vals = [o.static()] + [o.apply(*b) for b in batches]
    o.close()
    return vals


def batched(rounds):
    t0 = time.time()
    graphs, batches = batched_inputs(rounds)
    jobs = [(g, [batches[r][i] for r in range(rounds)]) for i, g in enumerate(graphs)]
    with ProcessPoolExecutor(max_workers=os.cpu_count()) as ex:
        values = list(ex.map(_solve_graph, jobs, chunksize=4))
    out = {"workload": "batched512", "rounds": rounds, "values": values,
           "source": "oracle/ (sequential push-relabel) per graph on gen.batched_graphs(512, seed=41000) "
                     "with BatchStream(g, 42000 + i) batches of round(0.01 * live edges); per graph the "
                     "static value, then the value after each round"}
    with open(os.path.join(HERE, "batched512_values.json"), "w") as f:
        json.dump(out, f)
    print(f"batched512: {len(values)} graphs, {rounds} rounds in {time.time() - t0:.1f}s", flush=True)


def serving_inputs():
    return gen.serving_workload(**SERVING, workers=min(7, os.cpu_count() or 1))


def serving():
    t0 = time.time()
    graphs, reqs = serving_inputs()
    per = [[] for _ in graphs]
    for j, (gi, _, u, v, c) in enumerate(reqs):
        per[gi].append((j, u, v, c))
    jobs = [(g, [(u, v, c) for _, u, v, c in per[i]]) for i, g in enumerate(graphs)]
    with ProcessPoolExecutor(max_workers=min(7, os.cpu_count() or 1)) as ex:
        vals = list(ex.map(_solve_graph, jobs))
    by_request = [0] * len(reqs)
    for i in range(len(graphs)):
        for (j, _, _, _), v in zip(per[i], vals[i][1:]):
            by_request[j] = v
    out = {"workload": "serving_fleet", "params": SERVING, "static": [v[0] for v in vals],
           "requests": by_request,
           "source": "oracle/ (sequential push-relabel) per graph on gen.serving_workload(**params); "
                     "static values per graph, then the value each request returns, in arrival order"}
    with open(os.path.join(HERE, "serving_fleet_values.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"serving fleet: {len(graphs)} graphs, {len(reqs)} requests in {time.time() - t0:.1f}s", flush=True)


if __name__ == "__main__":
    if sys.argv[1] == "batched":
        batched(int(sys.argv[2]) if len(sys.argv) > 2 else 2)
    elif sys.argv[1] == "serving":
        serving()
    else:
        raise SystemExit(__doc__)
