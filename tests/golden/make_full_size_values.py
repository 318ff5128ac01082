"""Writes oracle values for full-size workloads whose CPU static solve is too
slow to run inside a GPU test.

    python tests/golden/make_full_size_values.py grid2048 5

calls only the seeded generators and the CPU oracle: the static max-flow
value of the workload's graph, then the value after each of its first
`batches` update batches, into tests/golden/<workload>_values.json.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2511_01235_amd import gen  # noqa: E402


def main(name: str, batches: int):
    g, stream, k, _ = gen.workload(name)
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    t0 = time.time()
    values = [o.static()]
    print(f"{name}: static {values[0]} in {time.time() - t0:.1f}s", flush=True)
    for b in range(batches):
        values.append(o.apply(*stream.next_batch(k)))
        print(f"{name}: batch {b} -> {values[-1]}", flush=True)
    out = {"workload": name, "batch_size": k, "values": values,
           "source": "oracle/ (sequential push-relabel) on the seeded generator workload; static value "
                     "first, then the value after each update batch in stream order"}
    with open(os.path.join(HERE, f"{name}_values.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 5)
