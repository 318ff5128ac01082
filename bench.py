"""Benchmark: incremental max-flow repair per update batch on one MI355X.

Workload (default): RMAT scale 20 (a,b,c,d = .57,.19,.19,.05), edge factor 16,
capacities U[1,1000], duplicates summed, s = max out-degree vertex, t = a
different max in-degree vertex; update batches of 10,000 (40% increases by
U[1,50], 40% decreases to U[0,cap), 20% new edges with U[1,1000]).

A step is one mf_apply_batch_device call on a batch already resident in HBM:
locate/insert/apply/clamp, source re-saturation and the push-relabel loop
with global relabels until a fresh relabel finds no active vertex.  W
warm-up batches run untimed, then K batches are timed between device
synchronisations.  Beside it: the static solve of the initial graph
(edges/s) and a from-scratch recompute of the final graph, both on the GPU;
the dominant kernel's roofline from the library's HIP-event timing and
device-side byte counters; and the CPU oracle timed on a bounded sample.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("ms per update batch (incremental vs from-scratch); static edges/s; p99 latency")
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "rmat20": "RMAT scale 20 (a=.57,b=.19,c=.19), edge factor 16, caps U[1,1000], duplicates "
              "summed; batches of 10,000 updates (40% +U[1,50], 40% to U[0,cap), 20% new U[1,1000])",
    "er2000": "Erdos-Renyi n=2000 m=16000, caps U[1,100]; batches of 200 updates (40/40/20)",
    "grid2048": "2048x2048 4-connected grid, caps U[1,100], source/sink links 1000; batches of "
                "1,000 updates in random 64x64 patches (40/40/20)",
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat20", choices=sorted(WORKLOADS))
    ap.add_argument("--static-runs", type=int, default=3)
    ap.add_argument("--scratch-runs", type=int, default=3)
    ap.add_argument("--cpu-budget-s", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--kc", type=int, default=0, help="push/relabel cycles per launch (0: m/n)")
    ap.add_argument("--relabel-mode", type=int, default=0,
                    help="0: one launch per BFS level; 1: one cooperative launch per relabel")
    ap.add_argument("--cold-start", action="store_true",
                    help="repairs start with a global relabel (Algorithm 5 as printed) instead of "
                         "one sweep on the previous heights")
    ap.add_argument("--profile-all", action="store_true",
                    help="event-time every kernel class (adds event overhead to the steps)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (each graph or batch "
              "stream runs on one device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2511_01235_amd as mf
    from paper_2511_01235_amd import gen

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    t0 = time.time()
    g, bstream, k, nb = gen.workload(args.workload)
    total = args.warmup + args.steps
    if total > nb:
        log(f"note: {total} batches requested; the workload's stream continues past its nominal {nb}")
    batches_np = [bstream.next_batch(k) for _ in range(total)]
    log(f"generated {g.name}: n={g.n} m={g.m} batches={total}x{k} in {time.time() - t0:.1f}s")

    G = mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, stream=stream, device=0,
                        kernel_cycles=args.kc, warm_start=not args.cold_start,
                        relabel_mode=args.relabel_mode)
    st = G.stats()
    m_unique = None
    # static solve: median of a few from-zero runs on the loaded graph
    static_ms, static_val = [], None
    for r in range(max(1, args.static_runs)):
        torch.cuda.synchronize()
        a = time.perf_counter()
        v = G.maxflow()
        torch.cuda.synchronize()
        static_ms.append((time.perf_counter() - a) * 1e3)
        assert static_val in (None, v)
        static_val = v
    key = np.unique(g.src.astype(np.int64) * g.n + g.dst)
    m_unique = int(key.size)
    static_med = float(np.median(static_ms))
    log(f"static value {static_val}: {static_ms} ms; iterations {G.stats()['last_iterations']}")

    # a plain copy of known size (64 Mi int32 = 256 MiB read + 256 MiB written): under
    # `rocprofv3 --pmc FETCH_SIZE` / `WRITE_SIZE` it calibrates the counters' units
    cal_src = torch.ones(64 << 20, dtype=torch.int32, device=dev)
    cal_dst = torch.empty_like(cal_src)
    cal_dst.copy_(cal_src)
    torch.cuda.synchronize()
    del cal_src, cal_dst

    dev_batches = [torch.from_numpy(np.ascontiguousarray(np.stack(b, 1).astype(np.int32))).to(dev)
                   for b in batches_np]
    torch.cuda.synchronize()
    values = []
    for i in range(args.warmup):
        values.append(G.apply_batch_device(dev_batches[i]))

    # dominant kernel: timed live over the whole timed region (HIP events on the library's stream)
    G.profile(0xFF if args.profile_all else (1 << 0))
    per_batch, iters = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.warmup, total):
        a = time.perf_counter()
        values.append(G.apply_batch_device(dev_batches[i]))
        per_batch.append((time.perf_counter() - a) * 1e3)
        iters.append(G.stats()["last_iterations"])
    torch.cuda.synchronize()
    elapsed_ms = (time.perf_counter() - t_start) * 1e3
    prof = G.stats()
    G.profile(0)
    ms_per_step = elapsed_ms / args.steps

    # from-scratch recompute of the same (final) graph on the GPU
    scratch_ms, scratch_val = [], None
    for r in range(max(1, args.scratch_runs)):
        torch.cuda.synchronize()
        a = time.perf_counter()
        v = G.maxflow()
        torch.cuda.synchronize()
        scratch_ms.append((time.perf_counter() - a) * 1e3)
        scratch_val = v
    assert scratch_val == values[-1], (scratch_val, values[-1])
    scratch_med = float(np.median(scratch_ms))
    G.close()

    # roofline of the dominant kernel class
    cls = "global_relabel"
    if args.profile_all:
        cls = max(prof["kernel_ms"], key=lambda c: prof["kernel_ms"][c])
        log("kernel ms by class: " + json.dumps({c: round(x, 3) for c, x in prof["kernel_ms"].items() if x}))
        log("launches by class: " + json.dumps({c: x for c, x in prof["kernel_launches"].items() if x}))
    launches = prof["kernel_launches"][cls]
    kms = prof["kernel_ms"][cls]
    kbytes = prof["kernel_bytes"][cls]
    if cls == "global_relabel" and prof["kernel_launches"]["worklist"] == 0:
        kbytes += prof["kernel_bytes"]["worklist"]  # worklist build fused into the relabel launch
    achieved = (kbytes / (kms * 1e-3)) / 1e9 if kms > 0 else 0.0
    roofline = {"bound": "hbm", "kernel_class": cls, "achieved": round(achieved, 2),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": None, "launches": launches,
                "avg_launch_us": round(kms * 1e3 / launches, 3) if launches else None,
                "alg_bytes_per_launch": round(kbytes / launches, 1) if launches else None,
                "share_of_step": round(kms / elapsed_ms, 4) if elapsed_ms > 0 else None}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(g, batches_np, static_val, values, args.cpu_budget_s)

    arr = np.array(per_batch)
    out = {
        "metric": METRIC,
        "value": round(ms_per_step, 4),
        "unit": "ms/batch",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32/int64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "n": g.n,
                   "m_edges_generated": g.m, "m_pairs": m_unique, "s": g.s, "t": g.t,
                   "batch_size": k, "kernel_cycles": st["kernel_cycles"],
                   "warm_start": not args.cold_start, "relabel_mode": args.relabel_mode},
        "incremental_ms_p50": round(float(np.percentile(arr, 50)), 4),
        "incremental_ms_p90": round(float(np.percentile(arr, 90)), 4),
        "incremental_ms_p99": round(float(np.percentile(arr, 99)), 4),
        "from_scratch_ms": round(scratch_med, 4),
        "incremental_speedup_vs_from_scratch": round(scratch_med / ms_per_step, 3),
        "static_ms": round(static_med, 4),
        "static_edges_per_s": round(m_unique / (static_med * 1e-3), 1),
        "static_value": static_val,
        "final_value": values[-1],
        "mean_iterations_per_batch": round(float(np.mean(iters)), 2),
        "updates_per_s": round(k / (ms_per_step * 1e-3), 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(g, batches_np, static_val, gpu_values, budget_s):
    """The oracle as it stands (sequential push-relabel, one core), on the same
    graph and the first batches of the same stream, until the time budget is
    spent.  Its values are checked against the GPU's on the way."""
    import oracle
    o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
    a = time.perf_counter()
    v = o.static()
    static_s = time.perf_counter() - a
    if v != static_val:
        raise SystemExit(f"oracle static value {v} != GPU {static_val}")
    spent = static_s
    times = []
    for i, (u, vv, c) in enumerate(batches_np):
        if spent > budget_s and times:
            break
        a = time.perf_counter()
        val = o.apply(u, vv, c)
        dt = time.perf_counter() - a
        spent += dt
        times.append(dt)
        if val != gpu_values[i]:
            raise SystemExit(f"oracle value {val} != GPU {gpu_values[i]} at batch {i}")
    o.close()
    log(f"cpu oracle: static {static_s:.2f}s, {len(times)} batches {np.mean(times) * 1e3:.1f} ms each")
    return {"value": round(float(np.mean(times)) * 1e3, 2), "unit": "ms/batch", "cores": 1,
            "kind": "oracle",
            "sample": f"sequential push-relabel repair on the first {len(times)} batches of the same "
                      f"stream (values checked equal to the GPU's), after its own static solve of "
                      f"{static_s:.2f} s",
            "static_s": round(static_s, 3)}


if __name__ == "__main__":
    main()
