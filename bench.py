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
    "batch512": "512 independent graphs, alternately Erdos-Renyi and RMAT, n log-uniform in "
                "[1e3,1e5], out-degree 8, caps U[1,100]; one batched static solve, then one batch "
                "of 1% updates per graph (40/40/20) repaired in one batched launch",
    "rmat20": "RMAT scale 20 (a=.57,b=.19,c=.19), edge factor 16, caps U[1,1000], duplicates "
              "summed; batches of 10,000 updates (40% +U[1,50], 40% to U[0,cap), 20% new U[1,1000])",
    "er2000": "Erdos-Renyi n=2000 m=16000, caps U[1,100]; batches of 200 updates (40/40/20)",
    "grid2048": "2048x2048 4-connected grid, caps U[1,100], source/sink links 1000; batches of "
                "1,000 updates in random 64x64 patches (40/40/20)",
    "sweep": "update-batch sweep in the shape of the paper's experiments (Section 6.2): RMAT scale 20 "
             "(or --sweep-graph), batches of x% of |E| existing edges, source/sink edges 10x as likely, "
             "all increases / all decreases / mixed, each applied to the freshly solved graph; "
             "incremental vs from-scratch time",
    "serve64": "64 resident RMAT graphs, scale uniform in 14..20, edge factor 16, caps U[1,1000]; "
               "2,000 update batches (size log-uniform 10..10,000, 40/40/20) to uniformly chosen "
               "graphs with Poisson arrivals; HBM budget 50% of the fleet's footprint",
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 40; batch512: 3 rounds, the workload being one batch per graph)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps first (default 2; batch512: 1)")
    ap.add_argument("--workload", default="rmat20",
                    help="one of " + ", ".join(sorted(WORKLOADS)) + ", or a scaled generator workload "
                         "(rmat<scale>, grid<width>)")
    ap.add_argument("--static-runs", type=int, default=3)
    ap.add_argument("--roofline-steps", type=int, default=10,
                    help="batches applied after the timed ones with per-launch event timing of the "
                         "relabel's level kernel (the roofline); the timed batches run without events")
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
    ap.add_argument("--push-pull", action="store_true",
                    help="Section 5.2's O2: static push-pull and parallel push-pull repairs")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the handle (single-graph workloads) or the batch (batch512), untimed, "
                         "before the timed batches")
    ap.add_argument("--no-tune", action="store_true", help="batch512: skip the autotuner (the default; "
                                                          "--tune runs it)")
    ap.add_argument("--opt", action="append", default=[], metavar="KEY=INT",
                    help="graph workloads: a loop setting (bfs_alpha, bfs_beta, round_div, "
                         "bin_thread_max, bin_wave_max, long_row_cycles); repeatable")
    ap.add_argument("--sweep-graph", default="rmat20", help="sweep: generator workload of the graph")
    ap.add_argument("--sweep-pcts", default="0.01,0.1,1,5,10", help="sweep: batch sizes in %% of |E|")
    ap.add_argument("--serve-slots", type=int, default=8, help="serve64: concurrent slots")
    ap.add_argument("--serve-requests", type=int, default=2000, help="serve64: requests per run")
    ap.add_argument("--serve-load", type=float, default=0.5,
                    help="serve64: offered rate as a fraction of the measured saturation throughput")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 3 if args.workload == "batch512" else 40
    if args.warmup is None:
        args.warmup = 1 if args.workload == "batch512" else 2
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (each graph or batch "
              "stream runs on one device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    serve_inputs = None
    if args.workload == "serve64":
        # generated in worker processes before anything touches the GPU
        from paper_2511_01235_amd import gen
        t0 = time.time()
        serve_inputs = gen.serving_workload(64, args.serve_requests, workers=min(16, os.cpu_count() or 1))
        log(f"generated serving fleet and {args.serve_requests} requests in {time.time() - t0:.1f}s")

    import torch
    import paper_2511_01235_amd as mf
    from paper_2511_01235_amd import gen

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.workload == "batch512":
        return bench_batched(args, mf, gen, torch, stream)
    if args.workload == "serve64":
        return bench_serving(args, mf, serve_inputs)
    if args.workload == "sweep":
        return bench_sweep(args, mf, gen, torch, stream)

    t0 = time.time()
    g, bstream, k, nb = gen.workload(args.workload)
    total = args.warmup + args.steps
    n_roof = 0 if args.profile_all else max(1, args.roofline_steps)
    if total > nb:
        log(f"note: {total} batches requested; the workload's stream continues past its nominal {nb}")
    n_dev = 0 if args.profile_all else args.steps   # the device-resident pass after the timed one
    batches_np = [bstream.next_batch(k) for _ in range(total + n_roof + n_dev)]
    # host-memory batches as one [k, 3] int32 array each (what mf_apply_batch takes)
    host_batches = [np.ascontiguousarray(np.stack(b, 1).astype(np.int32)) for b in batches_np]
    log(f"generated {g.name}: n={g.n} m={g.m} batches={total}x{k} in {time.time() - t0:.1f}s")

    extra = {}
    for kv in args.opt:
        key, _, val = kv.partition("=")
        if key not in ("bfs_alpha", "bfs_beta", "round_div", "bin_thread_max", "bin_wave_max",
                       "long_row_cycles", "insert_slack_min", "insert_slack_pct") + mf.LOOP_FIELDS:
            raise SystemExit(f"--opt: unknown setting {key!r}")
        extra[key] = int(val)
    G = mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, stream=stream, device=0,
                        kernel_cycles=args.kc, warm_start=not args.cold_start,
                        relabel_mode=args.relabel_mode, push_pull=args.push_pull, **extra)
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
        log(f"static solve {r}: {static_ms[-1]:.1f} ms, {G.stats()['last_iterations']} iterations")
        assert static_val in (None, v)
        static_val = v
    key = np.unique(g.src.astype(np.int64) * g.n + g.dst)
    m_unique = int(key.size)
    static_med = float(np.median(static_ms))
    log(f"static value {static_val}: {static_ms} ms; iterations {G.stats()['last_iterations']}")

    # scattered-atomic reference rates for the push and relabel kernels (before
    # the copy below, which opens the profiled window)
    atomic_rates = {f"int{8 * w}_ops_per_s": round(mf.mf_debug_atomic_probe(1 << 26, w, 0), 1) for w in (4, 8)}
    # a plain copy of known size (64 Mi int32 = 256 MiB read + 256 MiB written): under
    # `rocprofv3 --pmc FETCH_SIZE` / `WRITE_SIZE` it calibrates the counters' units
    cal_src = torch.ones(64 << 20, dtype=torch.int32, device=dev)
    cal_dst = torch.empty_like(cal_src)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cal_dst.copy_(cal_src)  # first touch of the fresh pages; the timed copy is the second
    ev0.record()
    cal_dst.copy_(cal_src)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * cal_src.numel() * 4 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del cal_src, cal_dst
    log(f"copy probe {copy_gbs:.0f} GB/s; atomics {atomic_rates}")

    dev_batches = [torch.from_numpy(b).to(dev) for b in host_batches]
    torch.cuda.synchronize()
    values = []
    for i in range(args.warmup):
        values.append(G.apply_batch(host_batches[i]))
        log(f"warm-up batch {i} done")
    tuned = None
    if args.tune:
        from paper_2511_01235_amd.tune import tune_graph
        tuned = tune_graph(G, k, sync=torch.cuda.synchronize)
        log(f"tuned: {tuned}")

    # no per-launch events in the timed region (they would split the chained
    # BFS level launches); --profile-all times every class here instead
    G.profile(0xFF if args.profile_all else 0)
    per_batch, iters = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    # each step: mf_apply_batch on updates in host memory, from the call to the
    # int64 value on the host, the copy of the batch to the device included
    for i in range(args.warmup, total):
        a = time.perf_counter()
        values.append(G.apply_batch(host_batches[i]))
        per_batch.append((time.perf_counter() - a) * 1e3)
        iters.append(G.stats()["last_iterations"])
        if per_batch[-1] > 1000:
            log(f"batch {i}: {per_batch[-1]:.0f} ms, {iters[-1]} iterations")
    torch.cuda.synchronize()
    elapsed_ms = (time.perf_counter() - t_start) * 1e3
    prof = G.stats()
    G.profile(0)
    ms_per_step = elapsed_ms / args.steps
    roof_elapsed_ms = elapsed_ms

    # the same repairs with the batches already in HBM (mf_apply_batch_device),
    # on the next batches of the stream
    dev_ms = None
    if n_dev:
        base = total
        torch.cuda.synchronize()
        a = time.perf_counter()
        for i in range(base, base + n_dev):
            values_dev = G.apply_batch_device(dev_batches[i])
        torch.cuda.synchronize()
        dev_ms = (time.perf_counter() - a) * 1e3 / n_dev
        log(f"device-resident batches: {dev_ms:.3f} ms/batch")

    # from-scratch recompute of the same (final) graph on the GPU
    scratch_ms, scratch_val = [], None
    for r in range(max(1, args.scratch_runs)):
        torch.cuda.synchronize()
        a = time.perf_counter()
        v = G.maxflow()
        torch.cuda.synchronize()
        scratch_ms.append((time.perf_counter() - a) * 1e3)
        scratch_val = v
    assert scratch_val == (values_dev if n_dev else values[-1]), (scratch_val, values[-1])
    scratch_med = float(np.median(scratch_ms))
    if n_roof:
        # every kernel class timed with HIP events on the library's stream
        # (the relabel's level kernel is the roofline's) over further batches
        # of the same stream
        G.profile(0xFF)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for i in range(total + n_dev, total + n_dev + n_roof):
            G.apply_batch_device(dev_batches[i])
        torch.cuda.synchronize()
        roof_elapsed_ms = (time.perf_counter() - a) * 1e3
        prof = G.stats()
        G.profile(0)
    G.close()

    # roofline of the dominant kernel class: the relabel's BFS levels, in
    # the multi-block level kernel (RMAT, random graphs) or in the seeding,
    # one-workgroup and cooperative mid-size level kernels (grids), whichever
    # took longer
    cls = max(("global_relabel", "relabel_seed_narrow"), key=lambda c: prof["kernel_ms"][c])
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
    # HBM bytes per launch from the committed counter summary of this kernel
    # and workload, while the kernel source is unchanged since it was taken
    from paper_2511_01235_amd.prof import recorded_traffic
    traffic = None
    if cls == "global_relabel" and not args.cold_start and args.relabel_mode == 0:
        traffic = recorded_traffic(f"k_gr_level_{args.workload}", os.path.join(ROOT, "profiles"))
    kernel_names = {"global_relabel": "k_gr_level",
                    "relabel_seed_narrow": "k_gr_init, k_gr_narrow, k_gr_medium"}
    roofline = {"bound": "hbm", "kernel_class": cls, "kernel": kernel_names.get(cls, cls),
                "achieved": round(achieved, 2),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": traffic, "launches": launches,
                "avg_launch_us": round(kms * 1e3 / launches, 3) if launches else None,
                "alg_bytes_per_launch": round(kbytes / launches, 1) if launches else None,
                "share_of_step": round(kms / roof_elapsed_ms, 4) if roof_elapsed_ms > 0 else None,
                "timed_over": "every batch of the timed region" if not n_roof else
                              f"{n_roof} batches after the timed region (per-launch events)",
                "copy_probe_gbs": round(copy_gbs, 1), "atomic_probe": atomic_rates,
                "classes": {c: {"launches": prof["kernel_launches"][c],
                                "avg_launch_us": round(prof["kernel_ms"][c] * 1e3 / prof["kernel_launches"][c], 3),
                                "alg_bytes_per_launch": round(prof["kernel_bytes"][c] / prof["kernel_launches"][c], 1),
                                "achieved_gbs": round(prof["kernel_bytes"][c] / (prof["kernel_ms"][c] * 1e-3) / 1e9, 2)
                                if prof["kernel_ms"][c] > 0 else None}
                            for c in prof["kernel_launches"] if prof["kernel_launches"][c]}}

    cpu = None
    if not args.no_cpu:
        host = cpu_host()
        cpu = {**cpu_baseline(g, batches_np, static_val, values, args.cpu_budget_s), **host}

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
        "config": {"workload": f"{args.workload}: {WORKLOADS.get(args.workload, 'generator workload')}", "n": g.n,
                   "m_edges_generated": g.m, "m_pairs": m_unique, "s": g.s, "t": g.t,
                   "batch_size": k, "kernel_cycles": st["kernel_cycles"],
                   "warm_start": not args.cold_start, "relabel_mode": args.relabel_mode,
                   "push_pull": args.push_pull, **extra},
        "batches_from": "host memory (mf_apply_batch; the copy to the device is inside each step)",
        "device_resident_ms_per_batch": round(dev_ms, 4) if dev_ms else None,
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
        "relayouts": prof["relayouts"],
        "tuned": tuned,
        "updates_per_s": round(k / (ms_per_step * 1e-3), 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_batched(args, mf, gen, torch, stream):
    """512 graphs: one batched launch per step against one launch sequence per
    graph (mf_maxflow / mf_apply_batch on each), values required identical."""
    t0 = time.time()
    graphs = gen.batched_graphs(512, seed=41000)
    streams = [gen.BatchStream(g, 42000 + i, inc_max=50, new_cap_max=100) for i, g in enumerate(graphs)]
    rounds = args.warmup + args.steps
    batches = [[st.next_batch(max(1, int(round(0.01 * st.keys.size)))) for st in streams]
               for _ in range(rounds)]
    log(f"generated 512 graphs (sum n={sum(g.n for g in graphs)}, sum m={sum(g.m for g in graphs)}) "
        f"and {rounds} update rounds in {time.time() - t0:.1f}s")
    B = mf.MaxFlowBatch(graphs, stream=stream, device=0, kernel_cycles=args.kc,
                        warm_start=not args.cold_start)
    tuned = None
    if args.tune and not args.no_tune:
        from paper_2511_01235_amd.tune import tune_batch
        B.maxflow()
        tuned = tune_batch(B, graphs, sample=24, sync=torch.cuda.synchronize)
        log(f"tuned: {tuned}")
    torch.cuda.synchronize()
    a = time.perf_counter()
    static_vals = B.maxflow()
    torch.cuda.synchronize()
    static_ms = (time.perf_counter() - a) * 1e3
    log(f"batched static: {static_ms:.1f} ms")
    values = []
    step_ms = []
    rep_ms = rep_bytes = None
    for r in range(rounds):
        # the first round (untimed when there is a warm-up round) is the
        # roofline's: its batched repair launch timed with events and its
        # algorithmic bytes counted on the device
        prof_round = r == 0 and args.warmup > 0
        if prof_round:
            B.profile(True)
        torch.cuda.synchronize()
        a = time.perf_counter()
        values.append(B.apply(batches[r]))
        torch.cuda.synchronize()
        if prof_round:
            rep_ms, rep_bytes = B.kernel_stats()
            B.profile(False)
        if r >= args.warmup:
            step_ms.append((time.perf_counter() - a) * 1e3)
    B.close()
    roofline = None
    if rep_ms:
        roofline = {"bound": "hbm", "kernel_class": "batched repair launch (k_batch_repair_multi)",
                    "achieved": round(rep_bytes / (rep_ms * 1e-3) / 1e9, 2),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(rep_bytes / (rep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                    "traffic": None, "launches": 1, "avg_launch_us": round(rep_ms * 1e3, 1),
                    "alg_bytes_per_launch": round(rep_bytes, 1),
                    "timed_over": "the warm-up round's batched repair launch (HIP events around it)"}
        log(f"batched repair launch {rep_ms:.2f} ms, {rep_bytes / 1e6:.1f} MB algorithmic")
    # the same work one graph at a time
    single_static_ms, single_step_ms = 0.0, [0.0] * args.steps
    for i, g in enumerate(graphs):
        with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, stream=stream, device=0,
                             kernel_cycles=args.kc, warm_start=not args.cold_start) as G:
            torch.cuda.synchronize()
            a = time.perf_counter()
            v = G.maxflow()
            single_static_ms += (time.perf_counter() - a) * 1e3
            assert v == static_vals[i], ("static", i, v, static_vals[i])
            for r in range(rounds):
                a = time.perf_counter()
                v = G.apply_batch(*batches[r][i])
                if r >= args.warmup:
                    single_step_ms[r - args.warmup] += (time.perf_counter() - a) * 1e3
                assert v == values[r][i], ("repair", r, i, v, values[r][i])
    ms_per_step = float(np.mean(step_ms))
    per_inst = float(np.mean(single_step_ms))
    log(f"batched repair {ms_per_step:.1f} ms vs per-graph calls {per_inst:.1f} ms; static "
        f"{static_ms:.1f} vs {single_static_ms:.1f} ms")
    cpu = None
    if not args.no_cpu:
        host = cpu_host()
        cpu = {**cpu_baseline_batched(graphs, batches[0], static_vals, values[0], args.cpu_budget_s), **host}
    out = {
        "metric": METRIC, "value": round(ms_per_step, 3), "unit": "ms/batch", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "int32/int64",
        "data": "synthetic",
        "config": {"workload": f"batch512: {WORKLOADS['batch512']}", "graphs": 512,
                   "sum_n": int(sum(g.n for g in graphs)), "sum_m": int(sum(g.m for g in graphs))},
        "batched_repair_ms": round(ms_per_step, 3),
        "per_instance_repair_ms": round(per_inst, 3),
        "batched_speedup_repair": round(per_inst / ms_per_step, 3),
        "batched_static_ms": round(static_ms, 3),
        "per_instance_static_ms": round(single_static_ms, 3),
        "batched_speedup_static": round(single_static_ms / static_ms, 3),
        "graphs_per_s_static": round(512 / (static_ms * 1e-3), 1),
        "tuned": tuned,
        "per_instance_options": "defaults (the same row slack as the pool)",
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_sweep(args, mf, gen, torch, stream):
    """Incremental repair against a from-scratch solve of the same updated
    graph, for increase-only, decrease-only and mixed batches of growing size
    (x% of |E|); each batch hits the graph as first solved (reloaded and
    re-solved before each point, outside the timing)."""
    g, _, _, _ = gen.workload(args.sweep_graph)
    pcts = [float(x) for x in args.sweep_pcts.split(",")]
    rows = []
    for kind in ("inc", "dec", "mixed"):
        for pct in pcts:
            st = gen.BatchStream(g, 61000 + int(pct * 1000) + {"inc": 0, "dec": 1, "mixed": 2}[kind],
                                 inc_max=50)
            k = max(1, int(round(pct / 100 * st.keys.size)))
            u, v, c = st.paper_batch(k, kind)
            dev_upd = torch.from_numpy(np.ascontiguousarray(np.stack([u, v, c], 1))).to("cuda:0")
            with mf.MaxFlowGraph(g.n, g.src, g.dst, g.cap, g.s, g.t, stream=stream, device=0,
                                 push_pull=args.push_pull) as G:
                v0 = G.maxflow()
                torch.cuda.synchronize()
                a = time.perf_counter()
                v1 = G.apply_batch_device(dev_upd)
                torch.cuda.synchronize()
                inc_ms = (time.perf_counter() - a) * 1e3
                it = G.stats()["last_iterations"]
                a = time.perf_counter()
                v2 = G.maxflow()
                torch.cuda.synchronize()
                scratch_ms = (time.perf_counter() - a) * 1e3
            assert v1 == v2, (kind, pct, v1, v2)
            rows.append({"kind": kind, "pct_of_E": pct, "updates": k, "value_before": v0, "value_after": v1,
                         "incremental_ms": round(inc_ms, 3), "from_scratch_ms": round(scratch_ms, 3),
                         "speedup": round(scratch_ms / inc_ms, 3), "iterations": it})
            log(json.dumps(rows[-1]))
    crossover = {}
    for kind in ("inc", "dec", "mixed"):
        slower = [r["pct_of_E"] for r in rows if r["kind"] == kind and r["speedup"] < 1.0]
        crossover[kind] = min(slower) if slower else None
    mean_ms = float(np.mean([r["incremental_ms"] for r in rows]))
    out = {"metric": METRIC, "value": round(mean_ms, 3), "unit": "ms/batch (mean over the sweep)", "n_gpus": 1,
           "steps": len(rows), "warmup": 0, "ms_per_step": round(mean_ms, 3), "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32/int64", "data": "synthetic",
           "config": {"workload": f"sweep: {WORKLOADS['sweep']}", "graph": args.sweep_graph, "n": g.n,
                      "m_edges_generated": g.m, "pcts": pcts},
           "sweep": rows, "first_pct_where_from_scratch_wins": crossover,
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


def bench_serving(args, mf, inputs):
    """Serving loop over 64 graphs: saturation throughput (every request
    queued at once) one slot at a time (per-instance calls), with overlapping
    slots, and with overlapping slots under an HBM budget of half the fleet's
    footprint (evicted graphs offloaded to pinned host memory); then the
    Poisson trace at a fraction of the budget-limited throughput, with the
    budget and without.  Every run starts from freshly loaded graphs and must
    return the same value for every request."""
    from paper_2511_01235_amd.serve import Server, estimate_device_bytes
    graphs, reqs = inputs
    footprint = sum(estimate_device_bytes(g.n, g.m) for g in graphs)
    unlimited = 4 * footprint

    def run(slots, budget, arrivals, label, policy="residency"):
        trace = [(gi, float(a), u, v, c) for (gi, _, u, v, c), a in zip(reqs, arrivals)]
        with Server(graphs, budget, slots=slots, device=0, policy=policy) as srv:
            t0 = time.time()
            loaded = srv.preload(threads=16)
            log(f"{label}: preloaded {loaded} graphs in {time.time() - t0:.1f}s")
            res = srv.run(trace)
            vals = [r.value for r in srv.requests]
        log(f"{label}: " + json.dumps({k: (round(x, 3) if isinstance(x, float) else x) for k, x in res.items()}))
        return res, vals

    zero = np.zeros(len(reqs))
    budget = footprint // 2
    seq, v_seq = run(1, unlimited, zero, "saturation, 1 slot, unlimited budget")
    sat, v_sat = run(args.serve_slots, unlimited, zero, f"saturation, {args.serve_slots} slots, unlimited budget")
    assert v_sat == v_seq, "values differ between one slot and overlapping slots"
    satb, v_satb = run(args.serve_slots, budget, zero, f"saturation, {args.serve_slots} slots, budget 50%")
    assert v_satb == v_seq, "values differ under the HBM budget"
    # offered rate: a fraction of what the budget-limited server sustains in
    # arrival order (every request queued, served first come first served):
    # with requests spread over time there are few to group by residency, so
    # the residency-first saturation above would overload it
    satf, v_satf = run(args.serve_slots, budget, zero, f"saturation in arrival order, {args.serve_slots} slots, "
                       "budget 50%", policy="fifo")
    assert v_satf == v_seq, "values differ under the HBM budget (arrival order)"
    rate = args.serve_load * satf["batches_per_s"]
    gaps = np.array([r[1] for r in reqs])
    arrivals = np.cumsum(gaps) / rate
    pois, v_pois = run(args.serve_slots, budget, arrivals, f"poisson {rate:.0f}/s, budget 50%")
    assert v_pois == v_seq, "values differ under the HBM budget"
    light_rate = rate / 2
    light, v_light = run(args.serve_slots, budget, np.cumsum(gaps) / light_rate,
                         f"poisson {light_rate:.0f}/s, budget 50%")
    assert v_light == v_seq
    poisu, v_poisu = run(args.serve_slots, unlimited, arrivals, f"poisson {rate:.0f}/s, unlimited budget")
    assert v_poisu == v_seq
    cpu = None
    if not args.no_cpu:
        host = cpu_host()
        cpu = {**cpu_baseline_serving(graphs, reqs, v_seq, args.cpu_budget_s), **host}
    out = {
        "metric": METRIC, "value": round(pois["p99_ms"], 3), "unit": "ms p99 latency", "n_gpus": 1,
        "steps": len(reqs), "warmup": 0, "ms_per_step": round(1e3 / pois["batches_per_s"], 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "int32/int64",
        "data": "synthetic",
        "config": {"workload": f"serve64: {WORKLOADS['serve64']}", "graphs": len(graphs),
                   "sum_n": int(sum(g.n for g in graphs)), "sum_m": int(sum(g.m for g in graphs)),
                   "slots": args.serve_slots, "offered_rate_per_s": round(rate, 1),
                   "hbm_budget_bytes": int(budget), "fleet_footprint_bytes": int(footprint)},
        "p50_ms": round(pois["p50_ms"], 3), "p99_ms": round(pois["p99_ms"], 3),
        "batches_per_s": round(pois["batches_per_s"], 1), "evictions": pois["evictions"],
        "restores": pois["restores"], "eviction": "offload to pinned host memory",
        "saturation_batches_per_s_budget": round(satb["batches_per_s"], 1),
        "saturation_batches_per_s_budget_arrival_order": round(satf["batches_per_s"], 1),
        "half_rate": {"offered_rate_per_s": round(light_rate, 1), "p50_ms": round(light["p50_ms"], 3),
                      "p99_ms": round(light["p99_ms"], 3), "batches_per_s": round(light["batches_per_s"], 1),
                      "evictions": light["evictions"]},
        "unlimited_budget_p50_ms": round(poisu["p50_ms"], 3),
        "unlimited_budget_p99_ms": round(poisu["p99_ms"], 3),
        "saturation_batches_per_s_one_slot": round(seq["batches_per_s"], 1),
        "saturation_batches_per_s_slots": round(sat["batches_per_s"], 1),
        "overlap_speedup": round(sat["batches_per_s"] / seq["batches_per_s"], 3),
        "results_identical_across_runs": True,
        "roofline": None, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_host():
    """The oracle built -O3 -march=native for this host (loaded by every CPU
    baseline below), and what the host is: CPU model and usable cores."""
    import tempfile
    import oracle
    if "MF_ORACLE_LIB" not in os.environ:
        path = os.path.join(tempfile.mkdtemp(prefix="mforacle"), "liboracle_native.so")
        os.environ["MF_ORACLE_LIB"] = oracle.build_native(path)
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "build": "gcc -O3 -march=native"}


def cpu_baseline_serving(graphs, reqs, gpu_vals, budget_s):
    """The oracle replays the trace one request at a time (1 core), on the
    requests of the smallest graphs until the budget is spent; its values are
    checked against the GPU's."""
    import oracle
    order = sorted(range(len(graphs)), key=lambda i: graphs[i].m)
    spent, done, static_s = 0.0, 0, 0.0
    for gi in order:
        g = graphs[gi]
        mine = [j for j, r in enumerate(reqs) if r[0] == gi]
        if not mine:
            continue
        o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
        a = time.perf_counter()
        o.static()
        static_s += time.perf_counter() - a
        for j in mine:
            a = time.perf_counter()
            v = o.apply(*reqs[j][2:])
            spent += time.perf_counter() - a
            assert v == gpu_vals[j], ("serving", j, v, gpu_vals[j])
            done += 1
        o.close()
        if spent + static_s > budget_s:
            break
    log(f"cpu oracle: {done} requests in {spent:.2f}s (+{static_s:.2f}s static solves)")
    return {"value": round(done / spent, 2) if spent > 0 else None, "unit": "batches/s", "cores": 1,
            "kind": "oracle",
            "sample": f"sequential repair of the {done} requests addressed to the smallest graphs of the "
                      f"fleet, in trace order (values checked equal to the GPU's), after their static solves"}


def cpu_baseline_batched(graphs, batches, static_vals, rep_vals, budget_s):
    """The oracle on the host cores, one graph per worker thread (the ctypes
    calls release the GIL), static solve then the first update batch, until the
    budget is spent; values checked against the GPU's."""
    import concurrent.futures as cf
    import oracle
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = max(1, min(16, usable))
    done = []

    def one(i):
        g = graphs[i]
        o = oracle.DynOracle(g.n, g.src, g.dst, g.cap, g.s, g.t)
        a = time.perf_counter()
        v = o.static()
        v2 = o.apply(*batches[i])
        dt = time.perf_counter() - a
        o.close()
        if v != static_vals[i] or v2 != rep_vals[i]:
            raise SystemExit(f"oracle mismatch on graph {i}")
        return dt

    a = time.perf_counter()
    with cf.ThreadPoolExecutor(cores) as ex:
        futs = []
        for i in range(len(graphs)):
            futs.append(ex.submit(one, i))
        for f in futs:
            if time.perf_counter() - a > budget_s and done:
                f.cancel()
                continue
            done.append(f.result())
    wall = time.perf_counter() - a
    n = len(done)
    return {"value": round(wall * 1e3 * len(graphs) / n, 1), "unit": "ms/(static+1 batch, 512 graphs)",
            "cores": cores, "kind": "oracle",
            "sample": f"static solve and first repair of {n} of the 512 graphs on {cores} threads in "
                      f"{wall:.1f} s, scaled to 512 graphs (values checked equal to the GPU's)"}


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
    for i, (u, vv, c) in enumerate(batches_np[:len(gpu_values)]):
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
