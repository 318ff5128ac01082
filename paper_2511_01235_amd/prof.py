"""Summaries of rocprofv3 output for the benchmark (kernel trace and the
FETCH_SIZE / WRITE_SIZE counter passes), as markdown.

bench.py runs, in this order: the static solves (each starts with k_reset), the
atomic probes, a plain 256 MiB device copy done twice (the second one
calibrates the counters), the warm-up and timed update batches, then the
from-scratch solves (k_reset again).  The timed
window is therefore the dispatches after the calibration copy and before
the next k_reset; run the profiled bench with --warmup 0 so that the window holds
exactly the timed batches.

    python -m paper_2511_01235_amd.prof KT_DIR FETCH_DIR WRITE_DIR --kernel k_gr_level \\
        --command "..." > profiles/<kernel>_<workload>.md

The last line of the summary records the calibrated HBM bytes per launch of
the kernel with the SHA-256 of the kernel source it was measured on; bench.py
reports it as `traffic` only while the source is unchanged.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "kernels.hip")
CAL_BYTES = 256 << 20          # the calibration copy reads and writes this many bytes
TRAFFIC_TAG = "traffic_bytes_per_launch"


def source_hash() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def short(name: str) -> str:
    name = name.replace("mf::(anonymous namespace)::", "").replace("void ", "")
    return re.sub(r"\(.*", "", name)


def _rows(path):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    return rows


def _dur_us(r):
    return (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3


def _name(r):
    return r.get("Kernel_Name") or r.get("Name")


def calibration_copy(rows):
    """Index of the calibration copy: bench.py copies the 256 MiB twice (the
    first touches fresh pages); the last copy at least half as long as the
    longest is the timed one."""
    copies = [i for i, r in enumerate(rows) if "copyBuffer" in _name(r)]
    if not copies:
        raise ValueError("no calibration copy in the trace")
    longest = max(_dur_us(rows[i]) for i in copies)
    return max(i for i in copies if _dur_us(rows[i]) >= 0.5 * longest)


def timed_window(rows):
    """Indices [a, b) of the timed window (see the module docstring)."""
    a = calibration_copy(rows)
    later = [i for i, r in enumerate(rows) if i > a and "k_reset" in _name(r)]
    return a + 1, (later[0] if later else len(rows))


def stats_table(path, top=14):
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | total ms | avg us | min us | max us | % |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        out.append(f"| `{short(r['Name'])[:60]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def window_table(rows, a, b, top=10):
    agg = {}
    for r in rows[a:b]:
        k = short(_name(r))
        agg.setdefault(k, []).append(_dur_us(r))
    out = ["| kernel | calls | total ms | avg us |", "|---|---:|---:|---:|"]
    for k, d in sorted(agg.items(), key=lambda x: -sum(x[1]))[:top]:
        out.append(f"| `{k[:60]}` | {len(d)} | {sum(d) / 1e3:.3f} | {np.mean(d):.2f} |")
    return "\n".join(out), agg


def busy_split(rows, a, b):
    """(wall us, kernel-busy us) of dispatches a..b-1: the window from the
    first start to the last end, and the union of the kernel intervals in it
    (the rest is the device waiting on the host: launches and syncs)."""
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows[a:b])
    if not iv:
        return 0.0, 0.0
    busy, cs, ce = 0, iv[0][0], iv[0][1]
    for s, e in iv[1:]:
        if s > ce:
            busy += ce - cs
            cs, ce = s, e
        else:
            ce = max(ce, e)
    busy += ce - cs
    return (max(e for _, e in iv) - iv[0][0]) / 1e3, busy / 1e3


def gap_table(rows, a, b, top=12, min_us=1.0):
    """Where the device idles in dispatches a..b-1: every gap of at least
    min_us between the end of the work so far and the next dispatch's start,
    grouped by (kernel before, kernel after)."""
    iv = sorted(((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short(_name(r))) for r in rows[a:b]))
    agg = {}
    end, prev = None, None
    for s, e, k in iv:
        if end is not None and s - end >= min_us * 1e3:
            agg.setdefault((prev, k), []).append((s - end) / 1e3)
        if end is None or e > end:
            end, prev = e, k
    out = ["| before | after | gaps | idle ms | avg us |", "|---|---|---:|---:|---:|"]
    for (p, k), d in sorted(agg.items(), key=lambda x: -sum(x[1]))[:top]:
        out.append(f"| `{p[:40]}` | `{k[:40]}` | {len(d)} | {sum(d) / 1e3:.3f} | {np.mean(d):.1f} |")
    return "\n".join(out)


def counter_pass(path, kernel):
    """(counter name, calibration factor, mean KiB per dispatch of `kernel`
    in the timed window, dispatches)."""
    rows = _rows(path)
    name = rows[0]["Counter_Name"]
    a, b = timed_window(rows)
    cal = rows[calibration_copy(rows)]
    factor = (CAL_BYTES / 1024) / float(cal["Counter_Value"])
    vals = [float(r["Counter_Value"]) for r in rows[a:b] if kernel in _name(r)]
    return name, factor, float(np.mean(vals)) if vals else 0.0, len(vals)


# the library's kernel classes (mf_stats index order) and, for each, the
# kernels one class launch dispatches; the first is counted as the launch
CLASS_KERNELS = {
    "global_relabel": ["k_gr_level"],
    "push_relabel": ["k_pr_small", "k_pr_block"],
    "remove_invalid": ["k_rie_round"],
}


def counter_values(path, kernels):
    """{kernel: (counter name, factor, [KiB per dispatch in the timed window])}."""
    rows = _rows(path)
    name = rows[0]["Counter_Name"]
    a, b = timed_window(rows)
    cal = rows[calibration_copy(rows)]
    factor = (CAL_BYTES / 1024) / float(cal["Counter_Value"])
    out = {}
    for k in kernels:
        out[k] = (name, factor, [float(r["Counter_Value"]) for r in rows[a:b] if short(_name(r)) == k or
                                 short(_name(r)).startswith(k + "<")])
    return out


def traffic_table(fetch_dir, write_dir, kernels, classes):
    """Per kernel: calibrated HBM bytes per dispatch; per class: bytes per
    class launch against the algorithmic bytes the bench counted."""
    f = counter_values(os.path.join(fetch_dir, "run_counter_collection.csv"), kernels)
    w = counter_values(os.path.join(write_dir, "run_counter_collection.csv"), kernels)
    lines = ["| kernel | dispatches | FETCH MB | WRITE MB | HBM MB per dispatch |", "|---|---:|---:|---:|---:|"]
    per = {}
    for k in kernels:
        fv, wv = f[k][2], w[k][2]
        if not fv or not wv:
            continue
        fm = np.mean(fv) * 1024 * f[k][1] / 1e6
        wm = np.mean(wv) * 1024 * w[k][1] / 1e6
        per[k] = (len(fv), fm + wm)
        lines.append(f"| `{k}` | {len(fv)} | {fm:.3f} | {wm:.3f} | {fm + wm:.3f} |")
    out = "\n".join(lines) + "\n"
    if classes:
        out += ("\n| class | HBM MB per class launch | algorithmic MB per launch | HBM / algorithmic |\n"
                "|---|---:|---:|---:|\n")
        for cls, ks in CLASS_KERNELS.items():
            if cls not in classes or ks[0] not in per:
                continue
            launches = per[ks[0]][0]
            total = sum(per[k][0] * per[k][1] for k in ks if k in per)
            alg = classes[cls]["alg_bytes_per_launch"] / 1e6
            hbm = total / launches
            out += f"| {cls} | {hbm:.3f} | {alg:.3f} | {hbm / alg:.2f} |\n"
    return out


def atomic_table(kt_rows, atomic_dir, kernels):
    """Atomic requests at L2 (TCC_ATOMIC_sum) per dispatch of each kernel in
    the timed window, over the kernel's average duration in the kernel-trace
    run: the rate its pushes and relabels drive, next to the scattered-atomic
    probe's own rate measured the same way (its dispatches run before the
    window)."""
    rows = _rows(os.path.join(atomic_dir, "run_counter_collection.csv"))
    a, b = timed_window(rows)
    ka, kb = timed_window(kt_rows)
    dur = {}
    for r in kt_rows[ka:kb]:
        dur.setdefault(short(_name(r)), []).append(_dur_us(r))
    probe_dur = {}
    for r in kt_rows:
        k = short(_name(r))
        if k.startswith("k_atomic_probe"):
            probe_dur.setdefault(k, []).append(_dur_us(r))
    out = ["| kernel | dispatches | atomic requests per dispatch | avg us | G requests/s |",
           "|---|---:|---:|---:|---:|"]
    for k, d in sorted(probe_dur.items()):
        vals = [float(r["Counter_Value"]) for r in rows if short(_name(r)) == k]
        if vals:
            rate = np.mean(vals) / (np.mean(d) * 1e-6) / 1e9
            out.append(f"| `{k}` (probe) | {len(vals)} | {np.mean(vals):.0f} | {np.mean(d):.1f} | {rate:.2f} |")
    for k in kernels:
        vals = [float(r["Counter_Value"]) for r in rows[a:b] if short(_name(r)) == k or
                short(_name(r)).startswith(k + "<")]
        ds = [x for name, d in dur.items() if name == k or name.startswith(k + "<") for x in d]
        if not vals or not ds:
            continue
        rate = np.mean(vals) / (np.mean(ds) * 1e-6) / 1e9
        out.append(f"| `{k}` | {len(vals)} | {np.mean(vals):.0f} | {np.mean(ds):.1f} | {rate:.2f} |")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("kt_dir")
    ap.add_argument("fetch_dir", nargs="?")
    ap.add_argument("write_dir", nargs="?")
    ap.add_argument("--kernel", default="k_gr_level")
    ap.add_argument("--command", default="")
    ap.add_argument("--title", default="")
    ap.add_argument("--kernels", default="",
                    help="comma-separated kernels for a per-kernel traffic table (with --bench-json: per class)")
    ap.add_argument("--bench-json", default="", help="file whose last line is the bench's JSON result")
    ap.add_argument("--atomic-dir", default="", help="counter pass of TCC_ATOMIC_sum (same bench command)")
    args = ap.parse_args()
    kt = _rows(os.path.join(args.kt_dir, "run_kernel_trace.csv"))
    print(f"# {args.title or args.kernel}\n")
    if args.command:
        print("Commands (each from the repository root):\n\n```\n" + args.command.strip() + "\n```\n")
    print("## Whole run (rocprofv3 --stats)\n")
    print(stats_table(os.path.join(args.kt_dir, "run_kernel_stats.csv")) + "\n")
    try:
        a, b = timed_window(kt)
    except ValueError:
        a = b = None
    if a is None or not args.fetch_dir:
        durs = [_dur_us(r) for r in kt if args.kernel in _name(r)]
        print(f"`{args.kernel}` over the whole run: {len(durs)} launches, average {np.mean(durs):.2f} us\n")
    if a is not None:
        wt, agg = window_table(kt, a, b)
        mine = [d for k, d in agg.items() if args.kernel in k]
        durs = [x for d in mine for x in d]
        print("## Timed window (after the calibration copy, before the first from-scratch solve)\n")
        print(wt + "\n")
        print(f"`{args.kernel}` in the window: {len(durs)} launches, average {np.mean(durs):.2f} us\n")
        wall, busy = busy_split(kt, a, b)
        if wall > 0:
            print(f"Window: {wall / 1e3:.3f} ms from the first dispatch to the last, kernels busy "
                  f"{busy / 1e3:.3f} ms ({100 * busy / wall:.1f}%); the rest is the device waiting on "
                  f"host launches and synchronisations.\n")
            print("Idle gaps in the window by the kernels around them:\n")
            print(gap_table(kt, a, b) + "\n")
    if not args.fetch_dir:
        return
    if args.kernels:
        classes = None
        if args.bench_json:
            import json
            last = [ln for ln in open(args.bench_json) if ln.startswith("{")][-1]
            classes = json.loads(last)["roofline"].get("classes")
        print("## HBM traffic of each kernel (counter passes, timed window)\n")
        print(traffic_table(args.fetch_dir, args.write_dir, args.kernels.split(","), classes))
        if args.atomic_dir:
            print("## Atomics (TCC_ATOMIC_sum pass, timed window)\n")
            print(atomic_table(kt, args.atomic_dir, args.kernels.split(",")))
    total = 0.0
    lines = []
    for d in (args.fetch_dir, args.write_dir):
        name, factor, kib, n = counter_pass(os.path.join(d, "run_counter_collection.csv"), args.kernel)
        nbytes = kib * 1024 * factor
        total += nbytes
        lines.append(f"| {name} | {n} | {kib:.1f} | {factor:.3f} | {nbytes / 1e6:.3f} |")
    print("## HBM traffic (counter passes, timed window)\n")
    print("| counter | dispatches | KiB per dispatch (raw) | calibration factor | MB per dispatch |")
    print("|---|---:|---:|---:|---:|")
    print("\n".join(lines) + "\n")
    print("The factor is 256 MiB divided by what the counter reads for the plain 256 MiB copy.\n")
    print(f"{TRAFFIC_TAG}: {total:.0f} kernels.hip sha256 {source_hash()}")


def recorded_traffic(kernel_tag: str, profiles_dir: str):
    """Bytes per launch recorded for `kernel_tag` (a summary file name prefix)
    if it was measured on the current kernel source, else None."""
    if not os.path.isdir(profiles_dir):
        return None
    want = source_hash()
    for fn in sorted(os.listdir(profiles_dir)):
        if not fn.startswith(kernel_tag) or not fn.endswith(".md"):
            continue
        for line in open(os.path.join(profiles_dir, fn)):
            if line.startswith(TRAFFIC_TAG):
                parts = line.split()
                if len(parts) >= 5 and parts[-1] == want:
                    return float(parts[1])
    return None


if __name__ == "__main__":
    main()
