"""CPU tests of the rocprofv3 summary tooling (paper_2511_01235_amd/prof.py):
the timed window, the calibration copy, kernel-busy time and the traffic
line that bench.py reads back."""
import csv
import os

import pytest

from paper_2511_01235_amd import prof


def _row(name, start, end, **extra):
    r = {"Kernel_Name": name, "Start_Timestamp": str(start), "End_Timestamp": str(end)}
    r.update({k: str(v) for k, v in extra.items()})
    return r


def _trace():
    # static solve, atomic probe, cold then timed calibration copy, timed
    # batches (with an overlap and a gap), then a from-scratch solve
    return [
        _row("k_reset", 0, 10),
        _row("k_gr_level<false, 256>", 10, 20),
        _row("k_atomic_probe<unsigned int>", 30, 60),
        _row("__amd_rocclr_copyBuffer", 100, 400),      # first touch: longest
        _row("__amd_rocclr_copyBuffer", 410, 600),      # the timed copy
        _row("k_gr_level<false, 256>", 1000, 1010),
        _row("k_pr_block<false>", 1005, 1020),          # overlaps the previous one
        _row("__amd_rocclr_copyBuffer", 1030, 1031),    # a small counter read
        _row("k_gr_level<false, 256>", 1040, 1060),
        _row("k_reset", 2000, 2010),
        _row("k_gr_level<false, 256>", 2010, 2020),
    ]


def test_calibration_copy_is_the_last_large_copy():
    rows = _trace()
    assert prof.calibration_copy(rows) == 4
    with pytest.raises(ValueError):
        prof.calibration_copy([_row("k_reset", 0, 1)])


def test_timed_window_between_calibration_and_next_reset():
    rows = _trace()
    a, b = prof.timed_window(rows)
    assert (a, b) == (5, 9)
    names = [prof._name(r) for r in rows[a:b]]
    assert "k_reset" not in names and names[0].startswith("k_gr_level")


def test_busy_split_merges_overlaps_and_counts_gaps():
    rows = _trace()
    a, b = prof.timed_window(rows)
    wall, busy = prof.busy_split(rows, a, b)
    # window 1000..1060 ns; kernels cover 1000..1020, 1030..1031, 1040..1060
    assert wall == pytest.approx(0.060)
    assert busy == pytest.approx(0.041)
    assert prof.busy_split(rows, 3, 3) == (0.0, 0.0)


def test_counter_pass_scales_by_the_calibration_copy(tmp_path):
    rows = _trace()
    counters = {4: 2 * 256 * 1024 / 2.0}  # the timed copy reads half of its bytes: factor 2
    path = tmp_path / "run_counter_collection.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp",
                                          "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, r in enumerate(rows):
            val = counters.get(i, 100.0 if "k_gr_level" in prof._name(r) else 1.0)
            w.writerow(dict(r, Counter_Name="FETCH_SIZE", Counter_Value=val))
    name, factor, kib, n = prof.counter_pass(str(path), "k_gr_level")
    assert name == "FETCH_SIZE"
    assert factor == pytest.approx((256 << 20) / 1024 / counters[4])
    assert n == 2 and kib == pytest.approx(100.0)


def test_recorded_traffic_only_for_the_current_source(tmp_path):
    good = tmp_path / "k_gr_level_demo.md"
    good.write_text(f"# x\n\n{prof.TRAFFIC_TAG}: 12345 kernels.hip sha256 {prof.source_hash()}\n")
    assert prof.recorded_traffic("k_gr_level_demo", str(tmp_path)) == 12345.0
    stale = tmp_path / "k_gr_level_old.md"
    stale.write_text(f"{prof.TRAFFIC_TAG}: 999 kernels.hip sha256 {'0' * 64}\n")
    assert prof.recorded_traffic("k_gr_level_old", str(tmp_path)) is None
    assert prof.recorded_traffic("k_gr_level_demo", os.path.join(str(tmp_path), "missing")) is None


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N with N above 1 exits with a message (one GPU here)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
