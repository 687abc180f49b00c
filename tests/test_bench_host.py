"""Host logic of bench.py (CPU): the counter summary that turns rocprofv3's
per-dispatch counters into calibrated HBM bytes, dispatch times, VALU issue
shares and LDS conflict ratios, and the refusal of more than one GPU.

The counter files are synthetic, in the column layout rocprofv3 writes
(`*_counter_collection.csv`), with values chosen so that every figure has a
hand-computed answer.
"""
import csv
import subprocess
import sys

import pytest

import bench

KIB = 1024.0


def _write(path, rows):
    path.parent.mkdir(parents=True, exist_ok=True)
    cols = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp",
            "End_Timestamp"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(cols, r)))


def _passes(tmp_path, fetch_factor=0.5, write_factor=1.0):
    """Two dispatches of a lambda kernel per pass, plus the 256 MiB copy the
    calibration reads.  Lambda: 20 MB fetched and 4 MB written per dispatch
    (true bytes), dispatches of 10 and 30 us."""
    copy_kib = bench.COPY_BYTES / KIB
    lam = "void pbf::(anonymous namespace)::k_lambda<false>(int, ...)"
    copy = "__amd_rocclr_copyBuffer"
    t = [(1000, 11000), (20000, 50000)]  # ns
    fetch = [(i, lam, "FETCH_SIZE", 20e6 / KIB * fetch_factor, *t[i]) for i in range(2)]
    fetch.append((2, copy, "FETCH_SIZE", copy_kib * fetch_factor, 60000, 160000))
    write = [(i, lam, "WRITE_SIZE", 4e6 / KIB * write_factor, *t[i]) for i in range(2)]
    write.append((2, copy, "WRITE_SIZE", copy_kib * write_factor, 60000, 160000))
    # VALU: 614e9 instructions/s would be full issue; 6.14e6 in 10 us is 100 %,
    # in 30 us a third; over both dispatches 8.188e6 / 40 us = 1/3
    sq1 = []
    for i, (a, b) in enumerate(t):
        sq1 += [(i, lam, "SQ_INSTS_VALU", 6.14e6 if i == 0 else 2.048e6, a, b),
                (i, lam, "SQ_WAVE_CYCLES", 1000.0, a, b)]
    sq2 = []
    for i, (a, b) in enumerate(t):
        sq2 += [(i, lam, "SQ_WAIT_INST_ANY", 250.0, a, b),
                (i, lam, "SQ_LDS_BANK_CONFLICT", 30.0, a, b),
                (i, lam, "SQ_ACTIVE_INST_LDS", 10.0, a, b)]
    for sub, rows in (("fetch", fetch), ("write", write), ("sq1", sq1), ("sq2", sq2)):
        _write(tmp_path / sub / "x" / f"{sub}_counter_collection.csv", rows)
    return tmp_path


def test_counter_summary_calibrates_and_averages(tmp_path):
    rec = bench.summarize_counters(_passes(tmp_path))
    assert rec["fetch_factor"] == pytest.approx(0.5)
    assert rec["write_factor"] == pytest.approx(1.0)
    # calibrated bytes per dispatch: 20 MB read + 4 MB written
    assert rec["bytes_per_dispatch"]["lambda"] == pytest.approx(24e6, rel=1e-6)
    # dispatch time: the mean over both passes' dispatches (10 and 30 us)
    assert rec["dispatch_s"]["lambda"] == pytest.approx(20e-6)
    # VALU issue over the first pass's time: 8.188e6 / 40 us / 614e9
    assert rec["valu_issue"]["lambda"] == pytest.approx(8.188e6 / 40e-6 / bench.VALU_PEAK_WAVE_INSTR, abs=1e-4)
    assert rec["lds_conflict_ratio"]["lambda"] == pytest.approx(3.0)
    assert rec["wait_share"]["lambda"] == pytest.approx(0.25)
    assert rec["sources_sha1"] == bench.kernel_sources_digest()


def test_counter_summary_other_calibration(tmp_path):
    # a counter that reads the copy at face value needs no correction
    rec = bench.summarize_counters(_passes(tmp_path, fetch_factor=1.0, write_factor=1.0))
    assert rec["fetch_factor"] == pytest.approx(1.0)
    assert rec["bytes_per_dispatch"]["lambda"] == pytest.approx(24e6, rel=1e-6)


def test_counter_summary_without_passes_is_empty(tmp_path):
    rec = bench.summarize_counters(tmp_path)
    assert rec["fetch_factor"] is None and rec["bytes_per_dispatch"] == {}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(bench.ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
