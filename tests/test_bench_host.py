"""Host-side logic of the benchmark (no GPU): the single-GPU guard, the
kernel reported for each variant, and the committed HBM-traffic record
(its counters, calibration and per-launch bytes must agree)."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "--gpus 1" in r.stderr
    assert r.stdout.strip() == ""


def test_kernel_names_follow_the_library_choice():
    wide = [(1.0, 1), (1.0, 1), (1.0, 1), (0.0, 0)]
    narrow = [(1.0, 1), (1.0, 1), (0.0, 0), (0.0, 0)]
    assert bench.kernel_name("fp64", 2, wide) == "chain_dma<double, 8>"
    assert bench.kernel_name("fp64", 0, wide) == "chain_dma<double, 2>"
    assert bench.kernel_name("fp64", 1, narrow) == "chain_mfma<double, 4>"
    assert bench.kernel_name("fp64", 3, narrow) == "chain_dma<double, 16>"
    assert bench.kernel_name("fp32", 2, wide) == "chain_mfma<float, 8>"
    assert bench.kernel_name("bf16x3", 1, wide) == "chain_b3<4>"


def test_traffic_record_is_consistent():
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    fetch = np.mean(t["dispatches"]["fetch"])
    write = np.mean(t["dispatches"]["write"])
    assert abs(fetch - t["fetch_kib_per_dispatch"]) <= 1e-9 * fetch
    assert abs(write - t["write_kib_per_dispatch"]) <= 1e-9 * write
    # calibration: a plain copy of 1 GiB reads and writes 1 GiB
    assert abs(t["fetch_scale"] - 1048576.0 / t["copy_fetch_kib_per_GiB"]) <= 1e-12
    assert abs(t["write_scale"] - 1048576.0 / t["copy_write_kib_per_GiB"]) <= 1e-12
    hbm = 1024.0 * (fetch * t["fetch_scale"] + write * t["write_scale"])
    assert abs(hbm - t["hbm_bytes_per_launch"]) <= 1e-9 * hbm
    # reported only for its own variant and only while the kernel sources
    # are the ones the counters were taken on (the record is written by
    # bench.py --traffic-record from a measurement, never re-stamped)
    assert bench.measured_traffic(t["variant"] + 1) is None
    orig = bench.kernel_source_hash
    try:
        bench.kernel_source_hash = lambda: t["kernel_source_sha256"]
        assert bench.measured_traffic(t["variant"]) == t["hbm_bytes_per_launch"]
        bench.kernel_source_hash = lambda: "0" * 64
        assert bench.measured_traffic(t["variant"]) is None
    finally:
        bench.kernel_source_hash = orig
