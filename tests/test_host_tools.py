"""Host-side logic that needs no GPU: the rocprofv3 summariser, the traffic
lookup of bench.py, and the learned-start statistics."""

import csv
import json
import os

import pytest

from paper_1809_00845_amd import learned as LS
from paper_1809_00845_amd import profile_summary as PS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write_counters(d, name, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, name + "_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Counter_Name", "Counter_Value"])
        for k, v in rows:
            w.writerow([k, counter, v])


def _write_stats(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "kt_kernel_stats.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        for n, c, avg in rows:
            w.writerow([n, c, c * avg, avg, 0, avg, avg, 0])


def test_profile_summary_calibration(tmp_path, monkeypatch):
    prof = tmp_path / "prof"
    _write_stats(str(prof / "kt"), [("k_zpass", 10, 50000.0), ("k_fwd_xy", 10, 30000.0)])
    mib = 1024.0
    # copy probe: one fill (no reads) and five copies of 256 MiB, FETCH counts half
    _write_counters(str(prof / "cfetch"), "cfetch", "FETCH_SIZE",
                    [("vectorized_elementwise_kernel", 0.0)] + [("vectorized_elementwise_kernel", 128 * mib)] * 5)
    _write_counters(str(prof / "cwrite"), "cwrite", "WRITE_SIZE", [("vectorized_elementwise_kernel", 256 * mib)] * 6)
    _write_counters(str(prof / "fetch"), "fetch", "FETCH_SIZE", [("k_zpass", 1000.0), ("k_zpass", 1002.0)])
    _write_counters(str(prof / "write"), "write", "WRITE_SIZE", [("k_zpass", 500.0), ("k_zpass", 500.0)])
    monkeypatch.setattr(PS, "ROOT", str(tmp_path))
    rec = PS.summarise(str(prof), "wl", "demo")
    assert rec["fetch_factor"] == pytest.approx(2.0) and rec["write_factor"] == pytest.approx(1.0)
    z = rec["kernels"]["k_zpass"]
    assert z["read_bytes"] == pytest.approx(1001.0 * 1024 * 2.0)
    assert z["write_bytes"] == pytest.approx(500.0 * 1024)
    assert z["dispatches"] == 2
    text = open(tmp_path / "profiles" / "demo.md").read()
    assert "k_zpass | 10 | 50.0" in text
    assert json.load(open(tmp_path / "profiles" / "demo_counters.json"))["workload"] == "wl"


def test_traffic_lookup_needs_matching_workload_and_sources():
    import bench

    assert bench.measured_traffic("no-such-workload", "zpass") is None
    path = os.path.join(ROOT, "profiles", "apply_laplace3d_cube128_fp32_counters.json")
    rec = json.load(open(path))
    t = bench.measured_traffic(rec["workload"], "zpass")
    if rec["csrc_sha256"] == PS.apply_sources_sha256():
        k = rec["kernels"]["k_zpass"]
        assert t == pytest.approx(k["read_bytes"] + k["write_bytes"])
    else:
        assert t is None


def test_learned_summary():
    rows = [
        {"m": 10, "iters0": 30, "iters1": 28, "t0": 0.005, "t1": 0.006, "relres0": 9e-7, "relres1": 8e-7,
         "x0_used": 1, "x0_relres": 0.1, "status0": 0, "status1": 0},
        {"m": 12, "iters0": 32, "iters1": 32, "t0": 0.007, "t1": 0.007, "relres0": 5e-7, "relres1": 9.9e-7,
         "x0_used": 0, "x0_relres": 1.3, "status0": 0, "status1": 0},
    ]
    s = LS.summary(rows)
    assert s["problems"] == 2 and s["guess_kept"] == 1 and s["all_converged"]
    assert s["iters_plain_mean"] == 31.0 and s["iters_learned_mean"] == 30.0
    assert s["time_plain_ms_mean"] == pytest.approx(6.0) and s["relres_max"] == pytest.approx(9.9e-7)
    assert s["guess_relres_median"] == pytest.approx(0.7)
    rows[1]["status1"] = 1
    assert not LS.summary(rows)["all_converged"]


def test_oversampled_sphere_generator():
    """oversample = s: nodes follow the coarse spacing s h, sit on the sphere,
    and snap to the fine grid within half a cell per axis."""
    import numpy as np

    from paper_1809_00845_amd import inputs as I

    base = I.sphere3d(16, 0.35)
    g = I.sphere3d(64, 0.35, oversample=4)
    assert g.m == base.m and g.n == (64, 64, 64) and g.meta["oversample"] == 4
    assert abs(g.weights.sum() - base.weights.sum()) < 1e-9
    r = np.linalg.norm(g.nodes - g.center, axis=1)
    assert np.abs(r - 0.35).max() < 1e-12
    snapped = np.rint(g.nodes / g.h) * g.h
    assert np.abs(snapped - g.nodes).max() <= 0.5 * g.h + 1e-15
    # the s = 1 generator puts nodes on grid points
    assert np.abs(np.rint(base.nodes / base.h) * base.h - base.nodes).max() < 1e-15
