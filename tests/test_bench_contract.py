"""Host-side logic of bench.py: the roofline and per-kernel rate arithmetic, the traffic table's
validity by source hash, and the one-GPU rule.  No GPU is touched."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _prof():
    # per-kernel totals as the library's profile reports them: time, launches, work (bytes or flops)
    return {
        "trsv": {"total_ms": 8.6, "count": 10, "work": 10 * 4.0e9},
        "lu_update": {"total_ms": 5.0, "count": 5, "work": 5 * 6.0e10},
        "mgs": {"total_ms": 0.5, "count": 100, "work": 100 * 1.6e7},
    }


def test_roofline_picks_the_dominant_kernel_and_divides_algorithmic_work_by_time():
    r = bench.roofline(_prof(), "fp64", None, read_peak=5000.0)
    assert r["kernel"] == "trsv" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(4.0e10 / 8.6e-3 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, rel=1e-3)
    assert r["frac_of_measured_read_peak"] == pytest.approx(r["achieved"] / 5000.0, rel=1e-3)
    assert r["avg_launch_ms"] == pytest.approx(0.86) and r["launches"] == 10


def test_roofline_of_an_mfma_kernel_reports_the_executed_share(monkeypatch):
    monkeypatch.setattr(bench, "measured_mfma_peak", lambda prec: 70.0)
    prof = {"lu_update": {"total_ms": 5.0, "count": 5, "work": 5 * 6.0e10}}
    r = bench.roofline(prof, "fp64", None)
    assert r["bound"] == "mfma" and r["peak"] == bench.PEAK_FP64_TFLOPS
    assert r["achieved"] == pytest.approx(3.0e11 / 5e-3 / 1e12, rel=1e-3)
    assert r["mfma_executed_frac"] == pytest.approx(0.75 * r["achieved"] / bench.PEAK_FP64_TFLOPS, rel=1e-3)
    assert r["mfma_executed_frac_of_measured_peak"] == pytest.approx(0.75 * r["achieved"] / 70.0, rel=1e-3)
    r32 = bench.roofline(prof, "mixed", None)
    assert r32["peak"] == bench.PEAK_FP32_TFLOPS


def test_kernel_table_rates_per_step():
    t = bench.kernel_table(_prof(), 5, "fp64")
    assert t["trsv"]["count"] == 2 and t["trsv"]["total_ms"] == pytest.approx(1.72)
    assert t["trsv"]["avg_us"] == pytest.approx(860.0)
    assert t["trsv"]["GBs"] == pytest.approx(4.0e10 / 8.6e-3 / 1e9, rel=1e-3)
    assert "TFLOPs" in t["lu_update"] and "GBs" not in t["lu_update"]
    assert t["mgs"]["frac"] == pytest.approx(t["mgs"]["GBs"] / 8000.0, rel=1e-3)


def test_traffic_is_reported_only_for_the_sources_it_was_measured_on():
    for group in bench.PMC_GROUPS:
        assert len(bench.group_source_hash(group)) == 16
    assert bench.measured_traffic("c2", "fp64", "no_such_kernel") is None
    assert bench.measured_traffic("no_such_workload", "fp64", "trsv") is None
    for wl, rec in bench.PMC_MEASURED.items():
        for (prec, kernel), nbytes in rec["bytes"].items():
            group = bench.PMC_KERNEL_GROUP[kernel]
            current = rec["hash"].get(group) == bench.group_source_hash(group)
            assert bench.measured_traffic(wl, prec, kernel) == (nbytes if current else None), (wl, kernel)
    # a changed source of the group nulls the figure
    saved = bench.group_source_hash
    try:
        bench.group_source_hash = lambda g: "0" * 16
        assert all(bench.measured_traffic(wl, p, k) is None
                   for wl, rec in bench.PMC_MEASURED.items() for (p, k) in rec["bytes"])
    finally:
        bench.group_source_hash = saved


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
