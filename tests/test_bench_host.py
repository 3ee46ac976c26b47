"""Host logic of bench.py (no GPU): the one-GPU refusal, the roofline
arithmetic, and that counter figures are reported only for the sources
they were taken on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_roofline_arithmetic():
    n2, launch_s = 1 << 20, 40e-6
    roof = bench.roofline(n2, launch_s, flops_cell=1400.0, bytes_cell=100.0, prec="f64", key=("none", 1, 1, "f64"),
                          kernel="k")
    alu, hbm = (roof, roof["other_bound"]) if roof["bound"] == "alu" else (roof["other_bound"], roof)
    assert alu["achieved"] == pytest.approx(1400.0 * n2 / launch_s / 1e12, rel=1e-3)
    assert alu["peak"] == bench.FP64_PEAK_TFLOPS and alu["unit"] == "TFLOP/s"
    assert hbm["achieved"] == pytest.approx(100.0 * n2 / launch_s / 1e9, rel=1e-3)
    assert hbm["peak"] == bench.HBM_PEAK_GBS and hbm["unit"] == "GB/s"
    for b in (alu, hbm):
        assert b["frac"] == pytest.approx(b["achieved"] / b["peak"], abs=1e-4)
    assert roof["algorithmic_flops_per_launch"] == 1400.0 * n2
    assert roof["stage_us_per_launch"] == pytest.approx(40.0)
    # the bound reported is the one with the larger fraction
    assert roof["frac"] >= roof["other_bound"]["frac"]
    # no counters were taken for this workload: traffic is null, not guessed
    assert roof["traffic"] is None and "valu_issue" not in roof
    f32 = bench.roofline(n2, launch_s, 1500.0, 100.0, "f32", ("none", 1, 1, "f32"), "k")
    assert (f32 if f32["bound"] == "alu" else f32["other_bound"])["peak"] == bench.FP32_PEAK_TFLOPS


def test_counter_figures_only_for_their_sources(monkeypatch):
    key = ("cylinder", 1024, 512, "f64")
    entry = bench.MEASURED[key]
    assert len(entry["sources_sha256"]) == 64
    assert os.path.exists(os.path.join(ROOT, entry["profile"]))
    monkeypatch.setattr(bench, "stage_sources_sha256", lambda: entry["sources_sha256"])
    assert bench.measured(key) is entry
    roof = bench.roofline(524288, 34e-6, 1404.0, 86.3, "f64", key, "k")
    assert roof["traffic"] == entry["bytes_per_launch"] and "valu_issue" in roof
    monkeypatch.setattr(bench, "stage_sources_sha256", lambda: "0" * 64)
    assert bench.measured(key) is None
    assert bench.roofline(524288, 34e-6, 1404.0, 86.3, "f64", key, "k")["traffic"] is None
