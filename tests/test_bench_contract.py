"""CPU checks of bench.py's contract: one GPU only, the peaks it prices against, and the committed HBM-traffic summary
matching the current GETT source (bench.py reports `traffic` only while it does)."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_peaks():
    assert bench.PEAK_TFLOPS["fp32"] == pytest.approx(157.3)
    assert bench.PEAK_TFLOPS["fp64"] == pytest.approx(78.6)
    # three bf16 products per multiply-add share the 2.5 PFLOP/s dense bf16 peak
    assert bench.PEAK_TFLOPS["bf16x3"] == pytest.approx(2500.0 / 3)


def test_committed_traffic_summary_matches_the_kernel_source():
    src = os.path.join(ROOT, "paper_2007_03638_amd", "csrc", "gett.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    summary = open(os.path.join(ROOT, "profiles", "gett_f32_chi24_counters.md")).read()
    assert f"gett_source_sha256_prefix: {sha}" in summary
    traffic = bench.counter_traffic("gett<f32,192x192,Am,Bn,v,k2>")
    assert traffic is not None and 1e9 < traffic < 2e10
    # another variant has no committed figure
    assert bench.counter_traffic("gett<f32,128x128,Am,Bn,v,k2>") is None
