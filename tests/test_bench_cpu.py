"""Host logic of bench.py (no GPU): the roofline arithmetic, the counter-summary check and
the single-GPU rule."""
import os
import subprocess
import sys

import pytest

import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_roofline_arithmetic():
    inst = wl.day_hourly_small()
    per_launch = inst.candidates() / inst.T
    r = bench.roofline_of(inst, (2.0e-3 * inst.T, inst.T, 1.0e-3 * inst.T, inst.T), 12345)
    assert r["bound"] == "alu" and r["unit"] == "Gupd/s"
    assert r["avg_launch_us"] == pytest.approx(2.0)
    assert r["achieved"] == pytest.approx(per_launch / 2.0e-6 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], rel=1e-3, abs=1e-4)
    # an add and a max per candidate on 256 CUs x 4 SIMDs x 32 FP32 lanes at 2.4 GHz, which
    # is the published FP32 vector peak (157.3 TFLOP/s) at two operations per candidate
    assert r["peak"] == pytest.approx(256 * 4 * 32 * 2.4e9 / 2 / 1e9, rel=1e-6)
    assert r["peak"] == pytest.approx(157.3e12 / 2 / 2 / 1e9, rel=1e-3)
    assert r["traffic"] == 12345
    e = r["expectation"]
    flop = 2.0 * inst.K ** 2 * inst.storage.S
    assert e["achieved"] == pytest.approx(flop / 1.0e-6 / 1e12, rel=1e-3, abs=1e-3)
    assert e["peak"] == 157.3


def test_traffic_summary_matches_kernel_source():
    # a committed counter summary counts only while it is for the current sweep source
    import hashlib
    digest = hashlib.sha256(open(bench.KERNEL_SOURCE, "rb").read()).hexdigest()
    for workload in ("year_hourly", "day_5min"):
        path = bench.traffic_file(workload)
        t = bench.measured_traffic(workload)
        if not os.path.exists(path):
            assert t is None
            continue
        fields = dict(line.split(":", 1) for line in open(path)
                      if not line.startswith("#") and ":" in line)
        if fields["kernel_source_sha256"].strip() == digest:
            assert t == int(fields["bytes_per_launch"])
        else:
            assert t is None
    assert bench.measured_traffic("no_such_workload") is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "single GPU" in p.stderr
