"""The benchmark's host-side contract (no GPU): a run on more than one GPU is refused
with a message (the hot path is a single-device build), the roofline entry is the
algorithmic work over the duration against the stated peak, and the stored HBM traffic
of the dominant kernel is the counters scaled by their copy calibration."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_roofline_entry():
    # 2.1746e9 flop in 34.81 us against the FP32 vector peak (the default workload)
    e = bench._roof("alu", 2.1746e9, 34.81, bench.PEAK_FP32_VECTOR, "TFLOP/s", "k")
    assert e["achieved"] == pytest.approx(2.1746e9 / 34.81e-6 / 1e12)
    assert e["frac"] == pytest.approx(2.1746e9 / 34.81e-6 / 157.3e12)
    assert e["peak"] == pytest.approx(157.3)
    assert e["avg_launch_us"] == 34.81 and e["work_per_launch"] == 2.1746e9


def test_flops_per_pair_and_traffic():
    # the survey's count of one Eq. 1 pair term: 3 + 5 + 2 + 5 + 2 + 12
    assert bench.FLOPS_PER_PAIR == 3 + 5 + 2 + 5 + 2 + 12
    t = bench.TRAFFIC_BYTES["k_field<float,16,3>"]
    assert t == pytest.approx((1412.69 * 2.0 + 703.13 * 1.0) * 1024)
    # 5.0 times the algorithmic 48 B per particle and replica of the default workload
    assert t / (bench.ALG_BYTES_PER_NP * 5000 * 3) == pytest.approx(5.02, abs=0.01)
