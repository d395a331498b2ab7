"""The benchmark's contract on the CPU: one GPU only (a request for more is
refused with a message), the default run's legs and their switches, and the
roofline's per-pair pricing (flops plus each transcendental at
peak / measured rate; the fused sweep's count is the two sweeps' sum)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_help_lists_the_default_legs_and_their_switches():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0
    for flag in ("--no-batch", "--no-serve-quick", "--serve-abba", "--copy-calibration", "--mode"):
        assert flag in r.stdout


def test_flop_equivalents_per_pair():
    rates = {"fma": 5e13, "sin": 2e13, "cos": 1e13, "rcp": 4e13}
    peak = bench.PEAK_TFLOPS * 1e12
    for kind, a in bench.ALG.items():
        want = a["flops"] + a["sin"] * peak / 2e13 + a["cos"] * peak / 1e13 + a["rcp"] * peak / 4e13
        assert bench.flop_eq(kind, rates) == pytest.approx(want, rel=1e-12)
    for m in ("volume", "surface"):
        fused, fwd, vjp = bench.ALG["fused_" + m], bench.ALG["fwd"], bench.ALG["vjp_" + m]
        assert all(fused[k] == fwd[k] + vjp[k] for k in fwd)


def test_traffic_is_reported_only_for_the_source_it_was_measured_on():
    t = bench.TRAFFIC
    assert t["bytes_per_launch"] == t["read_bytes"] + t["write_bytes"]
    assert bench.measured_traffic("some other kernel") is None
    got = bench.measured_traffic(t["kernel"])
    assert got is None or got == t["bytes_per_launch"]
    assert (got is not None) == (bench.kernel_source_sha256() == t["source_sha256"])
