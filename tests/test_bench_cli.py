"""Benchmark host side on the CPU: more than one GPU is refused with a message before
anything touches a device, and the CPU baseline leg (the oracle on a bounded sample)."""
import subprocess
import sys
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and r.stdout == ""
    assert "one GPU" in r.stderr


def test_cpu_baseline_leg():
    sys.path.insert(0, ROOT)
    import bench
    b = bench.cpu_baseline(n_sample=64, steps=1)
    assert b["kind"] == "oracle" and b["cores"] == 1 and b["value"] > 0 and "64x64" in b["sample"]
