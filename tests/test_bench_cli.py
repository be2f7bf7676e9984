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
    """The oracle on all host cores (at most 16 threads, one copy of the sample each);
    the host's CPU count and model are stated."""
    sys.path.insert(0, ROOT)
    import bench
    b = bench.cpu_baseline(n_sample=64, max_threads=3)
    assert b["kind"] == "oracle" and b["cores"] == min(3, os.cpu_count()) and b["value"] > 0
    assert "64x64" in b["sample"] and b["nproc"] == os.cpu_count() and b["cpu_model"]
    assert b["per_thread_value"] > 0


def test_algorithmic_bytes():
    """Section 2's stage structure: a stage reads its input (and u^n in stages 2, 3) and
    writes its output once: 64/96/96 B per 2D cell, 256 per cell-update; the 2D x-sweep
    carries none of them."""
    from paper_2108_12742_amd import roofline as R
    assert [R.stage_bytes("euler2d", s) for s in (1, 2, 3)] == [64, 96, 96]
    assert R.cell_update_bytes("euler2d") == 256 and R.cell_update_bytes("euler1d") == 192
    assert R.algorithmic_bytes("euler2d", "x", 2) == 0 and R.algorithmic_bytes("euler2d", "y", 2) == 96
    assert R.algorithmic_bytes("euler1d", "x", 1) == 48
    e = R.hbm_entry(96 * 4194304, 140.6e-6)
    assert e["bound"] == "hbm" and abs(e["frac"] - 0.358) < 1e-3


def test_failing_extra_leg_is_recorded():
    """An extra leg that raises is reported in its own entry; the others and the main
    line go on.  A failed 8-stream baseline leaves the batched entry without a speedup."""
    sys.path.insert(0, ROOT)
    import bench
    out = {}
    bench.run_leg(out, "broken", lambda: 1 / 0)
    bench.run_leg(out, "fine", lambda k: {"value": k}, k=2)
    assert out["broken"] == {"error": "ZeroDivisionError: division by zero"} and out["fine"] == {"value": 2}
    batched = {"value": 1.0e10}
    bench.add_plain_8streams(batched, {"error": "RuntimeError: child failed"})
    assert batched["plain_8streams_error"] == "RuntimeError: child failed"
    assert "speedup_vs_plain_8streams" not in batched
    ok = {"value": 1.0e10}
    bench.add_plain_8streams(ok, {"values": {"cooperative": 2.0e8, "streaming": 2.5e8}, "identical": True,
                                  "streaming_by_stream_set": [2.5e8, 2.2e8]})
    assert ok["plain_8streams_solver"] == "streaming" and ok["speedup_vs_plain_8streams"] == 40.0
