"""The benchmark's output contract, on a reduced size: one JSON line with the metric,
the whole-job value, the roofline of the dominant kernel and the per-kernel times."""
import io
import json
import sys
from contextlib import redirect_stdout

import pytest

pytestmark = pytest.mark.gpu


def _run_bench(argv):
    import bench
    old = sys.argv
    sys.argv = ["bench.py"] + argv
    buf = io.StringIO()
    try:
        with redirect_stdout(buf):
            bench.main()
    finally:
        sys.argv = old
    lines = [l for l in buf.getvalue().splitlines() if l.strip()]
    assert len(lines) == 1, lines
    return json.loads(lines[0])


def test_bench_json_line():
    d = _run_bench(["--n", "256", "--steps", "4", "--warmup", "1", "--no-extras", "--no-cpu-baseline", "--no-tune"])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "kernels"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 4 and d["warmup"] == 1 and d["higher_is_better"] is True
    assert d["unit"] == "cell-updates/s" and d["dtype"] == "f64" and d["vs_baseline"] is None
    assert d["config"]["workload"] == "euler2d-quadrants-256x256-ao5"
    assert abs(d["value"] - 256 * 256 * 4 / (d["ms_per_step"] * 4e-3)) <= 1e-6 * d["value"]
    r = d["roofline"]
    assert r["bound"] in ("hbm", "mfma", "alu") and r["unit"] in ("GB/s", "TFLOP/s")
    assert r["peak"] > 0 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    assert r["traffic"] is None  # no byte counters were recorded for this size
    sweeps = {k: v for k, v in d["kernels"].items() if k.startswith("sweep")}
    assert len(sweeps) in (3, 6) and all(v["launches"] == 4 for v in sweeps.values())
    assert r["kernel"] in {v["symbol"] for v in sweeps.values()}
    # the dominant kernel completes a stage: HBM roof on the stage's algorithmic bytes
    assert r["bound"] == "hbm" and r["algorithmic_bytes_per_cell"] in (64, 96)
    st = r["step"]
    assert st["bytes_per_cell_update"] == 256
    assert abs(st["achieved_gbs"] - 256 * d["value"] / 1e9) <= 1e-3 * st["achieved_gbs"]
