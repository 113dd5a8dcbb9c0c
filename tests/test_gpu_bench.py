"""The benchmark's output contract on a GPU: one JSON line with the metric,
the whole-job value, the roofline object of the dominant kernel and the
workload description (a short run: 4 timed steps, no variants, no CPU leg)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_json_line():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "4", "--warmup", "2",
                        "--no-variants", "--no-cpu"], capture_output=True, text=True, timeout=110)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["unit"] == "MLUPS" and d["n_gpus"] == 1 and d["steps"] == 4 and d["warmup"] == 2
    assert d["value"] > 0 and d["higher_is_better"] is True and d["dtype"] == "f32"
    assert "workload" in d["config"]
    roof = d["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert 0 < roof["frac"] < 1 and abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3
    # the stated error of the FP32 run against the FP64 oracle (1000 steps)
    err = d["error_vs_fp64"]
    assert err is not None and err["steps"] == 1000
    assert err["rho"] < 1e-5 and err["u"] < 1e-5 and err["T"] < 1e-5
    # MLUPS and the roofline come from the same launches: 592 bytes per cell-step
    assert abs(d["value"] * 1e6 * 592 / 1e9 - roof["achieved"]) / roof["achieved"] < 0.05
