"""bench.py's output on a GPU: one JSON line with the metric, the throughput and its
context, a roofline object for the dominant kernel (with the whole-step fraction
and the half-sweep on a grid that streams from HBM), the serving and batch
objects and the CPU baseline of the oracle (a short run: two timed steps, three
small requests in each time-to-steady leg, a one-second oracle budget)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_complete_json_line():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "2", "--warmup", "1",
                        "--cpu-budget", "1", "--serving", "3", "--batch-steady", "3", "--stream-grid", "161"],
                       cwd=ROOT, capture_output=True, text=True, timeout=400)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [ln for ln in p.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, p.stdout[-2000:]
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["unit"] == "cell-updates/s" and d["value"] > 0 and d["higher_is_better"] is True
    assert d["dtype"] == "f64" and d["data"] == "synthetic" and "129^3" in d["config"]["workload"]
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert 0.0 < r["achieved"] < r["peak"] and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12
    assert r["traffic"] is None or r["traffic"] > 0
    st = r["step"]
    assert st["bytes_per_step"] > 0 and abs(st["frac"] - st["achieved"] / 8000.0) < 1e-12
    hs = r["hbm_streaming"]
    assert hs["grid"] == 161 and 0.0 < hs["frac"] < 1.0
    sv = d["serving"]
    assert sv["requests"] == 3 and sv["served_fp32_refined"]["steady"] >= 1
    assert sv["mix_vs_alone"]["sampled"] >= 1
    assert sv["mix_vs_alone"]["bitwise_equal"] == sv["mix_vs_alone"]["sampled"]
    b = d["batch"]
    assert b["cavities"] == 12 and b["max_abs_diff_vs_single_cavity"] == 0.0
    bt = b["to_steady"]
    assert bt["requests"] == 3 and bt["steady"] >= 1 and bt["steady"] + bt["failed"] <= 3
    assert bt["sampled"] >= 1 and bt["sampled_same_as_alone"] == bt["sampled"]
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["unit"] == "cell-updates/s" and c["value"] > 0 and c["cores"] >= 1
    assert "129^3" in c["sample"]
