"""The bench.py contract: one JSON line with the required keys (GPU), and a
clear refusal of more than one GPU (host only)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "--gpus 2" in r.stderr and r.stdout.strip() == ""


@pytest.mark.gpu
@pytest.mark.parametrize("cfg", ["c1", "c3", "c4b"])
def test_bench_line(cfg):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--config", cfg,
                        "--steps", "3", "--warmup", "1", "--no-cpu", "--no-copy", "--no-schemes"],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k, t in (("metric", str), ("value", float), ("unit", str), ("n_gpus", int),
                 ("steps", int), ("warmup", int), ("ms_per_step", float),
                 ("higher_is_better", bool), ("scaling", str), ("dtype", str), ("data", str),
                 ("config", dict), ("roofline", dict)):
        assert isinstance(d[k], t), k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1
    assert "workload" in d["config"] and "vs_baseline" in d
    assert d["kernel_ms_mean"] > 0
    if cfg in ("c1", "c3"):
        # batched vs per-image at the same accuracy (the default line carries
        # it beside the headline; the c3 line is the batched run itself)
        b = d["batched"]
        assert b["pairs"] == 64 and b["speedup_vs_per_image"] > 0
        a = b["accuracy"]
        assert a["same_bound"] and a["invalid_mismatches_batched"] == 0
        assert a["invalid_mismatches_per_image"] == 0
    if cfg == "c3":
        assert d["config"]["pairs"] == 64
    else:
        ev = d["per_launch_events"]
        assert 0 < ev["min_ms"] <= ev["median_ms"]
        a = d["accuracy"]
        assert a["flag_mismatches"] == 0 and a["flag_launch_equals_timed"]
        if cfg == "c1":
            assert a["bit_exact"] and not a["sampled"] and a["outputs_checked"] == 12_000_000
        else:
            assert a["within_bound"] and a["invalid_mismatches"] == 0
    roof = d["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3
    assert roof["traffic"] is None or roof["traffic"] > 0
