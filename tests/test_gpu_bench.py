"""bench.py's one JSON line on a short run of the headline workload: the
fields and types of the line, a roofline whose achieved rate follows from the
timed scan and the algorithmic bytes, and a round time that at least covers
the scan.  (The CPU baseline, batched and report legs are left out to keep
the run short; the default run adds them.)"""
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


def test_bench_line_contract():
    print("bench.py, 5 timed rounds of the headline workload", flush=True)
    cmd = [sys.executable, "bench.py", "--steps", "5", "--warmup", "2", "--no-cpu-baseline", "--batched=",
           "--sweep-precisions=", "--variants=", "--precision-rounds", "0", "--classifier-rounds", "0",
           "--no-retrain"]
    r = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=280)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [x for x in r.stdout.splitlines() if x.strip()]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    for k, t in (("metric", str), ("value", float), ("unit", str), ("n_gpus", int), ("steps", int), ("warmup", int),
                 ("ms_per_step", float), ("higher_is_better", bool), ("scaling", str), ("dtype", str),
                 ("data", str), ("config", dict), ("roofline", dict)):
        assert isinstance(d[k], t), k
    assert d["n_gpus"] == 1 and d["steps"] == 5 and d["warmup"] == 2
    assert d["higher_is_better"] is False and d["value"] == d["ms_per_step"] and d["value"] > 0
    assert d["vs_baseline"] is None
    assert d["config"]["workload"].startswith("162,336 Haar features x 15,000 windows")
    assert d["config"]["precision"] == "fp32_kahan"
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["alg_bytes_per_launch"] == 162336 * 15000 * 2
    # achieved = algorithmic bytes / the timed scan; the round covers the scan
    assert abs(rf["achieved"] - rf["alg_bytes_per_launch"] / (d["scan_ms_avg"] * 1e-3) / 1e9) <= 0.01 * rf["achieved"]
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert 0.3 < rf["frac"] < 1.0
    assert rf["traffic"] is None or 0.99 * rf["alg_bytes_per_launch"] < rf["traffic"] < 1.1 * rf["alg_bytes_per_launch"]
    assert d["scan_ms_avg"] <= d["event_instrumented_ms_per_round"]
    assert d["cpu_baseline"] is None
