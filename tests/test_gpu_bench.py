"""The benchmark's JSON output on a short run: detail lines, then the compact
headline as the last line, with the metric, the roofline object of the rule
kernel (bound, achieved, peak, unit, frac, traffic) and the CPU-oracle
baseline (value, unit, cores, kind, sample)."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_has_the_contract_fields():
    print("case bench short run", flush=True)
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "1", "--warmup",
                        "0", "--no-modes", "--taus", "1e-3,1e-5", "--cpu-seconds", "1"],
                       capture_output=True, text=True, timeout=110)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [l for l in p.stdout.splitlines() if l.strip()]
    # detail sections first, the compact headline last
    assert len(lines[-1].encode()) < 4096
    for l in lines[:-1]:
        assert "detail" in json.loads(l)
    out = json.loads(lines[-1])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config"):
        assert k in out, k
    assert out["n_gpus"] == 1 and out["steps"] == 1 and out["dtype"] == "f64"
    assert out["value"] > 0 and "workload" in out["config"]
    r = out["roofline"]
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert 0 < r["frac"] < 1 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12
    assert "traffic" in r
    cb = out["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] == 1 and cb["value"] > 0 and cb["sample"]


def test_full_bench_last_line_is_compact_and_complete():
    """The default benchmark with every mode (short steps and CPU sample): the
    detail lines come first and the last line, the one the record keeps, is a
    complete headline under 4 KB."""
    print("case bench full run", flush=True)
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "1", "--warmup",
                        "1", "--cpu-seconds", "1"], capture_output=True, text=True, timeout=600)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [l for l in p.stdout.splitlines() if l.strip()]
    last = lines[-1]
    assert len(last.encode()) < 4096, len(last)
    out = json.loads(last)
    for k in ("roofline", "cpu_baseline", "split_compaction", "batch", "grad", "config3",
              "degree9_suite", "time_to_tolerance_ms_by_rel_tol"):
        assert k in out, k
    assert out["grad"]["rel_tol"] == 1e-8 and out["grad"]["status"] == 0
    assert out["batch"]["all_ok"] and out["batch"]["speedup_vs_single_calls"] > 1
    assert set(out["config3"]) == {"corner_peak_d12", "product_peak_d12", "corner_peak_d16",
                                   "product_peak_d16"}
    assert out["cpu_baseline"]["omp"]["cores"] >= 1
    details = {json.loads(l)["detail"] for l in lines[:-1]}
    assert {"cases", "batch", "grad", "config3", "gauss_kronrod", "prune", "degree9"} <= details
