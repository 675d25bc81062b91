"""Host-side checks of the benchmark script: it refuses more than one GPU
before touching any device, and the HBM-traffic figure it reports comes from
a counter summary taken on the current rule-kernel sources."""
from __future__ import annotations

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_traffic_summary_matches_the_rule_sources():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.measured_traffic() is not None, (
        "profiles/rule_kernel_d8_suite_counters.md was taken on other rule-kernel sources")
