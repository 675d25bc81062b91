"""The -DGM_CHECK build (paper_2511_01573_amd/libgm_check.so, built by the
repository's build step): every kernel index the check covers (region
records, per-region results, tile counts and offsets, split destinations,
leaf slots, batch store rows and items) is compared with its buffer's size; a
violation makes the call return GM_EHIP.  The cases of
tests/bounds_check_cases.py (every family at d = 3 and 8 through both
bookkeeping paths, every rule-kernel mapping, d = 12 and 16, the degree-9 and
Gauss-Kronrod rules, pruning, gradients, the no-allocation entry point, a
128-item batch and the region-list rule) run in a child process on the check
build: none may report a violation, and every result must equal, bit for
bit, that of the same cases on libgm.so in this process.  A self-test first
checks (without any memory access) an index one past its bound and expects
the call to report it."""
from __future__ import annotations

import json
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHECK_LIB = os.path.join(ROOT, "paper_2511_01573_amd", "libgm_check.so")
sys.path.insert(0, os.path.join(ROOT, "tests"))

pytestmark = pytest.mark.gpu


def _same(a, b):
    if isinstance(a, list):
        return len(a) == len(b) and all(_same(x, y) for x, y in zip(a, b))
    if isinstance(a, float) and math.isnan(a):
        return isinstance(b, float) and math.isnan(b)
    return a == b


def test_check_build_reports_no_violation_and_gives_the_same_bits():
    assert os.path.exists(CHECK_LIB), "build it: python paper_2511_01573_amd/build.py --check"
    print("check build: child process", flush=True)
    p = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "bounds_check_cases.py"),
                        "--lib", CHECK_LIB, "--selftest"], capture_output=True, text=True,
                       timeout=240)
    assert p.returncode == 0, p.stderr[-4000:]
    checked = json.loads(p.stdout.strip().splitlines()[-1])
    # the check path itself: an index one past its bound (checked, never
    # accessed) is reported as GM_EHIP naming the index and the bound
    st = checked.pop("selftest")
    assert st["rc"] == -3, st
    assert "index 12345, bound 12345" in st["text"] and "(1 violations)" in st["text"], st
    print("normal build: this process", flush=True)
    import bounds_check_cases as cases
    normal = cases.run_cases()
    assert set(checked) == set(normal)
    for k in normal:
        assert _same(checked[k], normal[k]), (k, checked[k], normal[k])
