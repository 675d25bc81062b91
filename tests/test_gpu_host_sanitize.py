"""libgm's host code under AddressSanitizer and UndefinedBehaviorSanitizer:
tests/libgm_sanitize_main.cpp, linked with the host-logic units (gm_api,
gm_batch, gm_grad) built with host-side -fsanitize=address,undefined by
paper_2511_01573_amd/build.py (build_host_sanitize, called from the repository's
build step), walks every C-ABI entry point on the GPU: argument checks, runs
of every family and rule, pruning, timing, forced stops, the region-list rule,
gradient, batch, caller-owned workspace and the no-allocation entry point.
Any host out-of-bounds access, use after free or undefined operation fails
the run (device code is not instrumented).  LeakSanitizer is off by default:
its exit-time scan takes about 2.5 minutes with the ROCm runtime loaded; with
GM_SANITIZE_LEAKS=1 it runs, and reports only allocations the HSA runtime
keeps until exit (suppressed in tests/libgm_sanitize.supp)."""
from __future__ import annotations

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2511_01573_amd", "gm_host_sanitize")

pytestmark = pytest.mark.gpu


def test_libgm_host_code_clean_under_sanitizers():
    assert os.path.exists(EXE), "build it: python paper_2511_01573_amd/build.py --host-sanitize"
    supp = os.path.join(ROOT, "tests", "libgm_sanitize.supp")
    leaks = os.environ.get("GM_SANITIZE_LEAKS", "0") == "1"
    env = dict(os.environ,
               ASAN_OPTIONS=f"detect_leaks={int(leaks)}:abort_on_error=0:halt_on_error=1",
               LSAN_OPTIONS=f"suppressions={supp}:print_suppressions=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    print("running", EXE, flush=True)
    p = subprocess.run([EXE], capture_output=True, text=True, timeout=400 if leaks else 120, env=env)
    tail = (p.stdout[-2000:] + "\n" + p.stderr[-6000:])
    assert p.returncode == 0, tail
    assert "runtime error" not in p.stderr and "ERROR: AddressSanitizer" not in p.stderr, tail
    assert "ERROR: LeakSanitizer" not in p.stderr, tail
    assert "libgm sanitize run ok" in p.stdout, tail
