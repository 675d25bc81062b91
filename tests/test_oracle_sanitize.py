"""The CPU oracle under host AddressSanitizer and UndefinedBehaviorSanitizer:
tests/oracle_sanitize_main.c walks every oracle entry point on small inputs
(rules, adaptive runs with each rule and with pruning, batch, fixed-tree
quadrature and gradient); any out-of-bounds access, leak or undefined
operation fails the run."""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_host_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_sanitize")
        cmd = ["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "gm_oracle.c"),
               os.path.join(ROOT, "tests", "oracle_sanitize_main.c"), "-lm", "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        p = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert p.returncode == 0, p.stderr[-4000:]
        assert "runtime error" not in p.stderr and "ERROR:" not in p.stderr, p.stderr[-4000:]
        assert "oracle sanitize run ok" in p.stdout
