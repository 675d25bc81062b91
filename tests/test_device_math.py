"""Accuracy of the FP64 exp and cos that the rule kernel uses for its outer
functions, and of the sin of the adjoint kernel (paper_2511_01573_amd/csrc/
gm_math.hpp), compiled for the host from the same source, against 50-digit
references."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import tempfile

import mpmath as mp
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def harness():
    d = tempfile.mkdtemp()
    so = os.path.join(d, "libgmmath.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
                           "-I", os.path.join(ROOT, "paper_2511_01573_amd", "csrc"),
                           os.path.join(ROOT, "tests", "math_harness.cpp"), "-o", so])
    L = C.CDLL(so)
    for f in (L.gm_test_exp, L.gm_test_cos, L.gm_test_sin):
        f.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_long]
    return L


def call(f, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros_like(x)
    f(x.ctypes.data_as(C.POINTER(C.c_double)), y.ctypes.data_as(C.POINTER(C.c_double)), x.size)
    return y


def ulp_err(y, ref):
    out = np.zeros(len(y))
    for i, (a, b) in enumerate(zip(y, ref)):
        if b == 0:
            out[i] = 0.0 if a == 0 else np.inf
            continue
        u = max(mp.mpf(2) ** (mp.floor(mp.log(abs(b), 2)) - 52), mp.mpf(2) ** -1074)
        out[i] = float(abs(mp.mpf(a) - b) / u)
    return out


def test_exp_within_one_ulp(harness):
    mp.mp.dps = 50
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-30, 30, 3000), rng.uniform(-745, 709, 1000),
                        rng.uniform(-1e-3, 1e-3, 500), [0.0, -0.0, 1.0, -1.0, 709.7, -708.3]])
    y = call(harness.gm_test_exp, x)
    ref = [mp.exp(mp.mpf(v)) for v in x]
    e = ulp_err(y, ref)
    assert e.max() <= 1.0, (e.max(), x[np.argmax(e)])


def test_exp_special_values(harness):
    y = call(harness.gm_test_exp, [-np.inf, -2000.0, -746.0, 710.0, np.inf])
    assert y[0] == 0.0 and y[1] == 0.0 and y[2] == 0.0
    assert np.isinf(y[3]) and y[3] > 0


def test_cos_error_bound(harness):
    mp.mp.dps = 60
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.uniform(-10, 10, 3000), rng.uniform(-200, 200, 1000),
                        rng.uniform(-1e5, 1e5, 300), np.arange(-20, 21) * (np.pi / 2),
                        [0.0, 1e-300, 2e6, -3e7]])
    y = call(harness.gm_test_cos, x)
    ref = np.array([float(mp.cos(mp.mpf(v))) for v in x])
    # absolute error within 1.5 ulp of 1 (the reduction is exact to ~2^-106 |x|)
    err = np.abs(y - ref)
    assert err.max() <= 1.5 * 2.0 ** -52, (err.max(), x[np.argmax(err)])
    # and within 1 ulp relative where |cos x| >= 1/2
    big = np.abs(ref) >= 0.5
    rel = err[big] / np.abs(ref[big])
    assert rel.max() <= 2.0 ** -52


def test_sin_error_bound(harness):
    """sin (the oscillatory family's derivative in the adjoint kernel): within
    1.5 ulp of 1 absolutely and 1.5 ulp relative where |sin x| >= 1/2 (the
    leading term rh and its correction are rounded once more than cos's), and
    within 1 ulp near the zeros below pi/2 (no cancellation in the reduction
    there)."""
    mp.mp.dps = 60
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.uniform(-10, 10, 3000), rng.uniform(-200, 200, 1000),
                        rng.uniform(-1e5, 1e5, 300), np.arange(-20, 21) * (np.pi / 2),
                        [0.0, 1e-300, 2e6, -3e7]])
    y = call(harness.gm_test_sin, x)
    ref = np.array([float(mp.sin(mp.mpf(v))) for v in x])
    err = np.abs(y - ref)
    assert err.max() <= 1.5 * 2.0 ** -52, (err.max(), x[np.argmax(err)])
    big = np.abs(ref) >= 0.5
    rel = err[big] / np.abs(ref[big])
    assert rel.max() <= 1.5 * 2.0 ** -52
    small = rng.uniform(-1.5, 1.5, 2000) * 10.0 ** rng.uniform(-12, 0, 2000)
    ys = call(harness.gm_test_sin, small)
    refs = [mp.sin(mp.mpf(v)) for v in small]
    assert ulp_err(ys, refs).max() <= 1.0
