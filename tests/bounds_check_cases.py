"""Cases of the bounds-check test (tests/test_gpu_bounds_check.py): every kernel
of the library on small inputs, through the Python binding.  run_cases()
returns every result as plain numbers; run as a script with --lib PATH it loads
that library (the -DGM_CHECK build) instead of libgm.so and prints the results
as one JSON line."""
from __future__ import annotations

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2511_01573_amd import gm, workloads as W  # noqa: E402


def _f(x):
    return [float(v) for v in np.atleast_1d(np.asarray(x, dtype=np.float64))]


def _run(out, key, fn, *args, opts=None):
    opts = opts or {}
    for k, v in opts.items():
        gm.set_option(k, v)
    try:
        print(f"case {key}", file=sys.stderr, flush=True)
        r = fn(*args)
        s = gm.last_stats()
        out[key] = {"r": [_f(v) if isinstance(v, (np.ndarray, list)) else float(v) for v in r],
                    "iterations": int(s["iterations"]), "regions": int(s["regions_evaluated"])}
    finally:
        defaults = {"rule": 0, "prune": 0, "timing": 0, "lanes_per_region": 0,
                    "init_log2_regions": 12, "err_model": 0}
        for k in opts:
            gm.set_option(k, defaults[k])


def run_cases() -> dict:
    out: dict = {}
    box = W.unit_box
    for fam in range(1, 8):
        for d, tau in ((3, 1e-7), (8, 1e-4)):
            p = W.family_params(fam, d, seed=100 * fam + d)
            _run(out, f"fam{fam}_d{d}", gm.integrate, fam, p, *box(d), tau, 1e-16, 1 << 20)
            _run(out, f"fam{fam}_d{d}_four_kernels", gm.integrate, fam, p, *box(d), tau, 1e-16,
                 1 << 20, opts={"timing": 2})
    for lanes in (1, 4, 16, 64):
        p = W.family_params(4, 10, seed=410)
        _run(out, f"d10_lanes{lanes}", gm.integrate, 4, p, *box(10), 1e-3, 1e-16, 1 << 20,
             opts={"lanes_per_region": lanes})
    _run(out, "d12_corner", gm.integrate, 3, W.family_params(3, 12, seed=312, difficulty=1.0),
         *box(12), 1e-3, 1e-16, 1 << 20)
    _run(out, "d16_product", gm.integrate, 2, W.family_params(2, 16, seed=216, difficulty=6.0),
         *box(16), 1e-3, 1e-16, 1 << 16)
    for d in (5, 8):
        p = W.family_params(1, d, seed=900 + d)
        _run(out, f"rule9_d{d}", gm.integrate, 1, p, *box(d), 1e-7, 1e-16, 1 << 20,
             opts={"rule": 2, "err_model": 1})
    _run(out, "gk_d3", gm.integrate, 4, W.family_params(4, 3, seed=43), *box(3), 1e-10, 1e-16,
         1 << 16, opts={"rule": 1})
    _run(out, "prune_d8", gm.integrate, 4, W.family_params(4, 8, seed=48), *box(8), 1e-7, 1e-16,
         1 << 15, opts={"prune": 1})
    _run(out, "grad_d4", gm.integrate_grad, 4, W.family_params(4, 4, seed=44), *box(4), 1e-7)
    _run(out, "grad9_d5", gm.integrate_grad, 1, W.family_params(1, 5, seed=15), *box(5), 1e-6,
         opts={"rule": 2})
    _run(out, "noalloc_d5", gm.integrate_noalloc, 6, W.family_params(6, 5, seed=65), *box(5),
         1e-5, 1e-16, 1 << 16)
    rng = np.random.default_rng(7)
    n = 128
    fams = [int(f) for f in rng.choice([1, 2, 4], n)]
    ds = [int(d) for d in rng.integers(3, 11, n)]
    ps = [W.family_params(f, d, seed=1000 + i) for i, (f, d) in enumerate(zip(fams, ds))]
    los = [np.zeros(d) for d in ds]
    his = [np.ones(d) for d in ds]
    _run(out, "batch", gm.integrate_batch, fams, ps, ds, los, his, [1e-4] * n, [1e-16] * n,
         1 << 22)
    c = rng.uniform(0.2, 0.8, (50, 6))
    h = np.full((50, 6), 0.05)
    lvl = np.full(50, 6, dtype=np.int32)
    _run(out, "eval_regions", gm.eval_regions, 5, W.family_params(5, 6, seed=56), *box(6), c, h,
         lvl)
    return out


def selftest() -> dict:
    """(check build only) the check path on an index one past its bound that
    no kernel accesses: the status and message the library reports."""
    rc = gm.lib().gm_set_option(b"check_selftest", 12345)
    return {"rc": int(rc), "text": gm.status_string(rc)}


if __name__ == "__main__":
    if "--lib" in sys.argv:
        gm.LIB_PATH = sys.argv[sys.argv.index("--lib") + 1]
    res = {"selftest": selftest()} if "--selftest" in sys.argv else {}
    res.update(run_cases())
    print(json.dumps(res))
