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


def _full_result():
    """A result dict of the shape the default benchmark run builds, at full
    size: 18 suite cases, every mode section, the CPU baseline."""
    cases = [{"name": f"{f}_d8_r0_tau{t}", "status": 1 if (f, t) == ("oscillatory", "1e-07") else 0,
              "seconds": 0.0123456789, "evals": 12345678901, "regions": 30787727,
              "iterations": 27, "I": 0.123456789012345, "E": 1.23456789e-9,
              "rel_err_vs_closed_form": 1.234567e-9}
             for f in ("oscillatory", "product_peak", "corner_peak", "gaussian", "c0",
                       "discontinuous") for t in ("0.001", "1e-05", "1e-07")]
    batch = {"integrals": 4096, "batch_s": 0.1123, "batch_integrals_per_s": 36473.1,
             "batch_evals": 123456789012, "batch_evals_per_s": 1.1e12, "single_s": 0.798,
             "single_integrals_per_s": 5132.8, "speedup": 7.1234,
             "status_counts_batch": {"0": 4096}, "status_counts_single": {"0": 4096},
             "max_rel_diff_batch_vs_single": 2.2e-16,
             "max_rel_err_vs_closed_form_every_16th": 5.6e-7, "difficulty_scale": 0.35,
             "tile_table": "autotuned",
             "degree9": {"batch_s": 0.0118, "batch_integrals_per_s": 347118.6,
                         "batch_evals": 1234567890, "speedup_vs_degree7_batch": 9.5,
                         "speedup_vs_degree7_singles": 67.0, "status_counts": {"0": 4096},
                         "max_rel_err_vs_closed_form_every_16th": 1.3e-8}}
    grad = {"d": 8, "rel_tol": 1e-8, "rule": "degree9", "max_regions": 1 << 27, "status": 0,
            "grad_s": 0.0531, "regions": 123456789, "integral_rel_err": 3.4e-10,
            "E_over_I": 1e-8, "grad_max_err_rel_to_max": 3e-9, "fd_s": 1.234, "speedup": 23.2,
            "fd_all_ok": True, "fd_max_err_rel_to_max": 2.5e-6}
    c3 = [{"name": n, "status": 0, "seconds": 3.57, "evals": 6608123456789,
           "regions": 100123456, "iterations": 40, "max_active": 35123456,
           "evals_per_s": 1.87e12, "regions_per_s": 2.8e7, "rule_evals_per_s": 2.1e12,
           "rule_frac": 0.4512345, "rel_err_vs_closed_form": 6.1e-6,
           "E_over_I": 9.9e-5}
          for n in ("corner_peak_d12", "product_peak_d12", "corner_peak_d16", "product_peak_d16")]
    d9 = {"totals": {k: {"seconds": 0.0135, "evals": 3712345678, "regions": 3412345,
                         "rule_kernel_s": 0.011, "rule_evals_per_s": 3.3e11,
                         "status_counts": {"0": 18}, "max_rel_err_over_rel_tol": 9085.3}
                     for k in ("degree7", "degree9", "degree9_null_rule")},
          "cases": [{"name": c["name"]} for c in cases], "config3": c3}
    return {
        "metric": "integrand evals/s (d=8 six-family Genz suite, rel_tol 1e-3/1e-5/1e-7)",
        "value": 1.1612345678e12, "unit": "evals/s", "n_gpus": 1, "steps": 20, "warmup": 5,
        "ms_per_step": 59.712345678, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded Genz-family parameters)",
        "config": {"workload": "genz6_d8_tau1e-3_1e-5_1e-7", "d": 8, "families": 6,
                   "rel_tols": [1e-3, 1e-5, 1e-7], "max_regions": 1 << 24,
                   "integrals_per_step": 18},
        "regions_per_s": 2.9123456e9,
        "roofline": {"bound": "alu", "kernel": "rule (FP64 vector)", "achieved": 36.8123456,
                     "peak": 78.6, "unit": "TFLOP/s", "frac": 0.468345, "traffic": 1.9179e8,
                     "traffic_unit": "HBM bytes per launch",
                     "algorithmic_bytes_per_launch": 6.4633e7, "flops_per_eval": 23.7123,
                     "rule_kernel_s": 0.8912345, "rule_launches": 4380,
                     "rule_avg_launch_ms": 0.2036123, "rule_evals_per_s": 1.55123e12},
        "cases": cases,
        "flags": ["oscillatory_d8_r0_tau1e-07: status 1, time to capacity"]
                 + [f"discontinuous_d8_r0_tau{t}: E/I 7.0e-08, 9.1e-04 off the closed form "
                    "(jump unseen by the estimate)" for t in ("0.001", "1e-05", "1e-07")],
        "split_compaction": {"algorithmic_bytes": 2.5e10, "kept_regions": 86312345,
                             "device_ms": 9.51, "achieved_GBps": 2612.3, "peak_GBps": 8000.0,
                             "frac": 0.3265},
        "batch": batch, "grad": grad, "grad_degree7_1e-6": dict(grad, rule="degree7"),
        "config3": c3, "gauss_kronrod": [{"name": "x"}] * 6, "prune": [{"name": "y"}] * 3,
        "degree9": d9,
        "cpu_baseline": {"value": 6.3123e7, "unit": "integrand evals/s", "cores": 1,
                         "kind": "oracle", "model": "AMD EPYC 9575F 64-Core Processor",
                         "nproc": 16, "omp": {"value": 8.1e8, "cores": 16},
                         "sample": "2 pass(es) over 12 full oracle runs of the d=8 workload at "
                                   "rel_tol 1e-3/1e-5 (oscillatory_d8_r0_tau0.001, "
                                   "oscillatory_d8_r0_tau1e-05, product_peak_d8_r0_tau0.001, "
                                   "product_peak_d8_r0_tau1e-05); 1234567890 evals in 19.6 s"},
    }


def test_headline_is_the_compact_last_line():
    """The driver keeps the last 8 KB of stdout: the headline carries the
    contract fields, the roofline and CPU-baseline objects and the mode
    summaries in well under 4 KB."""
    sys.path.insert(0, ROOT)
    import bench
    full = _full_result()
    h = bench.headline(full)
    line = json.dumps(h)
    assert len(line.encode()) < 4096, len(line)
    back = json.loads(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline", "batch", "grad", "config3", "split_compaction"):
        assert k in back, k
    assert back["config"]["workload"] == "genz6_d8_tau1e-3_1e-5_1e-7"
    r = back["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r, k
    assert abs(back["value"] - full["value"]) <= 1e-5 * full["value"]
    assert back["cpu_baseline"]["kind"] == "oracle" and back["cpu_baseline"]["cores"] == 1
