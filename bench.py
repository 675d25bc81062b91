#!/usr/bin/env python3
"""Benchmark of the adaptive Genz-Malik cubature hot path on one MI355X.

Metric: integrand evaluations per second (whole job) on the d = 8 workload:
the six seeded Genz families (oscillatory, product peak, corner peak,
Gaussian, C0, discontinuous) on [0,1]^8, each at rel_tol 1e-3, 1e-5 and
1e-7, FP64, up to 2^24 active regions.  One step = the 18 integrals
(every iteration runs rule, reduction, classify, scan, split/compaction).

Output: one JSON line per detail section ({"detail": name, "data": ...}:
per-integral cases, batch, grad, config3, gauss_kronrod, prune, degree9),
then the compact headline as the LAST line (well under 4 KB), holding
  roofline          the rule kernel (dominant) against the FP64 vector peak:
                    algorithmic FP64 FLOPs (evals x FLOPs per evaluation of
                    the family as implemented) / rule-kernel device time
                    measured with HIP events on the launch stream;
  split_compaction  classify + scan + scatter against the HBM peak;
  cpu_baseline      the CPU oracle on a bounded sample of the workload;
  batch, grad, ...  one-number summaries of the modes against
                    one-call-per-integral;
and the time to tolerance per rel_tol: the sum over its six integrals of
each call's median over the timed steps (default 5, after 1 warm-up step).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--detail-out F]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published FP64 vector peak (256 CUs x 128 FP64 FLOP/clk x 2.4 GHz).
FP64_VECTOR_PEAK_TFLOPS = 78.6
# MI355X published HBM3E bandwidth.
HBM_PEAK_GBPS = 8000.0

# FP64 FLOPs per integrand evaluation as the rule kernel implements it:
# counted from the compiled corner-sweep loop of the one-lane-per-region rule
# kernel at d = 8 (the loop that evaluates 256 of the 401 nodes of a region),
# FMA = 2, ADD/MUL/RCP = 1, per corner: the amortized chain combinations of
# per-coordinate terms, the outer function (exp / cos / reciprocal / powers)
# and the compensated accumulation.  Cross-checked against the
# SQ_INSTS_VALU_*_F64 counters (profiles/).
FLOPS_PER_EVAL = {1: 42.75, 2: 7.0, 3: 16.8125, 4: 32.5, 5: 32.75, 6: 32.5, 7: 8.5}

# HBM traffic of the rule kernel, per launch, measured with rocprofv3 --pmc
# (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads for a
# plain device copy of known size) on this benchmark's own launches.  The
# summary file records the SHA-256 of the sources the rule kernel is compiled
# from; the figure is reported only while those sources are unchanged.
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "rule_kernel_d8_suite_counters.md")
RULE_SOURCES = [os.path.join(ROOT, "paper_2511_01573_amd", "csrc", f)
                for f in ("gm_rule.hip", "gm_corner.hpp", "gm_family.hpp", "gm_common.hpp",
                          "gm_math.hpp", "gm_api.hip")]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-modes", action="store_true", help="skip batch/grad comparisons")
    ap.add_argument("--taus", default="1e-3,1e-5,1e-7")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="budget of the CPU-oracle sample")
    ap.add_argument("--grad-tau", type=float, default=1e-8,
                    help="tolerance of the gradient workload (stated at 1e-8)")
    ap.add_argument("--grad-rule", type=int, default=2, choices=(0, 2),
                    help="rule of the gradient workload at --grad-tau: 2 degree 9 (default; the "
                         "degree-7 rule needs far more than one GPU's store at 1e-8), 0 degree 7")
    ap.add_argument("--detail-out", default=None,
                    help="also write the full result (every case and mode) to this JSON file")
    ap.add_argument("--grad-log2cap", type=int, default=27)
    ap.add_argument("--config3-log2cap", type=int, default=27)
    ap.add_argument("--rule", type=int, default=0, choices=(0, 2),
                    help="rule of the timed suite: 0 degree 7 (the benchmark), 2 degree 9 "
                         "(profiling runs; its line carries no FLOP roofline)")
    ap.add_argument("--only", choices=("batch", "grad"), default=None,
                    help="run one mode by itself (a warm-up and one timed call), for profiling")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy (counter calibration)")
    return ap.parse_args()


def rule_sources_sha256() -> str:
    h = hashlib.sha256()
    for f in RULE_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """Rule-kernel HBM bytes per launch from the committed counter summary, or
    None when the kernel sources changed since the counters were taken."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    m_sha = re.search(r"rule_sources_sha256:\s*([0-9a-f]{64})", text)
    m_val = re.search(r"hbm_bytes_per_rule_launch:\s*([0-9.eE+]+)", text)
    if not m_sha or not m_val or m_sha.group(1) != rule_sources_sha256():
        return None
    return float(m_val.group(1))


def copy_calibration():
    """A plain 1 GiB device copy, the reference that scales the HBM counters."""
    import torch
    n = 1 << 27
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8}))


def run_cases(gm, cases):
    out = []
    for c in cases:
        t0 = time.perf_counter()
        I, E, st = gm.integrate(c["family"], c["params"], c["lo"], c["hi"], c["rel_tol"],
                                c["abs_tol"], c["max_regions"])
        t1 = time.perf_counter()
        s = gm.last_stats()
        out.append({"name": c["name"], "family": c["family"], "I": I, "E": E, "status": st,
                    "seconds": t1 - t0, "evals": s["evals"], "regions": s["regions_evaluated"],
                    "iterations": s["iterations"], "rule_ms": s["rule_ms"],
                    "rule_launches": s["rule_launches"]})
    return out


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_passes(O, cases, budget_s: float):
    """Whole passes over the cases (every case equally represented), repeated
    while another pass fits the budget; the first pass always runs."""
    evals, secs, passes, pass_s = 0, 0.0, 0, 0.0
    while passes == 0 or secs + pass_s <= budget_s:
        t_pass = 0.0
        for c in cases:
            t0 = time.perf_counter()
            r = O.integrate(c["family"], c["params"], c["lo"], c["hi"], c["rel_tol"],
                            c["abs_tol"], c["max_regions"])
            t_pass += time.perf_counter() - t0
            evals += r["evals"]
        secs += t_pass
        pass_s = t_pass
        passes += 1
    return evals, secs, passes


def cpu_baseline(budget_s: float):
    """The CPU oracle on a bounded sample: the 12 d = 8 cases at rel_tol 1e-3
    and 1e-5 (full runs), whole passes repeated while another pass fits the
    budget.  The serial build (one core) is the baseline; the OpenMP build
    (per-region evaluation on every core the process may use, reductions
    serial, the same bits) runs the same sample in half the budget."""
    from oracle import oracle as O
    from paper_2511_01573_amd import workloads as W
    cases = W.config2(taus=(1e-3, 1e-5))
    O.use_openmp(False)
    evals, secs, passes = _oracle_passes(O, cases, budget_s)
    try:
        threads = O.use_openmp(True)
        oev, osecs, opasses = _oracle_passes(O, cases, budget_s / 2)
    finally:
        O.use_openmp(False)
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        allowed = os.cpu_count()
    return {"value": evals / secs, "unit": "integrand evals/s", "cores": 1, "kind": "oracle",
            "model": _cpu_model(), "nproc": allowed,
            "omp": {"value": oev / osecs, "cores": threads, "passes": opasses},
            "sample": f"{passes} pass(es) over the {len(cases)} full oracle runs of the d=8 "
                      f"workload at rel_tol 1e-3/1e-5 (6 families x 2); {evals} evals in "
                      f"{secs:.1f} s, serial C -O3, 1 thread"}


def bench_batch(gm, W, closed_forms):
    """4096 integrals (d 3..10, Gaussian/oscillatory/product peak, rel_tol
    10^U(-7,-3)) in one gm_integrate_batch call (shared store of 2^28 regions,
    graph replay of 8 iterations), against one gm_integrate call per integral
    over the same 4096 items (same tolerances; every item converges both ways,
    so both give each item's own adaptive result)."""
    import torch
    from paper_2511_01573_amd import autotune
    b = W.config4()
    args = (b["families"], b["params"], b["ds"], b["los"], b["his"], b["rel_tols"], b["abs_tols"])
    table = autotune.load()
    gm.set_option("graph_iters", 8)
    cap = 1 << 28  # shared by all 4096 items (~88 GiB at d <= 10)
    try:
        gm.integrate_batch(*args, cap)  # warm-up (module load, workspace)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, est, err, st = gm.integrate_batch(*args, cap)
        tb = time.perf_counter() - t0
        bstats = gm.last_stats()
    finally:
        gm.set_option("graph_iters", 0)
    n = len(b["families"])
    gm.integrate(b["families"][0], b["params"][0], b["los"][0], b["his"][0], b["rel_tols"][0],
                 b["abs_tols"][0], 1 << 26)  # warm-up of the single path
    t0 = time.perf_counter()
    single, sst = np.zeros(n), np.zeros(n, dtype=np.int64)
    for i in range(n):
        single[i], _, sst[i] = gm.integrate(b["families"][i], b["params"][i], b["los"][i],
                                            b["his"][i], b["rel_tols"][i], b["abs_tols"][i], 1 << 26)
    ts = time.perf_counter() - t0
    agree = float(np.max(np.abs(single - est) / np.maximum(np.abs(est), 1e-300)))

    def every16(values):
        out = []
        for i in range(0, n, 16):
            d = b["ds"][i]
            ex = float(closed_forms.exact(b["families"][i], b["params"][i][:d],
                                          b["params"][i][d:]))
            out.append(abs(values[i] - ex) / abs(ex))
        return max(out)

    relerr = [every16(est)]
    # the same batch with the degree-9 rule
    gm.set_option("graph_iters", 8)
    gm.set_option("rule", 2)
    try:
        gm.integrate_batch(*args, cap)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc9, est9, err9, st9 = gm.integrate_batch(*args, cap)
        t9 = time.perf_counter() - t0
        s9 = gm.last_stats()
    finally:
        gm.set_option("graph_iters", 0)
        gm.set_option("rule", 0)
    deg9 = {"batch_s": t9, "batch_integrals_per_s": n / t9, "batch_evals": s9["evals"],
            "speedup_vs_degree7_batch": tb / t9, "speedup_vs_degree7_singles": ts / t9,
            "status_counts": {str(k): int((st9 == k).sum()) for k in set(st9.tolist())},
            "max_rel_err_vs_closed_form_every_16th": every16(est9)}
    return {"integrals": n, "batch_s": tb, "batch_integrals_per_s": n / tb,
            "batch_evals": bstats["evals"], "batch_evals_per_s": bstats["evals"] / tb,
            "single_s": ts, "single_integrals_per_s": n / ts, "speedup": ts / tb,
            "status_counts_batch": {str(k): int((st == k).sum()) for k in set(st.tolist())},
            "status_counts_single": {str(k): int((sst == k).sum()) for k in set(sst.tolist())},
            "max_rel_diff_batch_vs_single": agree,
            "max_rel_err_vs_closed_form_every_16th": max(relerr),
            "difficulty_scale": W.BATCH_SCALE,
            "tile_table": "autotuned" if table else "default", "degree9": deg9}


def bench_config3(gm, W, closed_forms, log2cap: int):
    """d = 12 and 16, corner peak and product peak, rel_tol 1e-4, region store
    of 2^log2cap rows (the high-dimensional, many-lanes-per-region regime),
    each after a warm-up run of the same integral."""
    out = []
    for c in W.config3(max_regions=1 << log2cap):
        gm.integrate(c["family"], c["params"], c["lo"], c["hi"], c["rel_tol"], c["abs_tol"],
                     c["max_regions"])
        d = len(c["lo"])
        gm.set_option("timing", 1)
        t0 = time.perf_counter()
        I, E, st = gm.integrate(c["family"], c["params"], c["lo"], c["hi"], c["rel_tol"],
                                c["abs_tol"], c["max_regions"])
        dt = time.perf_counter() - t0
        s = gm.last_stats()
        gm.set_option("timing", 0)
        ex = float(closed_forms.exact(c["family"], c["params"][:d], c["params"][d:]))
        rule_s = max(s["rule_ms"] * 1e-3, 1e-12)
        out.append({"name": c["name"], "status": st, "seconds": dt, "evals": s["evals"],
                    "regions": s["regions_evaluated"], "iterations": s["iterations"],
                    "max_active": s["max_active"], "evals_per_s": s["evals"] / dt,
                    "regions_per_s": s["regions_evaluated"] / dt,
                    "rule_evals_per_s": s["evals"] / rule_s,
                    # the corner sweep (2^d of the N(d) nodes) costs what it costs at d = 8
                    "rule_frac": s["evals"] * FLOPS_PER_EVAL[c["family"]] / rule_s / 1e12
                                 / FP64_VECTOR_PEAK_TFLOPS,
                    "rel_err_vs_closed_form": abs(I - ex) / abs(ex), "E_over_I": E / abs(I)})
    return out


def bench_gk(gm, W, closed_forms):
    """The tensor-product Gauss-Kronrod rule (7-point Gauss / 15-point
    Kronrod per axis) against the Genz-Malik rule on the same integrals, both
    from an initial partition of 2^3 cells: time to tolerance, evaluations,
    rule-kernel throughput (a second, timed run) and accuracy against the
    closed form."""
    cases = []
    c1 = W.config1()
    cases.append(("gaussian_d3_a5", c1["family"], c1["params"], 3, 1e-6))
    cases.append(("gaussian_d3_a5", c1["family"], c1["params"], 3, 1e-11))
    for fam, d in ((1, 4), (2, 4), (4, 5), (5, 3)):
        cases.append((f"{W.NAMES[fam]}_d{d}", fam, W.family_params(fam, d, 500 + fam), d, 1e-8))
    out = []
    for name, fam, p, d, tau in cases:
        lo, hi = W.unit_box(d)
        ex = float(closed_forms.exact(fam, p[:d], p[d:]))
        row = {"name": name, "rel_tol": tau}
        for rule in (0, 1):
            gm.set_option("rule", rule)
            gm.set_option("init_log2_regions", 3)
            try:
                gm.integrate(fam, p, lo, hi, tau, 1e-16, 1 << 24)  # warm-up
                t0 = time.perf_counter()
                I, E, st = gm.integrate(fam, p, lo, hi, tau, 1e-16, 1 << 24)
                dt = time.perf_counter() - t0
                s = gm.last_stats()
                gm.set_option("timing", 1)
                try:
                    gm.integrate(fam, p, lo, hi, tau, 1e-16, 1 << 24)
                    rule_ms = gm.last_stats()["rule_ms"]
                finally:
                    gm.set_option("timing", 0)
            finally:
                gm.set_option("rule", 0)
                gm.set_option("init_log2_regions", 12)
            key = "gk" if rule else "gm"
            row[key] = {"status": st, "seconds": dt, "evals": s["evals"],
                        "regions": s["regions_evaluated"], "evals_per_s": s["evals"] / dt,
                        "rule_evals_per_s": s["evals"] / max(rule_ms * 1e-3, 1e-12),
                        "rel_err_vs_closed_form": abs(I - ex) / abs(ex)}
        out.append(row)
    return out


def bench_degree9(gm, W, closed_forms, log2cap: int):
    """The degree-9 rule (both error models) against the degree-7 rule on the
    d = 8 suite (the 18 integrals of one benchmark step): time to tolerance,
    integrand evaluations, rule-kernel time and accuracy against the closed
    form, per case and in total; then the d = 12 / 16 cases with degree 9."""
    cases = W.config2()
    variants = (("degree7", 0, 0), ("degree9", 2, 0), ("degree9_null_rule", 2, 1))
    rows = {c["name"]: {"name": c["name"]} for c in cases}
    totals = {}
    gm.set_option("timing", 1)
    try:
        for key, rule, model in variants:
            gm.set_option("rule", rule)
            gm.set_option("err_model", model)
            run_cases(gm, cases)  # warm-up
            res = run_cases(gm, cases)
            worst = 0.0
            for c, r in zip(cases, res):
                d = len(c["lo"])
                ex = float(closed_forms.exact(c["family"], c["params"][:d], c["params"][d:]))
                rel = abs(r["I"] - ex) / abs(ex)
                worst = max(worst, rel / c["rel_tol"])
                rows[c["name"]][key] = {"status": r["status"], "seconds": r["seconds"],
                                        "evals": r["evals"], "regions": r["regions"],
                                        "rel_err_vs_closed_form": rel}
            secs = sum(r["seconds"] for r in res)
            ev = sum(r["evals"] for r in res)
            rule_s = sum(r["rule_ms"] for r in res) / 1e3
            totals[key] = {"seconds": secs, "evals": ev, "regions": sum(r["regions"] for r in res),
                           "rule_kernel_s": rule_s, "rule_evals_per_s": ev / rule_s,
                           "status_counts": {str(k): sum(1 for r in res if r["status"] == k)
                                             for k in sorted({r["status"] for r in res})},
                           "max_rel_err_over_rel_tol": worst}
        # the d = 12 / 16 cases with the degree-9 rule (the degree-7 runs are
        # the "config3" section)
        gm.set_option("rule", 2)
        gm.set_option("err_model", 0)
        high = []
        for c in W.config3(max_regions=1 << log2cap):
            d = len(c["lo"])
            t0 = time.perf_counter()
            I, E, st = gm.integrate(c["family"], c["params"], c["lo"], c["hi"], c["rel_tol"],
                                    c["abs_tol"], c["max_regions"])
            dt = time.perf_counter() - t0
            s = gm.last_stats()
            ex = float(closed_forms.exact(c["family"], c["params"][:d], c["params"][d:]))
            high.append({"name": c["name"], "status": st, "seconds": dt, "evals": s["evals"],
                         "regions": s["regions_evaluated"],
                         "rule_evals_per_s": s["evals"] / max(s["rule_ms"] * 1e-3, 1e-12),
                         "rel_err_vs_closed_form": abs(I - ex) / abs(ex)})
    finally:
        gm.set_option("timing", 0)
        gm.set_option("rule", 0)
        gm.set_option("err_model", 0)
    return {"totals": totals, "cases": list(rows.values()), "config3": high}


def bench_prune(gm, W, closed_forms):
    """Memory-pressure pruning on the suite cases that outgrow their store:
    the oscillatory integral at rel_tol 1e-7 with 2^24 regions, and two d = 8
    cases on a store of 2^18 regions, each without and with pruning."""
    out = []
    cases = [c for c in W.config2(taus=(1e-7,)) if c["family"] == 1]
    cases += [dict(c, max_regions=1 << 18) for c in W.config2(taus=(1e-7,)) if c["family"] in (4, 5)]
    for c in cases:
        d = len(c["lo"])
        ex = float(closed_forms.exact(c["family"], c["params"][:d], c["params"][d:]))
        row = {"name": c["name"], "max_regions": c["max_regions"]}
        for prune in (0, 1):
            gm.set_option("prune", prune)
            try:
                t0 = time.perf_counter()
                I, E, st = gm.integrate(c["family"], c["params"], c["lo"], c["hi"], c["rel_tol"],
                                        c["abs_tol"], c["max_regions"])
                dt = time.perf_counter() - t0
                s = gm.last_stats()
            finally:
                gm.set_option("prune", 0)
            row["pruned" if prune else "plain"] = {
                "status": st, "seconds": dt, "iterations": s["iterations"], "evals": s["evals"],
                "E_over_I": E / abs(I), "rel_err_vs_closed_form": abs(I - ex) / abs(ex)}
        out.append(row)
    return out


def bench_grad(gm, W, closed_forms, tau: float, cap: int, rule: int, fd: bool = True):
    """The gradient workload (d = 8 Gaussian, 16 parameters): one
    gm_integrate_grad call against 1 + 32 gm_integrate calls (the estimate plus
    central differences h = 1e-6 of full adaptive runs), both with the same
    rule and tolerance, compared with the erf closed form."""
    import numpy as np
    c = W.config5()
    p = c["params"]
    d = 8
    a, u = p[:d], p[d:]
    want = np.array([float(x) for x in closed_forms.gaussian_grad(a, u)])
    exact = float(closed_forms.gaussian(a, u))
    scale = np.abs(want).max()
    gm.set_option("rule", rule)
    try:
        gm.integrate_grad(4, p, c["lo"], c["hi"], tau, 1e-16, cap)  # warm-up
        t0 = time.perf_counter()
        I, E, g, st = gm.integrate_grad(4, p, c["lo"], c["hi"], tau, 1e-16, cap)
        tg = time.perf_counter() - t0
        s = gm.last_stats()
        out = {"d": d, "rel_tol": tau, "rule": "degree9" if rule == 2 else "degree7",
               "max_regions": cap, "status": st, "grad_s": tg, "regions": s["regions_evaluated"],
               "integral_rel_err": abs(I - exact) / exact, "E_over_I": E / abs(I),
               "grad_max_err_rel_to_max": float(np.abs(g - want).max() / scale)}
        if fd:
            t0 = time.perf_counter()
            gm.integrate(4, p, c["lo"], c["hi"], tau, 1e-16, cap)
            fdg = np.zeros(2 * d)
            fst = []
            for k in range(2 * d):
                pp, pm = p.copy(), p.copy()
                pp[k] += 1e-6
                pm[k] -= 1e-6
                ip, _, sp = gm.integrate(4, pp, c["lo"], c["hi"], tau, 1e-16, cap)
                im, _, sm = gm.integrate(4, pm, c["lo"], c["hi"], tau, 1e-16, cap)
                fdg[k] = (ip - im) / 2e-6
                fst += [sp, sm]
            tf = time.perf_counter() - t0
            out.update({"fd_s": tf, "speedup": tf / tg, "fd_all_ok": all(x == 0 for x in fst),
                        "fd_max_err_rel_to_max": float(np.abs(fdg - want).max() / scale)})
    finally:
        gm.set_option("rule", 0)
    return out


def run_only(gm, W, mode: str, grad_tau: float, grad_cap: int, grad_rule: int):
    """One mode by itself, for a kernel trace that holds nothing else: the
    4096-integral batch (one warm-up and one timed gm_integrate_batch call,
    as in the batch section) or the d = 8 Gaussian gradient (one warm-up and
    one timed gm_integrate_grad call, as in the gradient section)."""
    import torch
    if mode == "batch":
        b = W.config4()
        args = (b["families"], b["params"], b["ds"], b["los"], b["his"], b["rel_tols"], b["abs_tols"])
        gm.set_option("graph_iters", 8)
        try:
            gm.integrate_batch(*args, 1 << 28)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, est, err, st = gm.integrate_batch(*args, 1 << 28)
            dt = time.perf_counter() - t0
        finally:
            gm.set_option("graph_iters", 0)
        return {"mode": "batch", "integrals": len(b["families"]), "seconds": dt,
                "evals": gm.last_stats()["evals"],
                "status_counts": {str(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))}}
    c = W.config5()
    gm.set_option("rule", grad_rule)
    try:
        gm.integrate_grad(4, c["params"], c["lo"], c["hi"], grad_tau, 1e-16, grad_cap)
        t0 = time.perf_counter()
        I, E, g, st = gm.integrate_grad(4, c["params"], c["lo"], c["hi"], grad_tau, 1e-16, grad_cap)
        dt = time.perf_counter() - t0
        s = gm.last_stats()
    finally:
        gm.set_option("rule", 0)
    return {"mode": "grad", "d": 8, "rel_tol": grad_tau, "rule": grad_rule, "seconds": dt,
            "status": st, "evals": s["evals"], "regions": s["regions_evaluated"]}


def split_compaction(gm, cases):
    """HBM rate of classify + split/compaction (scan and scatter) over one pass
    of the suite, timed per phase with HIP events on the launch stream
    (option timing = 2; a pass of its own, outside the timed steps).
    Algorithmic bytes: classify reads err, the level (one byte per region: two
    children share their parent's) and the axis byte and writes the flag
    (11 B per region) and reads Q of every retired region (8 B); the scatter
    reads the flag and the axis byte (2 B per region) and, per kept region,
    reads its parent record and writes its own (2 x (16d + 3) B)."""
    gm.set_option("timing", 2)
    try:
        res = []
        for c in cases:
            gm.integrate(c["family"], c["params"], c["lo"], c["hi"], c["rel_tol"], c["abs_tol"],
                         c["max_regions"])
            res.append((c, gm.last_stats()))
    finally:
        gm.set_option("timing", 0)
    by = 0.0
    ms = 0.0
    kept_total = 0
    for c, s in res:
        d = len(c["lo"])
        n0 = 1 << (d * (12 // d))
        kept = (s["regions_evaluated"] - n0) // 2  # every split's two children were evaluated
        kept_total += kept
        by += s["regions_evaluated"] * 13 + s["finished"] * 8 + kept * 2 * (16 * d + 3)
        ms += s["classify_ms"] + s["split_ms"]
    return {"algorithmic_bytes": by, "kept_regions": kept_total, "device_ms": ms,
            "achieved_GBps": by / (ms * 1e-3) / 1e9, "peak_GBps": HBM_PEAK_GBPS,
            "frac": by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS}


def _sig(x, n=4):
    """Round a float to n significant digits for the compact line."""
    if x is None or isinstance(x, (bool, int, str)):
        return x
    x = float(x)
    if x == 0.0 or x != x or x in (float("inf"), float("-inf")):
        return x
    return float(f"{x:.{n - 1}e}")


def headline(full: dict) -> dict:
    """The compact last line (well under 4 KB): the contract fields, the
    roofline and CPU-baseline objects, and one-number summaries of every
    other section (their full detail is printed on the lines before)."""
    S = _sig
    h = {k: full[k] for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                              "higher_is_better", "scaling", "vs_baseline", "dtype", "data",
                              "config")}
    h["value"] = S(h["value"], 6)
    h["ms_per_step"] = S(h["ms_per_step"], 6)
    h["regions_per_s"] = S(full["regions_per_s"])
    cases = full.get("cases", [])
    ttt = {}
    for c in cases:
        key = c["name"].rsplit("_tau", 1)[-1]
        ttt[key] = ttt.get(key, 0.0) + c["seconds"] * 1e3
    h["time_to_tolerance_ms_by_rel_tol"] = {k: S(v) for k, v in ttt.items()}
    h["status_counts"] = {}
    for c in cases:
        h["status_counts"][str(c["status"])] = h["status_counts"].get(str(c["status"]), 0) + 1
    if full.get("flags"):
        h["flags"] = full["flags"]
    r = full["roofline"]
    h["roofline"] = {k: v for k, v in r.items()
                     if k in ("bound", "kernel", "achieved", "peak", "unit", "frac", "traffic",
                              "algorithmic_bytes_per_launch", "rule_avg_launch_ms",
                              "rule_launches", "rule_evals_per_s", "flops_per_eval")}
    if "split_compaction" in full:
        sc = full["split_compaction"]
        h["split_compaction"] = {"bound": "hbm", "achieved": S(sc["achieved_GBps"]),
                                 "peak": sc["peak_GBps"], "unit": "GB/s", "frac": S(sc["frac"])}
    if "cpu_baseline" in full:
        cb = full["cpu_baseline"]
        h["cpu_baseline"] = {k: (S(v) if isinstance(v, float) else v) for k, v in cb.items()}
    if "batch" in full:
        b = full["batch"]
        h["batch"] = {"integrals": b["integrals"], "speedup_vs_single_calls": S(b["speedup"]),
                      "integrals_per_s": S(b["batch_integrals_per_s"]),
                      "single_integrals_per_s": S(b["single_integrals_per_s"]),
                      "all_ok": b["status_counts_batch"] == {"0": b["integrals"]},
                      "max_rel_err": S(b["max_rel_err_vs_closed_form_every_16th"], 2)}
        if "degree9" in b:
            h["batch"]["degree9_integrals_per_s"] = S(b["degree9"]["batch_integrals_per_s"])
    if "grad" in full:
        g = full["grad"]
        h["grad"] = {k: (S(v, 3) if isinstance(v, float) else v) for k, v in g.items()
                     if k in ("rel_tol", "rule", "status", "speedup", "grad_s",
                              "grad_max_err_rel_to_max", "fd_max_err_rel_to_max")}
    if "config3" in full:
        h["config3"] = {c["name"]: {"status": c["status"], "s": S(c["seconds"], 3),
                                    "regions": c["regions"], "max_active": c["max_active"],
                                    "evals_per_s": S(c["evals_per_s"], 3),
                                    "regions_per_s": S(c["regions_per_s"], 3),
                                    "rule_frac": S(c["rule_frac"], 3),
                                    "rel_err": S(c["rel_err_vs_closed_form"], 2)}
                        for c in full["config3"]}
    if "degree9" in full:
        t = full["degree9"]["totals"]
        h["degree9_suite"] = {k: {"s": S(v["seconds"], 3), "evals": v["evals"]}
                              for k, v in t.items()}
    # stay far inside the driver's stdout tail: drop the least important
    # summaries first if a run ever produced an unusually long line
    for k in ("degree9_suite", "config3", "flags"):
        if len(json.dumps(h)) <= 3800:
            break
        h.pop(k, None)
    return h


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is designed, not built)"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch
    from paper_2511_01573_amd import gm, workloads as W

    if args.only:
        print(json.dumps(run_only(gm, W, args.only, args.grad_tau, 1 << args.grad_log2cap,
                                  args.grad_rule)))
        return
    taus = tuple(float(x) for x in args.taus.split(","))
    cases = W.config2(taus=taus)
    gm.set_option("timing", 1)
    gm.set_option("rule", args.rule)
    for _ in range(args.warmup):
        run_cases(gm, cases)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = []
    for _ in range(args.steps):
        steps.append(run_cases(gm, cases))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gm.set_option("timing", 0)
    gm.set_option("rule", 0)

    evals = sum(c["evals"] for st in steps for c in st)
    regions = sum(c["regions"] for st in steps for c in st)
    value = evals / wall
    # roofline of the rule kernel (FP64 vector ALU bound)
    rule_s = sum(c["rule_ms"] for st in steps for c in st) / 1e3
    flops = sum(c["evals"] * FLOPS_PER_EVAL[c["family"]] for st in steps for c in st)
    launches = sum(c["rule_launches"] for st in steps for c in st)
    achieved = flops / rule_s / 1e12 if args.rule == 0 else None
    # algorithmic HBM bytes per rule launch: per region half of the parent
    # record two children share (8d + 1 B) read, Q, err and the axis byte (17 B)
    # written
    d = 8
    alg_bytes = regions / launches * (8 * d + 1 + 17)
    last = steps[-1]
    # time to tolerance of each integral: the median of its timed calls (the
    # warm-up calls load the code objects and size the workspace)
    for i, r in enumerate(last):
        r["seconds"] = float(np.median([st[i]["seconds"] for st in steps]))
        r["timed_calls"] = len(steps)
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import closed_forms
    flags = []
    for c, r in zip(cases, last):
        ex = float(closed_forms.exact(c["family"], c["params"][:d], c["params"][d:]))
        rel = abs(r["I"] - ex) / abs(ex)
        r["rel_err_vs_closed_form"] = rel
        if r["status"] != 0:
            flags.append(f"{r['name']}: status {r['status']}, time to capacity")
        elif rel > 10 * c["rel_tol"]:
            flags.append(f"{r['name']}: E/I {r['E'] / abs(r['I']):.1e}, {rel:.1e} off the "
                         "closed form (jump unseen by the estimate)")
    out = {
        "metric": "integrand evals/s (d=8 six-family Genz suite, rel_tol 1e-3/1e-5/1e-7)"
                  + (" with the degree-9 rule" if args.rule else ""),
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Genz-family parameters)",
        "config": {"workload": "genz6_d8_tau1e-3_1e-5_1e-7", "d": 8, "families": 6,
                   "rel_tols": list(taus), "max_regions": 1 << 24, "integrals_per_step": len(cases)},
        "regions_per_s": regions / wall,
        "roofline": {"bound": "alu", "kernel": "rule (FP64 vector)", "achieved": achieved,
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS if achieved else None,
                     "traffic": measured_traffic() if args.rule == 0 else None,
                     "traffic_unit": "HBM bytes per launch",
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "flops_per_eval": flops / evals,
                     "rule_kernel_s": rule_s, "rule_launches": launches,
                     "rule_avg_launch_ms": rule_s / launches * 1e3,
                     "rule_evals_per_s": evals / rule_s},
        "cases": [{k: c[k] for k in ("name", "status", "seconds", "timed_calls", "evals", "regions",
                                     "iterations", "I", "E", "rel_err_vs_closed_form")}
                  for c in last],
        "flags": flags,
    }
    if args.rule == 0:
        out["split_compaction"] = split_compaction(gm, cases)
    if not args.no_modes:
        out["batch"] = bench_batch(gm, W, closed_forms)
        out["grad"] = bench_grad(gm, W, closed_forms, args.grad_tau, 1 << args.grad_log2cap,
                                 args.grad_rule)
        out["grad_degree7_1e-6"] = bench_grad(gm, W, closed_forms, 1e-6, 1 << args.grad_log2cap,
                                              0, fd=False)
        out["config3"] = bench_config3(gm, W, closed_forms, args.config3_log2cap)
        out["gauss_kronrod"] = bench_gk(gm, W, closed_forms)
        out["prune"] = bench_prune(gm, W, closed_forms)
        out["degree9"] = bench_degree9(gm, W, closed_forms, args.config3_log2cap)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    # detail first (one line per section), the compact headline last
    for k, v in out.items():
        if isinstance(v, (list, dict)) and k not in ("config", "roofline", "cpu_baseline"):
            print(json.dumps({"detail": k, "data": v}))
    if args.detail_out:
        with open(args.detail_out, "w") as fh:
            json.dump(out, fh, indent=1)
    print(json.dumps(headline(out)), flush=True)


if __name__ == "__main__":
    main()
