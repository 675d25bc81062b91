"""Run-level parity of the HIP adaptive loop (Sec. 3 workflow, Sec. 4
stopping rule) with the CPU oracle: same status, iteration count, region
counts, final active set (bitwise geometry, stable order), and final estimate
within 1e-12 relative."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from paper_2511_01573_amd import gm, workloads as W
from parity import I_TOL, assert_regions_match

pytestmark = pytest.mark.gpu


def run_both(fam, p, lo, hi, tau, max_regions=1 << 22, init_log2=12, max_iters=10000,
             abs_tol=1e-16, compare_active=True):
    d = len(lo)
    gm.set_option("init_log2_regions", init_log2)
    gm.set_option("max_iters", max_iters)
    try:
        print(f"case fam={fam} d={d} tau={tau} L0={init_log2}", flush=True)
        I, E, st = gm.integrate(fam, p, lo, hi, tau, abs_tol, max_regions)
        stats = gm.last_stats()
        act = gm.last_active(d) if compare_active else None
    finally:
        gm.set_option("init_log2_regions", 12)
        gm.set_option("max_iters", 10000)
    run = O.Run(fam, p, lo, hi, tau, abs_tol, max_regions, init_log2, max_iters)
    run.run()
    ref = run.result()
    assert st == ref["status"], (st, ref)
    assert stats["iterations"] == ref["iterations"]
    assert stats["regions_evaluated"] == ref["regions"]
    assert stats["final_active"] == ref["active"]
    if st == O.NONFINITE:
        assert np.isnan(I) and np.isnan(E)
        return I, E, st, ref
    assert abs(I - ref["I"]) <= I_TOL * abs(ref["I"]) + 1e-300, (I, ref["I"])
    # each region's estimate agrees to 1e-13 of the magnitude it cancels
    assert abs(E - ref["E"]) <= 1e-13 * ref["escale"] + 1e-15 * abs(ref["E"]), (E, ref["E"])
    if compare_active:
        ra = run.active()
        assert np.array_equal(act["lvl"], ra["lvl"])
        assert np.array_equal(act["c"], ra["c"])
        assert np.array_equal(act["h"], ra["h"])
        full = O.rule_many(fam, p, ra["c"], ra["h"], ra["lvl"], run.vol_omega)
        assert_regions_match(act["Q"], act["err"], act["axis"], full, "final active set")
    return I, E, st, ref


def test_config1_gaussian_d3():
    c = W.config1()
    I, E, st, _ = run_both(c["family"], c["params"], c["lo"], c["hi"], c["rel_tol"],
                           max_regions=c["max_regions"])
    assert st == gm.OK
    assert abs(I - 0.044492261088252660431) <= 1e-6 * 0.0445


@pytest.mark.parametrize("tau", [1e-6, 1e-9])
def test_gaussian_d3_many_iterations(tau):
    c = W.config1()
    run_both(c["family"], c["params"], c["lo"], c["hi"], tau, init_log2=3)


@pytest.mark.parametrize("fam", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("d", [2, 5])
def test_families_small_d(fam, d):
    p = W.family_params(fam, d, seed=31 * fam + d)
    tau = {2: 1e-8, 5: 1e-5}[d]
    run_both(fam, p, *W.unit_box(d), tau, init_log2=4)


@pytest.mark.parametrize("fam", [1, 2, 3, 4, 5, 6])
def test_config2_d8_tau_1e3(fam):
    c = [x for x in W.config2(taus=(1e-3,)) if x["family"] == fam][0]
    run_both(c["family"], c["params"], c["lo"], c["hi"], c["rel_tol"],
             max_regions=c["max_regions"])


@pytest.mark.parametrize("lanes", [1, 4, 16])
@pytest.mark.parametrize("fam", [2, 4, 5])
def test_d8_every_mapping(fam, lanes):
    # the same run through each rule-kernel mapping gives the oracle's tree
    p = W.family_params(fam, 8, seed=77 + fam)
    gm.set_option("lanes_per_region", lanes)
    try:
        run_both(fam, p, *W.unit_box(8), 1e-4, max_regions=1 << 20)
    finally:
        gm.set_option("lanes_per_region", 0)


def test_d12_and_d16_small():
    p = W.family_params(3, 12, seed=3012, difficulty=1.0)
    run_both(3, p, *W.unit_box(12), 1e-3, max_regions=1 << 20)
    p = W.family_params(4, 16, seed=4016, difficulty=6.0)
    run_both(4, p, *W.unit_box(16), 1e-3, max_regions=1 << 16)


def test_status_codes_match_oracle():
    p25 = np.array([25.0] * 3 + [0.5] * 3)
    _, _, st, _ = run_both(4, p25, *W.unit_box(3), 1e-12, max_regions=5000)
    assert st == gm.MAX_REGIONS
    _, _, st, _ = run_both(4, p25, *W.unit_box(3), 1e-12, max_iters=1)
    assert st == gm.MAX_ITERS
    _, _, st, _ = run_both(3, np.array([-1.0, -1.0, 0.0, 0.0]), *W.unit_box(2), 1e-6,
                           compare_active=False)
    assert st == gm.NONFINITE
    _, _, st, _ = run_both(4, np.array([1e-3] * 3 + [0.5] * 3), *W.unit_box(3), 0.0,
                           abs_tol=1e-300)
    assert st == gm.PRECISION_LIMIT


def test_determinism():
    p = W.family_params(4, 6, seed=5)
    a = gm.integrate(4, p, *W.unit_box(6), 1e-7)
    b = gm.integrate(4, p, *W.unit_box(6), 1e-7)
    assert a == b
