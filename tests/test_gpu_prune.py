"""Memory-pressure pruning on the GPU against the oracle: the same budget
factors are chosen, so the runs take the same iterations, evaluate the same
regions and end with the same status, final active set (bitwise) and
estimate (1e-12); the gradient over the pruned frozen tree matches too."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from paper_2511_01573_amd import gm, workloads as W
from parity import I_TOL, assert_regions_match

pytestmark = pytest.mark.gpu


def _run_both(fam, d, cap, tau=1e-8, init_log2=8, seed=77):
    p = W.family_params(fam, d, seed)
    lo, hi = W.unit_box(d)
    gm.set_option("init_log2_regions", init_log2)
    gm.set_option("prune", 1)
    try:
        print(f"case prune fam={fam} d={d} cap={cap}", flush=True)
        I, E, st = gm.integrate(fam, p, lo, hi, tau, 1e-16, cap)
        stats = gm.last_stats()
        act = gm.last_active(d)
    finally:
        gm.set_option("init_log2_regions", 12)
        gm.set_option("prune", 0)
    run = O.Run(fam, p, lo, hi, tau, 1e-16, cap, init_log2, 10000, prune=True)
    run.run()
    ref = run.result()
    assert st == ref["status"], (st, ref)
    assert stats["iterations"] == ref["iterations"]
    assert stats["regions_evaluated"] == ref["regions"]
    assert stats["max_active"] == ref["max_active"] <= cap
    assert abs(I - ref["I"]) <= I_TOL * abs(ref["I"]), (I, ref["I"])
    assert abs(E - ref["E"]) <= 1e-13 * ref["escale"] + 1e-15 * abs(ref["E"]), (E, ref["E"])
    ra = run.active()
    assert np.array_equal(act["lvl"], ra["lvl"])
    assert np.array_equal(act["c"], ra["c"]) and np.array_equal(act["h"], ra["h"])
    full = O.rule_many(fam, p, ra["c"], ra["h"], ra["lvl"], run.vol_omega)
    assert_regions_match(act["Q"], act["err"], act["axis"], full, "pruned final active set")
    return ref


@pytest.mark.parametrize("fam,cap", [(4, 20000), (2, 6000), (3, 2000), (5, 4000), (1, 3000),
                                     (6, 3000)])
def test_pruned_runs_match_oracle(fam, cap):
    ref = _run_both(fam, 4, cap)
    plain = O.integrate(fam, W.family_params(fam, 4, 77), np.zeros(4), np.ones(4), 1e-8, 1e-16,
                        cap, 8)
    if plain["status"] == O.MAX_REGIONS:
        assert ref["pruned"] and ref["E"] <= plain["E"]


def test_prune_has_no_effect_when_store_suffices():
    ref = _run_both(1, 4, 1 << 20)
    assert not ref["pruned"] and ref["status"] == O.OK


def test_pruned_d8_suite_case():
    """A d = 8 case of the benchmark suite on a store small enough to prune."""
    _run_both(4, 8, 1 << 16, tau=1e-6, init_log2=12, seed=4000)


def test_pruned_gradient_matches_oracle():
    fam, d, cap = 4, 4, 20000
    p = W.family_params(fam, d, 77)
    lo, hi = W.unit_box(d)
    gm.set_option("init_log2_regions", 8)
    gm.set_option("prune", 1)
    try:
        I, E, g, st = gm.integrate_grad(fam, p, lo, hi, 1e-8, 1e-16, cap)
    finally:
        gm.set_option("init_log2_regions", 12)
        gm.set_option("prune", 0)
    run = O.Run(fam, p, lo, hi, 1e-8, 1e-16, cap, 8, keep_leaves=True, prune=True)
    run.run()
    ref = run.result()
    c, h, lvl = run.leaves()
    want = O.grad_leaves(fam, p, c, h, lvl, run.vol_omega)
    assert ref["pruned"] and st == ref["status"]
    assert np.max(np.abs(g - want)) <= 1e-12 * np.max(np.abs(want))


def test_batch_rejects_pruning():
    p = W.family_params(4, 3, 1)
    lo, hi = W.unit_box(3)
    gm.set_option("prune", 1)
    try:
        with pytest.raises(gm.GMError):
            gm.integrate_batch([4], [p], [3], [lo], [hi], [1e-6], [1e-16], 1 << 20)
    finally:
        gm.set_option("prune", 0)
