"""Memory-pressure pruning in the oracle (the classifier's budget relaxed by
the smallest power of two that lets the kept regions fit the store): no
effect while the store suffices, the store is never exceeded, the frozen tree
still tiles the domain, the pruned run ends with the capacity status and an
error estimate no worse than the unpruned run's, the estimate brackets the
closed form, and each pruning step keeps exactly the regions above the
smallest sufficient budget factor."""
from __future__ import annotations

import math

import numpy as np
import pytest

import closed_forms as CF
from oracle import oracle as O
from paper_2511_01573_amd import workloads as W


def _case(fam, d=4, seed=77):
    p = W.family_params(fam, d, seed)
    return p, np.zeros(d), np.ones(d)


@pytest.mark.parametrize("fam", [1, 5, 6])
def test_no_effect_when_store_suffices(fam):
    p, lo, hi = _case(fam)
    a = O.integrate(fam, p, lo, hi, 1e-8, 1e-16, 20000, 8)
    b = O.integrate(fam, p, lo, hi, 1e-8, 1e-16, 20000, 8, prune=True)
    assert not b["pruned"]
    assert (a["I"], a["E"], a["status"], a["regions"]) == (b["I"], b["E"], b["status"], b["regions"])


@pytest.mark.parametrize("fam,cap", [(4, 20000), (2, 6000), (3, 2000), (5, 4000)])
def test_pruned_run_properties(fam, cap):
    d = 4
    p, lo, hi = _case(fam, d)
    plain = O.integrate(fam, p, lo, hi, 1e-8, 1e-16, cap, 8)
    assert plain["status"] == O.MAX_REGIONS
    r = O.Run(fam, p, lo, hi, 1e-8, 1e-16, cap, 8, keep_leaves=True, prune=True)
    r.run()
    res = r.result()
    assert res["pruned"]
    assert res["status"] in (O.OK, O.MAX_REGIONS)
    assert res["max_active"] <= cap
    assert res["E"] <= plain["E"]
    c, h, lvl = r.leaves()
    assert sum(math.ldexp(1.0, -int(l)) for l in lvl) == 1.0
    exact = float(CF.exact(fam, p[:d], p[d:]))
    assert abs(res["I"] - exact) <= res["E"]


def test_each_step_keeps_the_regions_above_the_smallest_sufficient_factor():
    """Every iteration of a pruning run, re-derived from the evaluated set: the
    base classifier's retired regions, and when the rest does not fit half the
    store, the regions with err <= T 2^(k* - lvl) for the smallest k* >= 1
    whose survivors fit; the trace's retired count must match."""
    fam, d, cap = 4, 4, 20000
    p, lo, hi = _case(fam, d)
    r = O.Run(fam, p, lo, hi, 1e-8, 1e-16, cap, 8, prune=True)
    pruned_steps = 0
    while True:
        act = r.active()
        st = r.step()
        counts, IE = r.trace()
        n_act, n_fin = (int(v) for v in counts[-1])
        I = IE[-1][0]
        if st in (O.OK, O.MAX_ITERS):
            break
        T = max(1e-16, 1e-8 * abs(I))
        ref = O.rule_many(fam, p, act["c"], act["h"], act["lvl"], r.vol_omega)
        err, lvl, geo = ref["err"], act["lvl"], ref["geo"]
        base = [(e <= math.ldexp(T, -int(l))) or (abs(I) + e == abs(I)) or bool(g)
                for e, l, g in zip(err, lvl, geo)]
        kept = [i for i in range(n_act) if not base[i]]
        if 2 * len(kept) <= cap:
            assert n_fin == n_act - len(kept)
        else:
            def level(e, l):
                for k in range(1, 65):
                    if e <= math.ldexp(T, k - int(l)):
                        return k
                return 65
            ks = [level(err[i], lvl[i]) for i in kept]
            kstar = next(k for k in range(1, 65) if 2 * sum(1 for v in ks if v > k) <= cap)
            survivors = sum(1 for v in ks if v > kstar)
            assert n_fin == n_act - survivors
            pruned_steps += 1
        if st != O.RUNNING:
            break
    assert pruned_steps >= 1
