"""Parity at full size, in the launch configuration the benchmark times.

The d = 8 suite at rel_tol 1e-7 (millions of active regions; the serial
oracle would need minutes per integral) cannot be replayed by the oracle, so
each run is checked on sampled outputs.  The loop is stopped after k
iterations (option max_iters) for every k the run takes; windows of the k-th
active set -- the head, seeded random offsets and the ragged tail -- are
re-evaluated one region at a time by the oracle's rule (Sec. 2: Q, err, split
axis and geometry flag to the per-region bar).  The host picks the rule-kernel
mapping (one lane per region, or 4/16/64 lanes per region) from the active
count alone, so the stopped runs launch exactly what the full run launches.
On the whole run: the estimate against the closed form, and the status.

The batch of 4096 mixed-dimension integrals (one gm_integrate_batch call, the
benchmark's capacity and graph replay) is checked item by item against the
oracle's independent runs on a sample of items cheap enough for the oracle;
with every item converged below the shared capacity each item's tree is its
independent tree (lock-step iteration changes nothing else).
"""
from __future__ import annotations

import numpy as np
import pytest

import closed_forms as CF
from oracle import oracle as O
from paper_2511_01573_amd import gm, workloads as W
from parity import I_TOL, assert_regions_match

pytestmark = pytest.mark.gpu


def _windows(n: int, rng, window: int) -> list[tuple[int, int]]:
    if n <= 4 * window:
        return [(0, n)]
    offs = {0, n - window}
    offs.update(int(x) for x in rng.integers(0, n - window, size=3))
    return [(o, window) for o in sorted(offs)]


def _check_iteration(fam, p, d, rng, label):
    n = gm.last_active_count()
    window = 256 if d <= 10 else 32  # the oracle evaluates 2^d + 2d^2 + 2d + 1 nodes per region
    for off, cnt in _windows(n, rng, window):
        act = gm.last_active(d, off, cnt)
        ref = O.rule_many(fam, p, act["c"], act["h"], act["lvl"], 1.0)
        assert_regions_match(act["Q"], act["err"], act["axis"], ref, f"{label} [{off}, {off + cnt})")
    return n


def _sampled_run(c, max_iters_list=None):
    fam, p, d = c["family"], c["params"], len(c["lo"])
    print(f"case {c['name']} cap={c['max_regions']}", flush=True)
    I, E, st = gm.integrate(fam, p, c["lo"], c["hi"], c["rel_tol"], c["abs_tol"], c["max_regions"])
    iters = gm.last_stats()["iterations"]
    rng = np.random.default_rng(fam * 7919 + d)
    ks = range(1, iters + 1) if max_iters_list is None else [k for k in max_iters_list if k <= iters]
    sizes = []
    try:
        for k in ks:
            gm.set_option("max_iters", k)
            Ik, Ek, stk = gm.integrate(fam, p, c["lo"], c["hi"], c["rel_tol"], c["abs_tol"],
                                       c["max_regions"])
            if k < iters:
                assert stk == gm.MAX_ITERS, (k, stk)
            else:
                # deterministic: the same run, the same bits (a run that ran out
                # of capacity in its last iteration reports the iteration budget
                # first, which the loop checks before the classifier)
                assert (Ik, Ek) == (I, E)
                assert stk == st or (st == gm.MAX_REGIONS and stk == gm.MAX_ITERS), (st, stk)
            sizes.append(_check_iteration(fam, p, d, rng, f"{c['name']} iteration {k}"))
    finally:
        gm.set_option("max_iters", 10000)
    return I, E, st, sizes


@pytest.mark.parametrize("fam", W.SIX_FAMILIES)
def test_d8_suite_tightest_tolerance_sampled(fam):
    c = [x for x in W.config2(taus=(1e-7,)) if x["family"] == fam][0]
    I, E, st, sizes = _sampled_run(c)
    d = 8
    exact = float(CF.exact(fam, c["params"][:d], c["params"][d:]))
    assert max(sizes) > 1 << 16  # the full-size regime, not a toy run
    if fam == W.OSCILLATORY:
        # needs more than the 2^24-region store at rel_tol 1e-7
        assert st == gm.MAX_REGIONS
        assert abs(I - exact) <= 10 * E
    elif fam == W.DISCONTINUOUS:
        # converged by its own estimate, but a cut that falls between a
        # region's outermost nodes and its boundary is invisible to the rule,
        # so the true error exceeds the estimate (same on the oracle)
        assert st == gm.OK and E <= 1e-7 * abs(I)
        assert abs(I - exact) <= 2e-3 * abs(exact)
    else:
        assert st == gm.OK and E <= 1e-7 * abs(I)
        assert abs(I - exact) <= 1e-5 * abs(exact), (I, exact, E)


@pytest.mark.parametrize("name", ["corner_peak_d12", "product_peak_d12", "corner_peak_d16",
                                  "product_peak_d16"])
def test_high_dimension_sampled(name):
    """d = 12 and 16 at rel_tol 1e-4 with a 2^27-region store: the wide
    mappings (16 and 64 lanes per region); iterations 1, 2, 4, 8, 16 and the
    last are sampled."""
    c = [x for x in W.config3(max_regions=1 << 27) if x["name"] == name][0]
    I, E, st, sizes = _sampled_run(c, max_iters_list=[1, 2, 4, 8, 16, 10 ** 6])
    d = len(c["lo"])
    exact = float(CF.exact(c["family"], c["params"][:d], c["params"][d:]))
    assert st == gm.OK and E <= 1e-4 * abs(I)
    assert abs(I - exact) <= 1e-3 * abs(exact), (I, exact, E)


def test_batch_4096_sampled_items():
    """The 4096-integral batch as the benchmark runs it (graph replay of 8
    iterations, shared store of 2^28 regions); every 16th item of dimension
    <= 7 is replayed by the oracle as an independent run."""
    b = W.config4()
    n = len(b["families"])
    gm.set_option("graph_iters", 8)
    try:
        print("case batch 4096 cap 2^28", flush=True)
        rc, est, err, st = gm.integrate_batch(b["families"], b["params"], b["ds"], b["los"],
                                              b["his"], b["rel_tols"], b["abs_tols"], 1 << 28)
    finally:
        gm.set_option("graph_iters", 0)
    assert rc == gm.OK and (st == gm.OK).all()
    checked = 0
    for i in range(0, n, 16):
        if b["ds"][i] > 7:
            continue
        ref = O.integrate(b["families"][i], b["params"][i], b["los"][i], b["his"][i],
                          b["rel_tols"][i], b["abs_tols"][i], 1 << 26)
        assert ref["status"] == st[i] == gm.OK, (i, ref["status"], st[i])
        assert abs(est[i] - ref["I"]) <= I_TOL * abs(ref["I"]), (i, est[i], ref["I"])
        assert abs(err[i] - ref["E"]) <= 1e-13 * ref["escale"] + 1e-15 * abs(ref["E"]), (i, err[i], ref["E"])
        checked += 1
    assert checked >= 100


def _batch_high_d_items(b, lo_tau, hi_tau, every):
    """Items of dimension 8..10 with lo_tau <= rel_tol < hi_tau, every
    `every`-th in item order."""
    items = [i for i in range(len(b["families"]))
             if b["ds"][i] >= 8 and lo_tau <= b["rel_tols"][i] < hi_tau]
    return items[::every]


def test_batch_4096_high_dimension_items_to_convergence():
    """Batch items of dimension 8..10 (the batch-store rule kernels that take
    most of the batch's time) replayed by the oracle as independent runs:
    every second item with 1e-5 <= rel_tol < 1e-4 (they converge within 1..5
    iterations; the tighter items are covered by the stopped runs below)."""
    b = W.config4()
    gm.set_option("graph_iters", 8)
    try:
        print("case batch 4096 cap 2^28 (high-d items)", flush=True)
        rc, est, err, st = gm.integrate_batch(b["families"], b["params"], b["ds"], b["los"],
                                              b["his"], b["rel_tols"], b["abs_tols"], 1 << 28)
    finally:
        gm.set_option("graph_iters", 0)
    assert rc == gm.OK and (st == gm.OK).all()
    items = _batch_high_d_items(b, 1e-5, 1e-4, 2)
    assert len(items) >= 150
    multi = 0
    for i in items:
        ref = O.integrate(b["families"][i], b["params"][i], b["los"][i], b["his"][i],
                          b["rel_tols"][i], b["abs_tols"][i], 1 << 26)
        assert ref["status"] == st[i] == gm.OK, (i, ref["status"], st[i])
        assert abs(est[i] - ref["I"]) <= I_TOL * abs(ref["I"]), (i, est[i], ref["I"])
        assert abs(err[i] - ref["E"]) <= 1e-13 * ref["escale"] + 1e-15 * abs(ref["E"]), (i, err[i], ref["E"])
        multi += ref["iterations"] > 1
    assert multi >= 15  # items that refined, not only the initial partition
    assert {b["ds"][i] for i in items} == {8, 9, 10}


@pytest.mark.parametrize("k,count", [(3, 32), (6, 24)])
def test_batch_4096_high_dimension_items_stopped_after_k_iterations(k, count):
    """The whole batch stopped after k lock-step iterations (option
    max_iters, as the benchmark runs it: graph replay of 8 iterations, store of
    2^28 regions): items of dimension 8..10 with rel_tol < 1e-5, spread over
    the tolerance range, against independent oracle runs stopped after k
    iterations (same status, I, E: the rule, reduction, classification and
    splitting of every iteration up to k)."""
    b = W.config4()
    gm.set_option("graph_iters", 8)
    gm.set_option("max_iters", k)
    try:
        print(f"case batch 4096 cap 2^28 max_iters={k}", flush=True)
        rc, est, err, st = gm.integrate_batch(b["families"], b["params"], b["ds"], b["los"],
                                              b["his"], b["rel_tols"], b["abs_tols"], 1 << 28)
    finally:
        gm.set_option("graph_iters", 0)
        gm.set_option("max_iters", 10000)
    tight = sorted(_batch_high_d_items(b, 0.0, 1e-5, 1), key=lambda i: b["rel_tols"][i])
    items = tight[:: max(1, len(tight) // count)][:count]
    stopped = 0
    for i in items:
        ref = O.integrate(b["families"][i], b["params"][i], b["los"][i], b["his"][i],
                          b["rel_tols"][i], b["abs_tols"][i], 1 << 26, max_iters=k)
        assert ref["status"] == st[i], (i, ref["status"], st[i])
        assert abs(est[i] - ref["I"]) <= I_TOL * abs(ref["I"]), (i, est[i], ref["I"])
        assert abs(err[i] - ref["E"]) <= 1e-13 * ref["escale"] + 1e-15 * abs(ref["E"]), (i, err[i], ref["E"])
        stopped += st[i] == gm.MAX_ITERS
    assert stopped >= 3  # items the stop actually cut short
