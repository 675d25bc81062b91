"""Parity of the degree-9 rule kernel (the "9-order" fully symmetric rule of
Sec. 2, with its two error models) and of the adaptive loop run with it,
against the CPU oracle's degree-9 rule: per region Q, err, split axis and
geometry flag to the per-region bar; per run the same status, iteration
count, regions and final active set, I within 1e-12."""
from __future__ import annotations

import numpy as np
import pytest

import closed_forms as CF
from oracle import oracle as O
from paper_2511_01573_amd import gm, workloads as W
from parity import I_TOL, assert_regions_match

pytestmark = pytest.mark.gpu

R9 = O.DEGREE9
# regions per case: several blocks of the kernel's launch and a ragged tail
# (regions per block: 64 for d = 2..7, then 32, 16, 8 for d = 8, 9, 10 and 4 above)
SIZES = {2: 203, 3: 197, 4: 150, 5: 133, 6: 129, 7: 101, 8: 83, 9: 37, 10: 29, 11: 13, 12: 11, 13: 7,
         14: 6, 15: 5, 16: 5}


class _Rule9:
    def __init__(self, model=0):
        self.model = model

    def __enter__(self):
        gm.set_option("rule", 2)
        gm.set_option("err_model", self.model)

    def __exit__(self, *exc):
        gm.set_option("rule", 0)
        gm.set_option("err_model", 0)


@pytest.mark.parametrize("model", [0, 1])
@pytest.mark.parametrize("d", sorted(SIZES))
@pytest.mark.parametrize("fam", [1, 2, 3, 4, 5, 6, 7])
def test_rule9_kernel_matches_oracle(fam, d, model):
    n = SIZES[d]
    p = W.family_params(fam, d, seed=500 * fam + d)
    lo, hi = W.unit_box(d)
    c, h, lvl = W.random_regions(d, n, seed=13 * d + fam)
    ref = O.rule_many(fam, p, c, h, lvl, 1.0, rule_id=R9, err_model=model)
    print(f"case rule9 fam={fam} d={d} n={n} model={model}", flush=True)
    with _Rule9(model):
        gq, ge, gax = gm.eval_regions(fam, p, lo, hi, c, h, lvl)
    assert_regions_match(gq, ge, gax, ref, f"rule9 fam{fam} d{d} model{model}")


def _run_both(fam, p, d, tau, model=0, max_regions=1 << 20, init_log2=6, prune=False):
    lo, hi = W.unit_box(d)
    gm.set_option("init_log2_regions", init_log2)
    gm.set_option("prune", 1 if prune else 0)
    try:
        print(f"case rule9 loop fam={fam} d={d} tau={tau} model={model} cap={max_regions}",
              flush=True)
        with _Rule9(model):
            I, E, st = gm.integrate(fam, p, lo, hi, tau, 1e-16, max_regions)
            stats = gm.last_stats()
            act = gm.last_active(d)
    finally:
        gm.set_option("init_log2_regions", 12)
        gm.set_option("prune", 0)
    run = O.Run(fam, p, lo, hi, tau, 1e-16, max_regions, init_log2, 10000, rule_id=R9,
                err_model=model, prune=prune)
    run.run()
    ref = run.result()
    assert st == ref["status"], (st, ref)
    assert stats["iterations"] == ref["iterations"]
    assert stats["regions_evaluated"] == ref["regions"]
    assert stats["evals"] == ref["evals"] == ref["regions"] * O.num_nodes9(d)
    assert abs(I - ref["I"]) <= I_TOL * abs(ref["I"]), (I, ref["I"])
    assert abs(E - ref["E"]) <= 1e-13 * ref["escale"] + 1e-15 * abs(ref["E"]), (E, ref["E"])
    ra = run.active()
    assert np.array_equal(act["lvl"], ra["lvl"])
    assert np.array_equal(act["c"], ra["c"]) and np.array_equal(act["h"], ra["h"])
    full = O.rule_many(fam, p, ra["c"], ra["h"], ra["lvl"], run.vol_omega, rule_id=R9,
                       err_model=model)
    assert_regions_match(act["Q"], act["err"], act["axis"], full, "rule9 final active set")
    return I, E, st, ref


@pytest.mark.parametrize("fam,d,tau,init_log2,model", [
    (4, 3, 1e-10, 0, 0), (1, 4, 1e-9, 0, 0), (2, 3, 1e-8, 3, 0), (3, 5, 1e-8, 0, 0),
    (5, 3, 1e-6, 3, 0), (6, 3, 1e-5, 3, 0), (7, 3, 1e-12, 0, 0), (4, 8, 1e-6, 8, 0),
    (4, 3, 1e-10, 0, 1), (2, 4, 1e-7, 4, 1), (3, 5, 1e-8, 0, 1), (1, 6, 1e-7, 6, 1),
    (5, 2, 1e-9, 2, 1)])
def test_rule9_loop_matches_oracle(fam, d, tau, init_log2, model):
    p = W.family_params(fam, d, seed=600 * fam + d)
    _run_both(fam, p, d, tau, model, init_log2=init_log2)


def test_rule9_paper_gaussian_d3_closed_form():
    d = 3
    fam, a, u = CF.paper_params(4, d)
    p = np.concatenate([a, u])
    I, E, st, _ = _run_both(fam, p, d, 1e-10, init_log2=3)
    assert st == gm.OK
    assert abs(I - float(CF.exact(fam, a, u))) <= 1e-9 * abs(I)


def test_rule9_pruned_run_matches_oracle():
    fam, d = 4, 4
    p = W.family_params(fam, d, seed=77)
    plain = O.integrate(fam, p, np.zeros(d), np.ones(d), 1e-12, 1e-16, 3000, 8, rule_id=R9)
    assert plain["status"] == O.MAX_REGIONS
    _, _, st, ref = _run_both(fam, p, d, 1e-12, max_regions=3000, init_log2=8, prune=True)
    assert ref["pruned"] and ref["max_active"] <= 3000


@pytest.mark.parametrize("fam,d,tau", [(3, 12, 1e-6), (2, 10, 1e-7)])
def test_rule9_large_run_samples_match_oracle(fam, d, tau):
    """A run too large for the oracle to repeat: the final active set, sampled,
    against the oracle's rule region by region; the estimate against the
    closed form."""
    p = W.family_params(fam, d, seed=700 * fam + d)
    lo, hi = W.unit_box(d)
    print(f"case rule9 large fam={fam} d={d} tau={tau}", flush=True)
    with _Rule9(0):
        I, E, st = gm.integrate(fam, p, lo, hi, tau, 1e-16, 1 << 22)
        act = gm.last_active(d)
        stats = gm.last_stats()
    assert st == gm.OK
    exact = float(CF.exact(fam, p[:d], p[d:]))
    assert abs(I - exact) <= 10 * tau * abs(exact)
    assert stats["evals"] == stats["regions_evaluated"] * O.num_nodes9(d)
    n = act["lvl"].size
    assert n > 0
    idx = np.random.default_rng(d).choice(n, size=min(n, 40), replace=False)
    full = O.rule_many(fam, p, act["c"][idx], act["h"][idx], act["lvl"][idx], 1.0, rule_id=R9)
    assert_regions_match(act["Q"][idx], act["err"][idx], act["axis"][idx], full,
                         "rule9 large sample")


def _small_batch(n, seed, dmin=3, dmax=6, fams=(1, 2, 4, 3)):
    rng = np.random.default_rng(seed)
    out = [[] for _ in range(7)]
    for i in range(n):
        d = int(rng.integers(dmin, dmax + 1))
        fam = int(fams[int(rng.integers(0, len(fams)))])
        for lst, v in zip(out, (fam, W.family_params(fam, d, seed=seed * 100000 + i), d,
                                np.zeros(d), np.ones(d), 10 ** rng.uniform(-8, -4), 1e-16)):
            lst.append(v)
    return out


@pytest.mark.parametrize("graph_iters,model", [(0, 0), (4, 0), (0, 1)])
def test_rule9_batch_matches_oracle_lockstep(graph_iters, model):
    """Every item of a degree-9 batch: the oracle's lock-step batch with the
    same rule gives the same status and I within 1e-12; sampled items equal
    their own single-integral degree-9 runs."""
    b = _small_batch(48, seed=11 + model)
    gm.set_option("init_log2_regions", 6)
    gm.set_option("graph_iters", graph_iters)
    try:
        print(f"case rule9 batch graph_iters={graph_iters} model={model}", flush=True)
        with _Rule9(model):
            rc, est, err, st = gm.integrate_batch(*b, 1 << 22)
    finally:
        gm.set_option("init_log2_regions", 12)
        gm.set_option("graph_iters", 0)
    orc, oest, oerr, ost, oits = O.integrate_batch(*b, 1 << 22, init_log2=6, rule_id=R9,
                                                   err_model=model)
    assert rc == orc
    assert np.array_equal(st, ost)
    assert np.all(np.abs(est - oest) <= I_TOL * np.abs(oest) + 1e-300)
    for i in range(0, 48, 11):
        gm.set_option("init_log2_regions", 6)
        try:
            with _Rule9(model):
                I, E, s1 = gm.integrate(b[0][i], b[1][i], b[3][i], b[4][i], b[5][i], 1e-16,
                                        1 << 22)
                one = gm.last_stats()
        finally:
            gm.set_option("init_log2_regions", 12)
        assert s1 == st[i]
        assert abs(I - est[i]) <= I_TOL * abs(I), (i, I, est[i])
        assert abs(E - err[i]) <= 1e-9 * E, (i, E, err[i])
        assert one["evals"] == one["regions_evaluated"] * O.num_nodes9(b[2][i])


@pytest.mark.parametrize("fam,d,tau,model", [(4, 3, 1e-9, 0), (1, 4, 1e-8, 1), (2, 3, 1e-8, 0),
                                             (3, 4, 1e-8, 0), (5, 3, 1e-6, 0)])
def test_rule9_gradient_matches_oracle(fam, d, tau, model):
    """Gradient mode with the degree-9 rule: the frozen tree is the oracle's,
    and the adjoint over it matches the oracle's fixed-tree gradient with the
    degree-9 nodes and weights to 1e-12 of the largest component."""
    p = W.family_params(fam, d, seed=800 * fam + d)
    lo, hi = W.unit_box(d)
    gm.set_option("init_log2_regions", 6)
    try:
        print(f"case rule9 grad fam={fam} d={d} tau={tau} model={model}", flush=True)
        with _Rule9(model):
            I, E, g, st = gm.integrate_grad(fam, p, lo, hi, tau, 1e-16, 1 << 20)
    finally:
        gm.set_option("init_log2_regions", 12)
    ref = O.integrate_grad(fam, p, lo, hi, tau, 1e-16, 1 << 20, 6, rule_id=R9, err_model=model)
    assert st == ref["status"]
    assert abs(I - ref["I"]) <= I_TOL * abs(ref["I"])
    assert np.max(np.abs(g - ref["grad"])) <= 1e-12 * np.max(np.abs(ref["grad"]))
    if fam == 4:
        want = np.array([float(x) for x in CF.gaussian_grad(p[:d], p[d:])])
        assert np.abs(g - want).max() <= 1e-7 * np.abs(want).max()


def test_rule9_general_box_and_iteration_budget():
    """A box other than the unit cube (vol_omega != 1) and a run stopped by the
    iteration budget: status, iterations, regions, I and the final active set
    as the oracle's."""
    fam, d = 4, 3
    p = W.family_params(fam, d, seed=33)
    lo, hi = np.array([-0.5, 0.25, -1.0]), np.array([1.5, 1.0, 0.75])
    for max_iters in (3, 10000):
        gm.set_option("init_log2_regions", 3)
        gm.set_option("max_iters", max_iters)
        try:
            print(f"case rule9 box max_iters={max_iters}", flush=True)
            with _Rule9(0):
                I, E, st = gm.integrate(fam, p, lo, hi, 1e-11, 1e-16, 1 << 20)
                stats = gm.last_stats()
                act = gm.last_active(d)
        finally:
            gm.set_option("init_log2_regions", 12)
            gm.set_option("max_iters", 10000)
        run = O.Run(fam, p, lo, hi, 1e-11, 1e-16, 1 << 20, 3, max_iters, rule_id=R9)
        run.run()
        ref = run.result()
        assert st == ref["status"] == (gm.MAX_ITERS if max_iters == 3 else gm.OK)
        assert stats["iterations"] == ref["iterations"]
        assert stats["regions_evaluated"] == ref["regions"]
        assert abs(I - ref["I"]) <= I_TOL * abs(ref["I"])
        ra = run.active()
        assert np.array_equal(act["c"], ra["c"]) and np.array_equal(act["h"], ra["h"])
        full = O.rule_many(fam, p, ra["c"], ra["h"], ra["lvl"], run.vol_omega, rule_id=R9)
        assert_regions_match(act["Q"], act["err"], act["axis"], full, "rule9 general box")


@pytest.mark.parametrize("rule_id", [O.DEGREE9, O.GAUSS_KRONROD])
def test_other_rules_status_codes_match_oracle(rule_id):
    """The non-finite and precision-limit stops under the degree-9 and
    Gauss-Kronrod rules: the corner peak with a = (-1, -1) on [0,1]^2 is
    infinite at cell centres of the initial grid (both rules evaluate the
    centre); a nearly constant integrand with rel_tol 0 ends when every
    region's error falls below the resolution of |I|."""
    cases = [(3, np.array([-1.0, -1.0, 0.0, 0.0]), 2, 1e-6, 1e-16, gm.NONFINITE),
             (4, np.array([1e-3] * 3 + [0.5] * 3), 3, 0.0, 1e-300, gm.PRECISION_LIMIT)]
    for fam, p, d, tau, atol, want in cases:
        lo, hi = W.unit_box(d)
        gm.set_option("rule", int(rule_id))
        gm.set_option("init_log2_regions", 4)
        try:
            print(f"case rule{rule_id} status fam={fam} d={d}", flush=True)
            I, E, st = gm.integrate(fam, p, lo, hi, tau, atol, 1 << 20)
            stats = gm.last_stats()
        finally:
            gm.set_option("rule", 0)
            gm.set_option("init_log2_regions", 12)
        run = O.Run(fam, p, lo, hi, tau, atol, 1 << 20, 4, 10000, rule_id=int(rule_id))
        run.run()
        ref = run.result()
        assert st == ref["status"] == want, (st, ref)
        assert stats["iterations"] == ref["iterations"]
        if want == gm.NONFINITE:
            assert np.isnan(I) and np.isnan(E)
        else:
            assert abs(I - ref["I"]) <= I_TOL * abs(ref["I"])
