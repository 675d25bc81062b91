"""Parity of the tensor-product Gauss-Kronrod rule kernel (the framework's
second rule, Sec. 3) and of the adaptive loop run with it, against the CPU
oracle's Gauss-Kronrod rule: per region Q, err, split axis and geometry flag
to the per-region bar; per run the same status, iteration count, regions and
final active set, I within 1e-12."""
from __future__ import annotations

import numpy as np
import pytest

import closed_forms as CF
from oracle import oracle as O
from paper_2511_01573_amd import gm, workloads as W
from parity import I_TOL, assert_regions_match

pytestmark = pytest.mark.gpu

GK = O.GAUSS_KRONROD
# regions per case: the oracle evaluates 15^d nodes per region
SIZES = {2: 1000, 3: 300, 4: 67, 5: 9, 6: 2}


def _with_gk(fn, *args, **kw):
    gm.set_option("rule", 1)
    try:
        return fn(*args, **kw)
    finally:
        gm.set_option("rule", 0)


@pytest.mark.parametrize("d", sorted(SIZES))
@pytest.mark.parametrize("fam", [1, 2, 3, 4, 5, 6, 7])
def test_gk_rule_kernel_matches_oracle(fam, d):
    n = SIZES[d]
    p = W.family_params(fam, d, seed=300 * fam + d)
    lo, hi = W.unit_box(d)
    c, h, lvl = W.random_regions(d, n, seed=11 * d + fam)
    ref = O.rule_many(fam, p, c, h, lvl, 1.0, rule_id=GK)
    print(f"case gk fam={fam} d={d} n={n}", flush=True)
    gq, ge, gax = _with_gk(gm.eval_regions, fam, p, lo, hi, c, h, lvl)
    assert_regions_match(gq, ge, gax, ref, f"gk fam{fam} d{d}")


def _run_both(fam, p, d, tau, max_regions=1 << 20, init_log2=6):
    lo, hi = W.unit_box(d)
    gm.set_option("init_log2_regions", init_log2)
    gm.set_option("rule", 1)
    try:
        print(f"case gk loop fam={fam} d={d} tau={tau}", flush=True)
        I, E, st = gm.integrate(fam, p, lo, hi, tau, 1e-16, max_regions)
        stats = gm.last_stats()
        act = gm.last_active(d)
    finally:
        gm.set_option("init_log2_regions", 12)
        gm.set_option("rule", 0)
    run = O.Run(fam, p, lo, hi, tau, 1e-16, max_regions, init_log2, 10000, rule_id=GK)
    run.run()
    ref = run.result()
    assert st == ref["status"], (st, ref)
    assert stats["iterations"] == ref["iterations"]
    assert stats["regions_evaluated"] == ref["regions"]
    assert stats["evals"] == ref["evals"] == ref["regions"] * 15 ** d
    assert abs(I - ref["I"]) <= I_TOL * abs(ref["I"]), (I, ref["I"])
    assert abs(E - ref["E"]) <= 1e-13 * ref["escale"] + 1e-15 * abs(ref["E"]), (E, ref["E"])
    ra = run.active()
    assert np.array_equal(act["lvl"], ra["lvl"])
    assert np.array_equal(act["c"], ra["c"]) and np.array_equal(act["h"], ra["h"])
    full = O.rule_many(fam, p, ra["c"], ra["h"], ra["lvl"], 1.0, rule_id=GK)
    assert_regions_match(act["Q"], act["err"], act["axis"], full, "gk final active set")
    return I, E, st


@pytest.mark.parametrize("fam,d,tau,init_log2", [
    (1, 2, 1e-13, 0), (2, 2, 1e-12, 0), (4, 3, 1e-11, 0), (5, 3, 1e-6, 3), (3, 3, 1e-12, 0),
    (6, 2, 1e-7, 2), (2, 4, 1e-8, 0), (7, 3, 1e-13, 0), (1, 5, 1e-8, 0)])
def test_gk_loop_matches_oracle(fam, d, tau, init_log2):
    p = W.family_params(fam, d, seed=400 * fam + d)
    _run_both(fam, p, d, tau, init_log2=init_log2)


def test_gk_paper_gaussian_d3_closed_form():
    d = 3
    fam, a, u = CF.paper_params(4, d)
    p = np.concatenate([a, u])
    I, E, st = _run_both(fam, p, d, 1e-10, init_log2=3)
    assert st == gm.OK
    assert abs(I - float(CF.exact(fam, a, u))) <= 1e-9 * abs(I)


def test_gk_rejects_unsupported_calls():
    """d = 7 single integrals and the gradient mode are refused."""
    lo, hi = W.unit_box(7)
    p = W.family_params(4, 7, seed=1)
    gm.set_option("rule", 1)
    try:
        with pytest.raises(gm.GMError):
            gm.integrate(4, p, lo, hi, 1e-6, 1e-16, 1 << 20)
        lo3, hi3 = W.unit_box(3)
        p3 = W.family_params(4, 3, seed=1)
        with pytest.raises(gm.GMError):
            gm.integrate_grad(4, p3, lo3, hi3, 1e-6, 1e-16, 1 << 20)
    finally:
        gm.set_option("rule", 0)
    with pytest.raises(gm.GMError):
        gm.set_option("rule", 3)


def test_gk_batch_matches_oracle_lockstep():
    """A batch run with the Gauss-Kronrod rule: per item the oracle's lock-step
    batch with the same rule (same status, I within 1e-12); an item of d = 7
    is invalid under this rule."""
    rng = np.random.default_rng(5)
    fams, ps, ds, los, his, rts = [], [], [], [], [], []
    for i in range(24):
        d = int(rng.integers(2, 5))
        fam = int((1, 2, 4, 3)[int(rng.integers(0, 4))])
        fams.append(fam)
        ps.append(W.family_params(fam, d, seed=3000 + i))
        ds.append(d)
        los.append(np.zeros(d))
        his.append(np.ones(d))
        rts.append(10 ** rng.uniform(-9, -5))
    fams.append(4)
    ps.append(W.family_params(4, 7, seed=1))
    ds.append(7)
    los.append(np.zeros(7))
    his.append(np.ones(7))
    rts.append(1e-6)
    ats = [1e-16] * len(fams)
    gm.set_option("init_log2_regions", 2)
    try:
        print("case gk batch", flush=True)
        rc, est, err, st = _with_gk(gm.integrate_batch, fams, ps, ds, los, his, rts, ats, 1 << 20)
    finally:
        gm.set_option("init_log2_regions", 12)
    assert st[-1] == gm.EINVAL and np.isnan(est[-1])
    orc, oest, oerr, ost, oits = O.integrate_batch(fams[:-1], ps[:-1], ds[:-1], los[:-1], his[:-1],
                                                   rts[:-1], ats[:-1], 1 << 20, init_log2=2,
                                                   rule_id=GK)
    assert np.array_equal(st[:-1], ost)
    assert np.all(np.abs(est[:-1] - oest) <= I_TOL * np.abs(oest))


@pytest.mark.parametrize("fam,d,n", [(4, 3, 70000), (2, 4, 40000), (3, 5, 20000)])
def test_gk_rule_kernel_grid_stride_sampled(fam, d, n):
    """More regions than one pass of the grid covers (16384 workgroups of
    four regions up to d = 3, of one region from d = 4 on), so every
    workgroup loops: a sample of the regions, spread over the whole range,
    against the oracle, and every region's Q finite and err >= 0."""
    p = W.family_params(fam, d, seed=700 * fam + d)
    lo, hi = W.unit_box(d)
    c, h, lvl = W.random_regions(d, n, seed=13 * d + fam)
    print(f"case gk grid-stride fam={fam} d={d} n={n}", flush=True)
    gq, ge, gax = _with_gk(gm.eval_regions, fam, p, lo, hi, c, h, lvl)
    assert np.all(np.isfinite(gq)) and np.all(ge >= 0.0)
    idx = np.unique(np.concatenate([np.arange(8), n - 8 + np.arange(8),
                                    np.random.default_rng(d).integers(0, n, 48)]))
    ref = O.rule_many(fam, p, c[idx], h[idx], lvl[idx], 1.0, rule_id=GK)
    assert_regions_match(gq[idx], ge[idx], gax[idx], ref, f"gk grid-stride fam{fam} d{d}")
