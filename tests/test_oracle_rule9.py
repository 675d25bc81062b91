"""Pins of the oracle's degree-9 rule (the "9-order" reading of Sec. 2 of
arXiv 2511.01573) against mathematics that does not come from the oracle.

- constants: derived here from scratch by solving the even-moment equations of
  degree <= 8 for the generator structure {0, l2 e_i, l3 e_i, l4 (e_i + e_j),
  l5 (1, .., 1), l6 e_i, (l2 e_i + l3 e_j), l4 (e_i + e_j + e_k)} stage by
  stage; the oracle's doubles must be the correctly rounded solution;
- nodes: count, class sizes, distinctness, full symmetry;
- exactness on every monomial of total degree <= 9 over arbitrary boxes,
  failure on degree 10;
- the error estimates' exact values on x^8 (both models), and zero on
  degree <= 7;
- the fourth-difference split pins (shared with the degree-7 rule);
- brute force: the rule evaluated at 50 digits on the same nodes;
- adaptive runs: closed-form accuracy and a complete frozen tree.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest
import sympy as sp

import closed_forms as cf
from oracle import oracle as O

R = sp.Rational
L2, L3, L5 = R(9, 70), R(9, 10), R(9, 19)


def _derive(d):
    """Solve the 12 even-moment equations (degree <= 8, mean measure on
    [-1,1]^d, d >= 4) stage by stage.  Unknowns: the 8 class weights, the
    triple's lambda^2 (t), the asymmetric pair's lambda^2 (p on the first
    coordinate, q on the second) and l6^2 (s); the pair class reuses l4^2 =
    l3^2 = 9/10, corners and axis classes 2, 3 the degree-7 lambdas."""
    w = sp.symbols("w1:9")
    t, p, q, s = sp.symbols("t p q s", positive=True)
    mom = lambda *e: math.prod(R(1, k + 1) for k in e)  # E[x^e1 y^e2 ...]
    corner = lambda k: w[4] * 2 ** d * L5 ** k  # all 2^d corners, monomial of degree 2k

    # x^2 y^2 z^2 w^2: corners only
    sol = {w[4]: sp.solve(sp.Eq(corner(4), mom(2, 2, 2, 2)), w[4])[0]}
    # x^2 y^2 z^2, x^4 y^2 z^2: triples (8 nodes per triple containing x, y, z) + corners
    e1 = sp.Eq(8 * w[7] * t ** 3 + corner(3), mom(2, 2, 2))
    e2 = sp.Eq(8 * w[7] * t ** 4 + corner(4), mom(4, 2, 2))
    r = sp.solve([e1.subs(sol), e2.subs(sol)], [w[7], t], dict=True)
    assert len(r) == 1
    sol.update(r[0])

    # two-coordinate moments x^a y^b: pair class (4 nodes), asymmetric class
    # (ordered pairs (x, y) and (y, x)), triples containing x and y (d - 2 of
    # them), corners
    def two(a, b):
        pair = 4 * w[3] * L3 ** ((a + b) // 2)
        asym = 4 * w[6] * (p ** (a // 2) * q ** (b // 2) + q ** (a // 2) * p ** (b // 2))
        tri = 8 * (d - 2) * w[7] * t ** ((a + b) // 2)
        return sp.Eq(pair + asym + tri + corner((a + b) // 2), mom(a, b))

    eqs = [two(2, 2).subs(sol), two(4, 2).subs(sol), two(6, 2).subs(sol), two(4, 4).subs(sol)]
    r = [x for x in sp.solve(eqs, [w[3], w[6], p, q], dict=True) if x[p] < x[q]]
    assert len(r) == 1  # unique up to swapping the roles of p and q
    sol.update(r[0])

    # one-coordinate moments x^2 .. x^8: axis classes 2, 3, 6 (2 nodes each),
    # pairs containing x (d - 1), asymmetric nodes with x perturbed (2 (d - 1)
    # ordered pairs), triples containing x (C(d-1, 2)), corners
    def one(a):
        k = a // 2
        ax = 2 * (w[1] * L2 ** k + w[2] * L3 ** k + w[5] * s ** k)
        pair = 4 * (d - 1) * w[3] * L3 ** k
        asym = 4 * (d - 1) * w[6] * (p ** k + q ** k)
        tri = 8 * sp.binomial(d - 1, 2) * w[7] * t ** k
        return sp.Eq(ax + pair + asym + tri + corner(k), mom(a))

    eqs = [one(a).subs(sol) for a in (2, 4, 6, 8)]
    r = sp.solve(eqs, [w[1], w[2], w[5], s], dict=True)
    assert len(r) == 1
    sol.update(r[0])
    counts = [1, 2 * d, 2 * d, 2 * d * (d - 1), 2 ** d, 2 * d, 4 * d * (d - 1),
              8 * math.comb(d, 3)]
    sol[w[0]] = sp.solve(sp.Eq(sum(n * x for n, x in zip(counts[1:], w[1:])).subs(sol) + w[0], 1),
                         w[0])[0]
    lam2 = {"t": sol[t], "p": sol[p], "q": sol[q], "s": sol[s]}
    return [sol[x] for x in w], lam2


def _gm7_weights(d):
    return [Fraction(400 * d * d - 9120 * d + 12824, 19683), Fraction(980, 6561),
            Fraction(1820 - 400 * d, 19683), Fraction(200, 19683),
            Fraction(6859, 19683 * 2 ** d), 0, 0, 0]


@pytest.mark.parametrize("d", [4, 5, 8, 12, 16])
def test_constants_solve_moment_equations(d):
    w, lam2 = _derive(d)
    # the derived lambdas: the triple sits at l4, the asymmetric pair at (l2, l3)
    assert lam2["t"] == L3 and (lam2["p"], lam2["q"]) == (L2, L3)
    assert lam2["s"] == R(759, 1190)
    lam, ow, oe = O.constants9(d)
    w7 = _gm7_weights(d)
    for k in range(8):
        wk = Fraction(int(sp.fraction(w[k])[0]), int(sp.fraction(w[k])[1]))
        assert ow[k] == float(wk), (k, ow[k], float(wk))
        assert oe[k] == float(wk - w7[k]), (k, oe[k], float(wk - w7[k]))
    for k, l2 in zip(range(1, 6), (L2, L3, L3, L5, R(759, 1190))):
        assert lam[k] == float(mp.sqrt(mp.mpf(float(l2))))


def test_node_counts():
    for d in range(2, 12):
        x, cls = O.nodes9(d, np.zeros(d), np.ones(d))
        N = 1 + 6 * d + 6 * d * (d - 1) + 8 * math.comb(d, 3) + 2 ** d
        assert O.num_nodes9(d) == N == x.shape[0]
        counts = [int((cls == k).sum()) for k in range(1, 9)]
        assert counts == [1, 2 * d, 2 * d, 2 * d * (d - 1), 2 ** d, 2 * d, 4 * d * (d - 1),
                          8 * math.comb(d, 3)]
        assert len({tuple(r) for r in x}) == N
        # the degree-7 rule's nodes come first, in its own order
        x7, cls7 = O.nodes(d, np.zeros(d), np.ones(d))
        assert np.array_equal(x[:len(x7)], x7) and np.array_equal(cls[:len(x7)], cls7)


@pytest.mark.parametrize("d", [2, 3, 5])
def test_nodes_fully_symmetric(d):
    x, cls = O.nodes9(d, np.zeros(d), np.ones(d))
    rng = np.random.default_rng(d + 90)
    for _ in range(4):
        perm = rng.permutation(d)
        sign = rng.choice([-1.0, 1.0], size=d)
        for k in range(1, 9):
            a = {tuple(r) for r in x[cls == k]}
            b = {tuple(r) for r in (x[cls == k][:, perm] * sign)}
            assert a == b


@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_rule_exact_on_monomials_over_boxes(d):
    rng = np.random.default_rng(900 + d)
    c = rng.uniform(-1, 1, d)
    h = rng.uniform(0.1, 0.7, d)
    u = rng.uniform(-1, 1, d)
    vol = float(np.prod(2 * h))
    for deg in range(10):
        for ex in cf.all_exponents(d, deg):
            p = np.concatenate([np.array(ex, float), u])
            r = O.rule(O.MONOMIAL, p, c, h, 0, vol, rule_id=O.DEGREE9)
            exact = float(cf.monomial_moment_box(ex, c, h, u)) * vol
            assert abs(r["Q"] - exact) <= 1e-14 * r["scaleQ"] + 1e-300, (ex, r["Q"], exact)
            if deg <= 7:
                assert r["err"] <= 1e-14 * r["scaleE"] + 1e-300, (ex, r["err"])
    # degree 10 is not integrated exactly
    ex = [10] + [0] * (d - 1)
    p = np.concatenate([np.array(ex, float), np.zeros(d)])
    r = O.rule(O.MONOMIAL, p, np.zeros(d), np.ones(d), 0, 2.0 ** d, rule_id=O.DEGREE9)
    assert abs(r["Q"] / 2 ** d - 1 / 11) > 1e-6


def _q_on_x8(w, d):
    """A rule with classes 1..5 of the degree-7 node set applied to x_1^8 on
    [-1,1]^d (mean measure), exact rational."""
    l2, l3, l5 = Fraction(9, 70), Fraction(9, 10), Fraction(9, 19)
    return (2 * w[1] * l2 ** 4 + 2 * w[2] * l3 ** 4 + 4 * (d - 1) * w[3] * l3 ** 4 +
            2 ** d * w[4] * l5 ** 4)


@pytest.mark.parametrize("d", [3, 5, 8, 11])
def test_error_estimate_pins_x8(d):
    """x_1^8: Q9 is exact (1/9); n1 = |1/9 - Q7|, n2 = |Q7 - Q5|, n3 = |Q5 - Q3|
    with the degree-7 and degree-5 weights (pinned by their own moment
    equations) and the degree-3 rule on classes 1 and 3 (exact on 1 and x^2:
    5/27 = 1/(6 l3^2)); model 1 gives n1 min(1, 2 max(n1/n2, n2/n3)).  All are
    independent of d."""
    w7 = _gm7_weights(d)
    v5 = [Fraction(50 * d * d - 950 * d + 729, 729), Fraction(245, 486),
          Fraction(265 - 100 * d, 1458), Fraction(25, 729), Fraction(0)]
    q7 = _q_on_x8(w7, d)
    q5 = _q_on_x8(v5, d)
    q3 = Fraction(5, 27) * 2 * Fraction(9, 10) ** 4
    assert Fraction(5, 27) * 2 * Fraction(9, 10) == Fraction(1, 3)  # Q3 exact on x^2
    n1 = abs(Fraction(1, 9) - q7)
    n2 = abs(q7 - q5)
    n3 = abs(q5 - q3)
    ex = [8] + [0] * (d - 1)
    p = np.concatenate([np.array(ex, float), np.zeros(d)])
    for model, want in ((0, n1), (1, n1 * min(Fraction(1), 2 * max(n1 / n2, n2 / n3)))):
        r = O.rule(O.MONOMIAL, p, np.zeros(d), np.ones(d), 0, 2.0 ** d, rule_id=O.DEGREE9,
                   err_model=model)
        assert abs(r["Q"] / 2 ** d - 1 / 9) <= 1e-15
        assert abs(r["n1"] / 2 ** d - float(n1)) <= 1e-15
        assert abs(r["n2"] / 2 ** d - float(n2)) <= 1e-15
        assert abs(r["n3"] / 2 ** d - float(n3)) <= 1e-15
        assert abs(r["err"] / 2 ** d - float(want)) <= 1e-15 * max(1.0, float(want)), (model,)
    # the numbers themselves: n1 = 1/9 - Q7(x^8), with Q7(x^8) independent of d
    assert n1 == abs(Fraction(1, 9) - _q_on_x8(_gm7_weights(4), 4))


def test_null_rule_model_limits():
    """Model 1 never exceeds model 0 and follows its formula on smooth
    integrands; it is 0 where n1 is 0."""
    rng = np.random.default_rng(5)
    d = 4
    for fam in (cf.GAUSSIAN, cf.OSCILLATORY, cf.PRODUCT_PEAK, cf.CORNER_PEAK):
        for _ in range(5):
            c = rng.uniform(0.2, 0.8, d)
            h = rng.uniform(0.01, 0.2, d)
            p = np.concatenate([rng.uniform(0.5, 4, d), rng.uniform(0, 1, d)])
            r0 = O.rule(fam, p, c, h, 0, None, rule_id=O.DEGREE9, err_model=0)
            r1 = O.rule(fam, p, c, h, 0, None, rule_id=O.DEGREE9, err_model=1)
            assert r1["err"] <= r0["err"] == r0["n1"]
            want = r0["n1"] * min(1.0, 2.0 * max(r0["n1"] / r0["n2"], r0["n2"] / r0["n3"]))
            assert abs(r1["err"] - want) <= 1e-14 * want
    # degree 6 in x: n1 = 0 exactly (Q9 and Q7 both exact), n2 > 0
    ex = [6, 0, 0, 0]
    p = np.concatenate([np.array(ex, float), np.zeros(d)])
    r = O.rule(O.MONOMIAL, p, np.zeros(d), np.ones(d), 0, 16.0, rule_id=O.DEGREE9, err_model=1)
    assert r["n2"] > 0 and r["err"] <= 1e-15 * r["scaleE"]


@pytest.mark.parametrize("d", [2, 4, 7])
def test_fourth_difference_pins(d):
    rng = np.random.default_rng(11 * d)
    c = rng.uniform(-1, 1, d)
    h = rng.uniform(0.05, 0.5, d)
    vol = float(np.prod(2 * h))
    for i in range(d):
        ex = np.zeros(d)
        ex[i] = 4
        r = O.rule(O.MONOMIAL, np.concatenate([ex, c]), c, h, 0, vol, rule_id=O.DEGREE9)
        want = 243 / 1225 * h[i] ** 4
        assert abs(r["D"][i] - want) <= 1e-14 * want
        assert all(r["D"][j] == 0.0 for j in range(d) if j != i)
        assert r["axis"] == i


def _mp_rule9(fam, a, u, c, h):
    d = len(c)
    l2, l3, l5, l6 = (mp.sqrt(mp.mpf(n) / m) for n, m in ((9, 70), (9, 10), (9, 19), (759, 1190)))
    W = [mp.mpf(-160 * (6325 * d ** 3 - 345345 * d ** 2 + 1801355 * d - 1902813)) / 403363719,
         mp.mpf(-490 * (2020 * d - 8711)) / 17891847,
         mp.mpf(5 * (10400 * d * d - 236080 * d + 404019)) / 13817466,
         mp.mpf(-1000 * (2 * d - 9)) / 531441, mp.mpf(130321) / 531441 / 2 ** d,
         mp.mpf(20462645) / 484331562, mp.mpf(4900) / 177147, mp.mpf(1000) / 531441]
    cm = [mp.mpf(float(v)) for v in c]
    hm = [mp.mpf(float(v)) for v in h]
    am = [mp.mpf(float(v)) for v in a]
    um = [mp.mpf(float(v)) for v in u]

    def f(x):
        if fam == cf.GAUSSIAN:
            return mp.exp(-sum((am[j] * (x[j] - um[j])) ** 2 for j in range(d)))
        if fam == cf.CORNER_PEAK:
            return (1 + sum(am[j] * x[j] for j in range(d))) ** (-(d + 1))
        raise ValueError(fam)

    def node(off):
        return [cm[j] + off.get(j, 0) * hm[j] for j in range(d)]

    S = [mp.mpf(0)] * 8
    S[0] = f(node({}))
    for k, l in ((1, l2), (2, l3), (5, l6)):
        for i in range(d):
            S[k] += f(node({i: l})) + f(node({i: -l}))
    for i, j in itertools.combinations(range(d), 2):
        for si, sj in itertools.product((1, -1), repeat=2):
            S[3] += f(node({i: si * l3, j: sj * l3}))
    for i, j in itertools.permutations(range(d), 2):
        for si, sj in itertools.product((1, -1), repeat=2):
            S[6] += f(node({i: si * l2, j: sj * l3}))
    for i, j, k in itertools.combinations(range(d), 3):
        for sg in itertools.product((1, -1), repeat=3):
            S[7] += f(node({i: sg[0] * l3, j: sg[1] * l3, k: sg[2] * l3}))
    for b in range(2 ** d):
        S[4] += f(node({j: (-l5 if (b >> j) & 1 else l5) for j in range(d)}))
    vol = 1
    for v in hm:
        vol *= 2 * v
    return vol * sum(W[k] * S[k] for k in range(8))


@pytest.mark.parametrize("fam", [cf.GAUSSIAN, cf.CORNER_PEAK])
@pytest.mark.parametrize("d", [2, 3, 4])
def test_rule_brute_force_50_digits(fam, d):
    mp.mp.dps = 50
    try:
        rng = np.random.default_rng(fam * 31 + d)
        for _ in range(3):
            c = rng.uniform(0.2, 0.8, d)
            h = rng.uniform(0.01, 0.2, d)
            a = rng.uniform(0.5, 4.0, d)
            u = rng.uniform(0, 1, d)
            r = O.rule(fam, np.concatenate([a, u]), c, h, 0, float(np.prod(2 * h)),
                       rule_id=O.DEGREE9)
            ref = _mp_rule9(fam, a, u, c, h)
            assert abs(r["Q"] - float(ref)) <= 4e-15 * r["scaleQ"], (r["Q"], float(ref))
    finally:
        mp.mp.dps = 40


@pytest.mark.parametrize("fam,d,tau", [(cf.GAUSSIAN, 3, 1e-10), (cf.OSCILLATORY, 4, 1e-9),
                                       (cf.PRODUCT_PEAK, 3, 1e-8), (cf.CORNER_PEAK, 5, 1e-8),
                                       (cf.C0, 3, 1e-6)])
@pytest.mark.parametrize("model", [0, 1])
def test_adaptive_runs_reach_closed_form(fam, d, tau, model):
    from paper_2511_01573_amd import workloads as W
    p = W.family_params(fam, d, 17)
    r = O.Run(fam, p, np.zeros(d), np.ones(d), tau, 1e-16, 1 << 20, 6, keep_leaves=True,
              rule_id=O.DEGREE9, err_model=model)
    r.run()
    res = r.result()
    assert res["status"] == O.OK
    exact = float(cf.exact(fam, p[:d], p[d:]))
    # the closed form lies within a few times the requested tolerance
    assert abs(res["I"] - exact) <= 10 * tau * abs(exact) + 1e-15
    assert res["evals"] == res["regions"] * O.num_nodes9(d)
    _, _, lvl = r.leaves()
    assert sum(math.ldexp(1.0, -int(v)) for v in lvl) == 1.0


def test_degree9_fewer_evaluations_on_a_smooth_integrand():
    """On a smooth integrand at a tight tolerance the higher degree pays: fewer
    integrand evaluations than the degree-7 rule for the same accuracy."""
    from paper_2511_01573_amd import workloads as W
    d, fam, tau = 4, cf.GAUSSIAN, 1e-10
    p = W.family_params(fam, d, 3)
    r7 = O.integrate(fam, p, np.zeros(d), np.ones(d), tau, 1e-16, 1 << 22, 4)
    r9 = O.integrate(fam, p, np.zeros(d), np.ones(d), tau, 1e-16, 1 << 22, 4, rule_id=O.DEGREE9)
    exact = float(cf.exact(fam, p[:d], p[d:]))
    assert r7["status"] == r9["status"] == O.OK
    assert abs(r9["I"] - exact) <= 10 * tau * abs(exact)
    assert r9["evals"] < r7["evals"]


def test_degree9_tree_quadrature_and_gradient():
    """Over the degree-9 frozen tree: the quadrature of the leaves equals the
    run's estimate, and the gradient of that fixed-tree quadrature matches
    central differences of the same quadrature (h = 1e-6) and, for the
    Gaussian, the erf closed form to the run's accuracy."""
    from paper_2511_01573_amd import workloads as W
    d, fam = 3, cf.GAUSSIAN
    p = W.family_params(fam, d, 21)
    res = O.integrate_grad(fam, p, np.zeros(d), np.ones(d), 1e-10, 1e-16, 1 << 20, 3,
                           rule_id=O.DEGREE9)
    c, h, lvl = res["leaves"]
    q, rc = O.quad_leaves(fam, p, c, h, lvl, res["vol_omega"], rule_id=O.DEGREE9)
    assert rc == 0 and abs(q - res["I"]) <= 1e-14 * abs(q)
    g = res["grad"]
    for j in range(2 * d):
        e = np.zeros(2 * d)
        e[j] = 1e-6
        qp, _ = O.quad_leaves(fam, p + e, c, h, lvl, res["vol_omega"], rule_id=O.DEGREE9)
        qm, _ = O.quad_leaves(fam, p - e, c, h, lvl, res["vol_omega"], rule_id=O.DEGREE9)
        fd = (qp - qm) / 2e-6
        assert abs(g[j] - fd) <= 1e-7 * np.abs(g).max(), (j, g[j], fd)
    want = np.array([float(x) for x in cf.gaussian_grad(p[:d], p[d:])])
    assert np.abs(g - want).max() <= 1e-8 * np.abs(want).max()
    # the degree-7 weights on the degree-9 tree give a different (less exact) gradient
    g7 = O.grad_leaves(fam, p, c, h, lvl, res["vol_omega"], 0)
    assert np.abs(g7 - g).max() > 0


def test_degree9_batch_items_equal_independent_runs():
    """The oracle's lock-step batch with the degree-9 rule: below the shared
    budget every item is bitwise its own independent run."""
    from paper_2511_01573_amd import workloads as W
    fams, ds = [4, 1, 2, 3, 5, 4], [2, 3, 4, 5, 3, 6]
    ps = [W.family_params(f, d, 40 + i) for i, (f, d) in enumerate(zip(fams, ds))]
    lo = [np.zeros(d) for d in ds]
    hi = [np.ones(d) for d in ds]
    taus = [1e-9, 1e-8, 1e-7, 1e-7, 1e-5, 1e-6]
    for model in (0, 1):
        rc, est, err, st, its = O.integrate_batch(fams, ps, ds, lo, hi, taus, [1e-16] * 6, 1 << 22,
                                                  init_log2=4, rule_id=O.DEGREE9,
                                                  err_model=model)
        for i in range(6):
            r = O.integrate(fams[i], ps[i], lo[i], hi[i], taus[i], 1e-16, 1 << 22, 4,
                            rule_id=O.DEGREE9, err_model=model)
            assert (est[i], err[i], st[i], its[i]) == (r["I"], r["E"], r["status"],
                                                       r["iterations"])
