"""Pins of the CPU oracle against mathematics that does not come from the oracle.

- rule constants: re-derived here by solving the moment equations of a
  degree-7 fully symmetric rule (and its embedded degree-5 rule) exactly;
- nodes: count 2^d + 2d^2 + 2d + 1, class sizes, distinctness, symmetry;
- exactness on every monomial of total degree <= 7 (<= 5 for the embedded
  rule) over arbitrary boxes, failure on x^8;
- the error estimate's exact values on x^6, x^4 y^2, x^2 y^2 z^2;
- the fourth-difference pins (243/1225 h^4 on (x_i - c_i)^4, zero on cubics);
- brute force: the rule evaluated at 50 digits on the same nodes.
The rule and estimator follow Sec. 2 of arXiv 2511.01573.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest
import sympy

import closed_forms as cf
from oracle import oracle as O

L2, L3, L4, L5 = Fraction(9, 70), Fraction(9, 10), Fraction(9, 10), Fraction(9, 19)


def sym_rule_on_monomial(d, exps, wts):
    """Mean-measure rule on [-1,1]^d with generator classes 1..5 applied to an
    even monomial; exact rational (lambda^2 are rational)."""
    if any(k % 2 for k in exps):
        return Fraction(0)
    nz = [j for j in range(d) if exps[j]]
    tot = Fraction(0)
    # class 1: the centre
    if not nz:
        tot += wts[0]
    # classes 2, 3: +-lambda e_i
    for cls, l2 in ((1, L2), (2, L3)):
        for i in range(d):
            if all(j == i for j in nz):
                tot += wts[cls] * 2 * l2 ** (exps[i] // 2)
    # class 4: +-lambda e_i +- lambda e_j, i < j
    for i in range(d):
        for j in range(i + 1, d):
            if all(k in (i, j) for k in nz):
                tot += wts[3] * 4 * L4 ** ((exps[i] + exps[j]) // 2)
    # class 5: all 2^d sign corners
    tot += wts[4] * 2 ** d * L5 ** (sum(exps) // 2)
    return tot


def exact_mean(exps):
    m = Fraction(1)
    for k in exps:
        m *= Fraction(0) if k % 2 else Fraction(1, k + 1)
    return m


def solve_weights(d, degree):
    """Solve the moment equations for the class weights (5 for degree 7,
    4 for degree 5 with no corner class)."""
    ws = sympy.symbols("w1:6")
    if degree == 7:
        mons = [(0,), (2,), (4,), (2, 2), (6,), (4, 2), (2, 2, 2)]
        unknowns = ws
    else:
        mons = [(0,), (2,), (4,), (2, 2)]
        unknowns = ws[:4]
    eqs = []
    for m in mons:
        if len(m) > d:
            continue
        exps = list(m) + [0] * (d - len(m))
        wts = list(ws) if degree == 7 else list(ws[:4]) + [0]
        lhs = sym_rule_on_monomial(d, exps, [sympy.Rational(w) if isinstance(w, Fraction) else w
                                             for w in wts])
        eqs.append(sympy.Eq(sympy.nsimplify(lhs) if not isinstance(lhs, Fraction) else lhs,
                            sympy.Rational(exact_mean(exps).numerator, exact_mean(exps).denominator)))
    sol = sympy.solve(eqs, unknowns, dict=True)
    assert len(sol) == 1
    return [Fraction(int(sympy.fraction(sol[0][u])[0]), int(sympy.fraction(sol[0][u])[1]))
            for u in unknowns]


def sym_rule_frac(d, exps, wts):
    # Fraction version for use with Fraction weights
    return sym_rule_on_monomial(d, exps, wts)


@pytest.mark.parametrize("d", [3, 4, 5, 8, 12, 16])
def test_constants_solve_moment_equations(d):
    w = solve_weights(d, 7)
    v = solve_weights(d, 5) + [Fraction(0)]
    lam, ow, ov, oe = O.constants(d)
    for k in range(5):
        assert ow[k] == float(w[k]), (k, ow[k], float(w[k]))
        assert ov[k] == float(v[k]), (k, ov[k], float(v[k]))
        assert oe[k] == float(w[k] - v[k]), (k, oe[k], float(w[k] - v[k]))
    counts = [1, 2 * d, 2 * d, 2 * d * (d - 1), 2 ** d]
    assert sum(n * x for n, x in zip(counts, w)) == 1
    assert sum(n * x for n, x in zip(counts, v)) == 1
    for k, l2 in zip(range(1, 5), (L2, L3, L4, L5)):
        # correctly rounded sqrt of the correctly rounded ratio
        assert lam[k] == float(mp.sqrt(mp.mpf(float(l2))))


def test_constants_d2_exact_on_degree7():
    # d = 2 has no x^2 y^2 z^2 equation; the closed-form weights still integrate degree 7
    _, ow, _, _ = O.constants(2)
    d = 2
    w = [Fraction(400 * d * d - 9120 * d + 12824, 19683), Fraction(980, 6561),
         Fraction(1820 - 400 * d, 19683), Fraction(200, 19683), Fraction(6859, 19683 * 2 ** d)]
    for k in range(5):
        assert ow[k] == float(w[k])
    for deg in range(8):
        for ex in cf.all_exponents(d, deg):
            assert sym_rule_frac(d, ex, w) == exact_mean(ex)


@pytest.mark.parametrize("d", list(range(2, 11)))
def test_node_count_and_classes(d):
    c = np.zeros(d)
    h = np.ones(d)
    x, cls = O.nodes(d, c, h)
    N = 2 ** d + 2 * d * d + 2 * d + 1
    assert O.num_nodes(d) == N == x.shape[0]
    counts = [int((cls == k).sum()) for k in range(1, 6)]
    assert counts == [1, 2 * d, 2 * d, 2 * d * (d - 1), 2 ** d]
    assert len({tuple(r) for r in x}) == N  # all distinct


@pytest.mark.parametrize("d", [2, 3, 5])
def test_nodes_fully_symmetric(d):
    x, cls = O.nodes(d, np.zeros(d), np.ones(d))
    rng = np.random.default_rng(d)
    for _ in range(4):
        perm = rng.permutation(d)
        sign = rng.choice([-1.0, 1.0], size=d)
        for k in range(1, 6):
            a = {tuple(r) for r in x[cls == k]}
            b = {tuple(r) for r in (x[cls == k][:, perm] * sign)}
            assert a == b


def _box(rng, d):
    c = rng.uniform(-1, 1, d)
    h = rng.uniform(0.1, 0.7, d)
    u = rng.uniform(-1, 1, d)
    return c, h, u


@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_rule_exact_on_monomials_over_boxes(d):
    rng = np.random.default_rng(100 + d)
    c, h, u = _box(rng, d)
    vol = float(np.prod(2 * h))
    for deg in range(8):
        for ex in cf.all_exponents(d, deg):
            p = np.concatenate([np.array(ex, float), u])
            r = O.rule(O.MONOMIAL, p, c, h, 0, vol)
            exact = float(cf.monomial_moment_box(ex, c, h, u)) * vol
            assert abs(r["Q"] - exact) <= 1e-14 * r["scaleQ"] + 1e-300, (ex, r["Q"], exact)
            if deg <= 5:
                # embedded degree-5 rule exact as well -> estimate at round-off level
                assert r["err"] <= 1e-14 * r["scaleE"] + 1e-300, (ex, r["err"])
    # degree 8 is not integrated exactly
    ex = [8] + [0] * (d - 1)
    p = np.concatenate([np.array(ex, float), np.zeros(d)])
    r = O.rule(O.MONOMIAL, p, np.zeros(d), np.ones(d), 0, 2.0 ** d)
    assert abs(r["Q"] / 2 ** d - 1 / 9) > 1e-3


@pytest.mark.parametrize("d", [3, 5, 8])
def test_error_estimate_pins(d):
    # per unit mean measure on [-1,1]^d: err(x^6) = 17/700, err(x^4 y^2) = 1/30,
    # err(x^2 y^2 z^2) = 1/27, independent of d
    cases = [([6], Fraction(17, 700)), ([4, 2], Fraction(1, 30)), ([2, 2, 2], Fraction(1, 27))]
    for m, val in cases:
        ex = m + [0] * (d - len(m))
        p = np.concatenate([np.array(ex, float), np.zeros(d)])
        r = O.rule(O.MONOMIAL, p, np.zeros(d), np.ones(d), 0, 2.0 ** d)
        assert abs(r["err"] / 2 ** d - float(val)) <= 1e-14, (m, r["err"] / 2 ** d)


@pytest.mark.parametrize("d", [2, 4, 7])
def test_fourth_difference_pins(d):
    rng = np.random.default_rng(7 * d)
    c = rng.uniform(-1, 1, d)
    h = rng.uniform(0.05, 0.5, d)
    vol = float(np.prod(2 * h))
    for i in range(d):
        ex = np.zeros(d)
        ex[i] = 4
        p = np.concatenate([ex, c])  # (x_i - c_i)^4
        r = O.rule(O.MONOMIAL, p, c, h, 0, vol)
        want = 243 / 1225 * h[i] ** 4
        assert abs(r["D"][i] - want) <= 1e-14 * want
        for j in range(d):
            if j != i:
                assert r["D"][j] == 0.0
        assert r["axis"] == i
        # a cubic in x_i: second derivative cancelled by the 1/7 ratio
        ex3 = np.zeros(d)
        ex3[i] = 3
        p3 = np.concatenate([ex3, c + 0.3])
        r3 = O.rule(O.MONOMIAL, p3, c, h, 0, vol)
        assert abs(r3["D"][i]) <= 1e-13 * (1 + np.abs(c + h).max()) ** 3


def test_axis_tie_goes_to_widest_then_lowest():
    # every D is ~0 for a cubic -> all axes are within the noise band
    d = 3
    c = np.array([0.1, 0.2, 0.3])
    h = np.array([0.1, 0.3, 0.2])
    p = np.concatenate([np.array([3.0, 0, 0]), np.zeros(3)])
    assert O.rule(O.MONOMIAL, p, c, h)["axis"] == 1
    h2 = np.array([0.25, 0.25, 0.25])
    assert O.rule(O.MONOMIAL, p, c, h2)["axis"] == 0


def _mp_rule(fam, a, u, c, h):
    d = len(c)
    lam = [0, mp.sqrt(mp.mpf(9) / 70), mp.sqrt(mp.mpf(9) / 10), mp.sqrt(mp.mpf(9) / 10),
           mp.sqrt(mp.mpf(9) / 19)]
    W = [mp.mpf(400 * d * d - 9120 * d + 12824) / 19683, mp.mpf(980) / 6561,
         mp.mpf(1820 - 400 * d) / 19683, mp.mpf(200) / 19683, mp.mpf(6859) / 19683 / 2 ** d]
    cm = [mp.mpf(float(v)) for v in c]
    hm = [mp.mpf(float(v)) for v in h]
    am = [mp.mpf(float(v)) for v in a]
    um = [mp.mpf(float(v)) for v in u]

    def f(x):
        if fam == cf.GAUSSIAN:
            return mp.exp(-sum((am[j] * (x[j] - um[j])) ** 2 for j in range(d)))
        if fam == cf.OSCILLATORY:
            return mp.cos(mp.mpf(6.283185307179586476925286766559 * float(u[0])) +
                          sum(am[j] * x[j] for j in range(d)))
        if fam == cf.PRODUCT_PEAK:
            p = mp.mpf(1)
            for j in range(d):
                p /= 1 / am[j] ** 2 + (x[j] - um[j]) ** 2
            return p
        if fam == cf.CORNER_PEAK:
            return (1 + sum(am[j] * x[j] for j in range(d))) ** (-(d + 1))
        raise ValueError(fam)

    def node(offsets):
        return [cm[j] + offsets.get(j, 0) * hm[j] for j in range(d)]

    S = [mp.mpf(0)] * 5
    S[0] = f(node({}))
    for k, l in ((1, lam[1]), (2, lam[2])):
        for i in range(d):
            S[k] += f(node({i: l})) + f(node({i: -l}))
    for i in range(d):
        for j in range(i + 1, d):
            for si in (1, -1):
                for sj in (1, -1):
                    S[3] += f(node({i: si * lam[3], j: sj * lam[3]}))
    for b in range(2 ** d):
        S[4] += f(node({j: (-lam[4] if (b >> j) & 1 else lam[4]) for j in range(d)}))
    vol = 1
    for v in hm:
        vol *= 2 * v
    return vol * sum(W[k] * S[k] for k in range(5))


@pytest.mark.parametrize("fam", [cf.GAUSSIAN, cf.OSCILLATORY, cf.PRODUCT_PEAK, cf.CORNER_PEAK])
@pytest.mark.parametrize("d", [2, 3])
def test_rule_brute_force_50_digits(fam, d):
    mp.mp.dps = 50
    rng = np.random.default_rng(fam * 10 + d)
    for _ in range(4):
        c = rng.uniform(0.2, 0.8, d)
        h = rng.uniform(0.01, 0.2, d)
        a = rng.uniform(0.5, 4.0, d)
        u = rng.uniform(0, 1, d)
        p = np.concatenate([a, u])
        r = O.rule(fam, p, c, h, 0, float(np.prod(2 * h)))
        ref = _mp_rule(fam, a, u, c, h)
        # coordinates are rounded once (fma) in the oracle: allow a few ulp
        assert abs(r["Q"] - float(ref)) <= 4e-15 * r["scaleQ"], (r["Q"], float(ref))
    mp.mp.dps = 40
