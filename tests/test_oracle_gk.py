"""Pins of the oracle's tensor-product Gauss-Kronrod rule (the framework's
second rule, Sec. 3) against what the mathematics fixes, independently of the
oracle's own construction:

- the 7 Gauss abscissae are the roots of P7 (mpmath's Legendre polynomial) and
  their weights follow the closed form 2 / ((1 - x^2) P7'(x)^2);
- the 15-point Kronrod rule is exact for every monomial up to degree 22 (the
  defining property of the extension, 3n + 1 for n = 7) and not for x^24;
- the Gauss rule's error on x^14 equals the textbook remainder
  2^(2n+1) (n!)^4 / ((2n+1) ((2n)!)^3) * f^(2n) for n = 7;
- on boxes, the tensor rule reproduces these per axis, its one-axis
  estimates single out the axis a monomial depends on, brute-force 50-digit
  evaluation of the same nodes agrees, and adaptive runs converge to closed
  forms.
"""
from __future__ import annotations

import itertools

import mpmath as mp
import numpy as np
import pytest

import closed_forms as CF
from oracle import oracle as O

mp.mp.dps = 50
GK = O.GAUSS_KRONROD


def test_gauss_abscissae_are_roots_of_p7_and_weights_closed_form():
    x, wk, wg = O.gk_constants()
    gauss = [x[i] for i in range(1, 15, 2)]
    assert all(wg[i] == 0.0 for i in range(0, 15, 2))
    for xi, wi in zip(gauss, [wg[i] for i in range(1, 15, 2)]):
        root = mp.findroot(lambda t: mp.legendre(7, t), mp.mpf(xi))
        assert abs(mp.mpf(xi) - root) <= mp.mpf(2) ** -53 * max(1, abs(root))
        dp = mp.diff(lambda t: mp.legendre(7, t), root)
        w_exact = 2 / ((1 - root ** 2) * dp ** 2) / 2  # mean measure on [-1, 1]
        assert abs(mp.mpf(wi) - w_exact) <= mp.mpf(2) ** -52 * w_exact


def _rule_1d(x, w, k):
    return mp.fsum(mp.mpf(wi) * mp.mpf(xi) ** k for xi, wi in zip(x, w))


def test_kronrod_exact_to_degree_22_not_24():
    x, wk, wg = O.gk_constants()
    assert abs(mp.fsum(mp.mpf(v) for v in wk) - 1) < 1e-15
    for k in range(0, 23):
        exact = mp.mpf(1) / (k + 1) if k % 2 == 0 else mp.mpf(0)
        assert abs(_rule_1d(x, wk, k) - exact) < 2e-16, k
    assert abs(_rule_1d(x, wk, 24) - mp.mpf(1) / 25) > 1e-12
    # abscissae interlace: Kronrod nodes strictly between consecutive Gauss nodes
    assert np.all(np.diff(x) > 0) and x[0] > -1 and x[-1] < 1


def test_gauss_exact_to_13_and_textbook_remainder_at_14():
    x, wk, wg = O.gk_constants()
    for k in range(0, 14):
        exact = mp.mpf(1) / (k + 1) if k % 2 == 0 else mp.mpf(0)
        assert abs(_rule_1d(x, wg, k) - exact) < 2e-16, k
    n = 7
    remainder = (mp.mpf(2) ** (2 * n + 1) * mp.factorial(n) ** 4 /
                 ((2 * n + 1) * mp.factorial(2 * n) ** 3)) * mp.factorial(2 * n)
    got = (mp.mpf(1) / 15 - _rule_1d(x, wg, 14)) * 2  # back to the [-1, 1] measure
    # the double-rounded nodes and weights move G7(x^14) (about 0.13) by a few
    # ulps; a wrong node or weight would move it by orders of magnitude more
    assert abs(got - remainder) <= 2e-15


def _fma(a, b, c):
    """a * b + c rounded once (the product is exact at 50 digits)."""
    return float(mp.mpf(a) * mp.mpf(b) + mp.mpf(c))


def _monomial_params(ks, u):
    return np.concatenate([np.asarray(ks, float), np.asarray(u, float)])


@pytest.mark.parametrize("d", [2, 3])
def test_tensor_rule_exact_on_monomials_of_each_axis_degree_le_22(d):
    rng = np.random.default_rng(100 + d)
    c = rng.uniform(-1, 1, d)
    h = rng.uniform(0.1, 0.6, d)
    u = rng.uniform(-1, 1, d)
    degs = [0, 1, 5, 13, 14, 22] if d == 2 else [0, 3, 14, 22]
    for ks in itertools.product(degs, repeat=d):
        r = O.rule(O.MONOMIAL, _monomial_params(ks, u), c, h, rule_id=GK)
        exact = float(CF.monomial_moment_box(ks, c, h, u) * np.prod(2 * h))
        assert abs(r["Q"] - exact) <= 1e-13 * max(abs(exact), r["scaleQ"]), (ks, r["Q"], exact)


def test_tensor_error_and_axis_on_x14():
    d = 3
    c = np.array([0.3, -0.2, 0.1])
    h = np.array([0.25, 0.5, 0.125])
    for axis in range(d):
        ks = [0] * d
        ks[axis] = 14
        r = O.rule(O.MONOMIAL, _monomial_params(ks, c), c, h, rule_id=GK)
        vol = float(np.prod(2 * h))
        n = 7
        rem = (mp.mpf(2) ** (2 * n + 1) * mp.factorial(n) ** 4 /
               ((2 * n + 1) * mp.factorial(2 * n) ** 3)) * mp.factorial(2 * n) / 2
        want = float(vol * mp.mpf(h[axis]) ** 14 * rem)
        assert abs(r["err"] - want) <= 2e-12 * want
        assert r["axis"] == axis
        others = [r["D"][j] for j in range(d) if j != axis]
        assert max(others) <= 1e-13 * r["scaleQ"]
        assert abs(r["D"][axis] - want) <= 2e-12 * want


@pytest.mark.parametrize("fam", [1, 2, 4, 5])
def test_tensor_rule_brute_force_50_digits(fam):
    d = 2
    rng = np.random.default_rng(fam)
    p = np.concatenate([rng.uniform(0.5, 4, d), rng.uniform(0, 1, d)])
    c = np.array([0.4, 0.6])
    h = np.array([0.25, 0.125])
    x, wk, wg = O.gk_constants()
    sk = mp.mpf(0)
    sg = mp.mpf(0)
    for k0 in range(15):
        for k1 in range(15):
            # the same (rounded) node coordinates; f and the sums in 50 digits
            xx = [_fma(x[k0], h[0], c[0]), _fma(x[k1], h[1], c[1])]
            a, u = [mp.mpf(v) for v in p[:d]], [mp.mpf(v) for v in p[d:]]
            X = [mp.mpf(v) for v in xx]
            if fam == 1:
                fv = mp.cos(mp.mpf(6.283185307179586476925286766559 * p[d]) + a[0] * X[0] + a[1] * X[1])
            elif fam == 2:
                fv = 1 / ((1 / a[0] ** 2 + (X[0] - u[0]) ** 2) * (1 / a[1] ** 2 + (X[1] - u[1]) ** 2))
            elif fam == 4:
                fv = mp.exp(-((a[0] * (X[0] - u[0])) ** 2 + (a[1] * (X[1] - u[1])) ** 2))
            else:
                fv = mp.exp(-(a[0] * abs(X[0] - u[0]) + a[1] * abs(X[1] - u[1])))
            sk += mp.mpf(wk[k0]) * mp.mpf(wk[k1]) * fv
            sg += mp.mpf(wg[k0]) * mp.mpf(wg[k1]) * fv
    vol = mp.mpf(float(np.prod(2 * h)))
    r = O.rule(fam, p, c, h, rule_id=GK)
    assert abs(mp.mpf(r["Q"]) - vol * sk) <= 4e-16 * r["scaleQ"]
    assert abs(mp.mpf(r["err"]) - vol * abs(sk - sg)) <= 4e-16 * r["scaleE"]


def test_node_count_and_rejects_high_dimension():
    assert [O.gk_num_nodes(d) for d in (2, 3, 6)] == [225, 3375, 15 ** 6]
    with pytest.raises(ValueError):
        O.Run(4, np.ones(14), np.zeros(7), np.ones(7), 1e-6, rule_id=GK)


@pytest.mark.parametrize("k", [1, 3, 4, 7])
def test_adaptive_gk_converges_to_paper_closed_forms_d3(k):
    d = 3
    fam, a, u = CF.paper_params(k, d)
    p = np.concatenate([a, u])
    exact = float(CF.exact(fam, a, u))
    res = O.integrate(fam, p, np.zeros(d), np.ones(d), 1e-10, max_regions=1 << 16, init_log2=3,
                      rule_id=GK)
    assert res["status"] == O.OK
    assert abs(res["I"] - exact) <= 1e-9 * abs(exact), (res["I"], exact)


def test_gk_frozen_tree_volume_and_determinism():
    d = 3
    fam, a, u = CF.paper_params(4, d)
    p = np.concatenate([a, u])
    runs = []
    for _ in range(2):
        r = O.Run(fam, p, np.zeros(d), np.ones(d), 1e-9, max_regions=1 << 16, init_log2=3,
                  keep_leaves=True, rule_id=GK)
        r.run()
        res = r.result()
        c, h, lvl = r.leaves()
        assert sum(2.0 ** -int(l) for l in lvl) == 1.0
        runs.append((res["I"], res["E"], res["regions"]))
    assert runs[0] == runs[1]
