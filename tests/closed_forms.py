"""Closed-form integrals of the test integrands over [0,1]^d (pins for the oracle).

These are the exact values of the Sec. 4 test functions and their seeded
Genz-family generalisations, derived by integrating each formula
analytically; they are independent of the cubature rule.  Evaluated with
mpmath at 40 digits (exact rationals where an alternating sum would cancel).
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import mpmath as mp

mp.mp.dps = 40

OSCILLATORY, PRODUCT_PEAK, CORNER_PEAK, GAUSSIAN, C0, DISCONTINUOUS, POLY = range(1, 8)


def _mpf(x: float):
    return mp.mpf(float(x))


def oscillatory(a, u):
    """int cos(2 pi u_1 + sum a_j x_j) = cos(2 pi u_1 + sum a_j/2) prod 2 sin(a_j/2)/a_j."""
    two_pi_u = _mpf(6.283185307179586476925286766559 * float(u[0]))  # the double the integrand uses
    s = two_pi_u + sum(_mpf(x) / 2 for x in a)
    p = mp.mpf(1)
    for x in a:
        x = _mpf(x)
        p *= 2 * mp.sin(x / 2) / x
    return mp.cos(s) * p


def product_peak(a, u):
    """int prod 1/(a^-2 + (x-u)^2) = prod a [atan(a(1-u)) + atan(a u)]."""
    p = mp.mpf(1)
    for x, y in zip(a, u):
        x, y = _mpf(x), _mpf(y)
        p *= x * (mp.atan(x * (1 - y)) + mp.atan(x * y))
    return p


def corner_peak(a, u=None):
    """int (1 + sum a_j x_j)^-(d+1) = sum_S (-1)^|S| / (1 + sum_S a) / (d! prod a).

    The alternating sum cancels heavily (at d = 16 by ~25 digits), so it is
    formed from the exact subset sums (the a_j are exact binary fractions) with
    mpmath at 120 digits."""
    d = len(a)
    with mp.workdps(120):
        A = [mp.mpf(float(x)) for x in a]
        sums = [(mp.mpf(1), 1)]
        for x in A:
            sums = sums + [(s + x, -sg) for s, sg in sums]
        tot = mp.fsum(sg / s for s, sg in sums)
        den = mp.factorial(d)
        for x in A:
            den *= x
        val = tot / den
    return +val


def gaussian_factor(a, u):
    a, u = _mpf(a), _mpf(u)
    return mp.sqrt(mp.pi) / (2 * a) * (mp.erf(a * (1 - u)) + mp.erf(a * u))


def gaussian(a, u):
    """int exp(-sum a^2 (x-u)^2) = prod sqrt(pi)/(2a) [erf(a(1-u)) + erf(a u)]."""
    p = mp.mpf(1)
    for x, y in zip(a, u):
        p *= gaussian_factor(x, y)
    return p


def gaussian_grad(a, u):
    """d/da_j and d/du_j of the Gaussian closed form; returns a list of 2d mpf."""
    d = len(a)
    F = [gaussian_factor(a[j], u[j]) for j in range(d)]
    I = mp.mpf(1)
    for x in F:
        I *= x
    ga, gu = [], []
    for j in range(d):
        aj, uj = _mpf(a[j]), _mpf(u[j])
        e0 = mp.exp(-(aj * uj) ** 2)
        e1 = mp.exp(-(aj * (1 - uj)) ** 2)
        dF_du = e0 - e1
        dF_da = -F[j] / aj + ((1 - uj) * e1 + uj * e0) / aj
        ga.append(I / F[j] * dF_da)
        gu.append(I / F[j] * dF_du)
    return ga + gu


def c0(a, u):
    """int exp(-sum a|x-u|) = prod (2 - e^{-a u} - e^{-a(1-u)})/a."""
    p = mp.mpf(1)
    for x, y in zip(a, u):
        x, y = _mpf(x), _mpf(y)
        p *= (2 - mp.exp(-x * y) - mp.exp(-x * (1 - y))) / x
    return p


def c0_grad(a, u):
    """d/da_j and d/du_j of the C0 closed form (2d mpf): with the factor
    F_j = (2 - e^{-a u} - e^{-a(1-u)})/a,
      dF/da = (u e^{-a u} + (1-u) e^{-a(1-u)})/a - F/a,
      dF/du = e^{-a u} - e^{-a(1-u)},
    and dI/dtheta_j = I / F_j * dF_j/dtheta_j."""
    d = len(a)
    fs, da, du = [], [], []
    for x, y in zip(a, u):
        x, y = _mpf(x), _mpf(y)
        e0, e1 = mp.exp(-x * y), mp.exp(-x * (1 - y))
        F = (2 - e0 - e1) / x
        fs.append(F)
        da.append((y * e0 + (1 - y) * e1) / x - F / x)
        du.append(e0 - e1)
    I = mp.mpf(1)
    for F in fs:
        I *= F
    return [I / fs[j] * da[j] for j in range(d)] + [I / fs[j] * du[j] for j in range(d)]


def discontinuous(a, u):
    """f = 0 if x_j > u_j for ANY j, else exp(sum a x): prod (e^{a b} - 1)/a, b = clip(u, 0, 1)."""
    p = mp.mpf(1)
    for x, y in zip(a, u):
        x = _mpf(x)
        b = min(max(_mpf(y), mp.mpf(0)), mp.mpf(1))
        p *= (mp.exp(x * b) - 1) / x
    return p


def poly_f7(d: int):
    """int (sum x^2)^11 = sum_{|k|=11} 11!/prod k_i! prod 1/(2k_i+1), exact rational."""
    n = 11
    tot = Fraction(0)

    def compositions(n, d):
        if d == 1:
            yield (n,)
            return
        for k in range(n + 1):
            for rest in compositions(n - k, d - 1):
                yield (k,) + rest

    for ks in compositions(n, d):
        term = Fraction(math.factorial(n))
        for k in ks:
            term /= math.factorial(k) * (2 * k + 1)
        tot += term
    return mp.mpf(tot.numerator) / tot.denominator


def exact(fam: int, a, u):
    d = len(a)
    if fam == OSCILLATORY:
        return oscillatory(a, u)
    if fam == PRODUCT_PEAK:
        return product_peak(a, u)
    if fam == CORNER_PEAK:
        return corner_peak(a)
    if fam == GAUSSIAN:
        return gaussian(a, u)
    if fam == C0:
        return c0(a, u)
    if fam == DISCONTINUOUS:
        return discontinuous(a, u)
    if fam == POLY:
        return poly_f7(d)
    raise ValueError(fam)


def paper_params(k: int, d: int):
    """Parameters that turn the seeded families into the paper's f1..f7 (Sec. 4)."""
    idx = list(range(1, d + 1))
    if k == 1:
        return OSCILLATORY, [float(i) for i in idx], [0.0] * d
    if k == 2:
        return PRODUCT_PEAK, [50.0] * d, [0.5] * d
    if k == 3:
        return CORNER_PEAK, [float(i) for i in idx], [0.0] * d
    if k == 4:
        return GAUSSIAN, [25.0] * d, [0.5] * d
    if k == 5:
        return C0, [10.0] * d, [0.5] * d
    if k == 6:
        return DISCONTINUOUS, [float(i + 4) for i in idx], [(3 + i) / 10.0 for i in idx]
    if k == 7:
        return POLY, [0.0] * d, [0.0] * d
    raise ValueError(k)


def monomial_moment_box(exps, c, h, u):
    """Exact mean of prod (x_j - u_j)^k_j over the box prod [c_j - h_j, c_j + h_j]."""
    m = Fraction(1)
    for k, cj, hj, uj in zip(exps, c, h, u):
        lo = Fraction(cj) - Fraction(hj) - Fraction(uj)
        hi = Fraction(cj) + Fraction(hj) - Fraction(uj)
        m *= (hi ** (k + 1) - lo ** (k + 1)) / (k + 1) / (hi - lo)
    return m


def all_exponents(d: int, deg: int):
    for ks in itertools.product(range(deg + 1), repeat=d):
        if sum(ks) == deg:
            yield ks
