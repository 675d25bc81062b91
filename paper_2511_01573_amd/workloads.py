"""Seeded synthetic inputs (integrand parameters, boxes, tolerances).

This module holds no cubature arithmetic: it only draws parameters with numpy's
PCG64 generator and rescales them, so the HIP path and the CPU oracle receive
bit-identical inputs.  The workloads follow the paper's test-function suite
(arXiv 2511.01573, Sec. 4: oscillatory, product peak, corner peak, Gaussian,
C0 and discontinuous Genz-type families on [0,1]^d) with seeded parameters
standing in for the fixed parameters of the paper's f1..f6.
"""
from __future__ import annotations

import numpy as np

OSCILLATORY, PRODUCT_PEAK, CORNER_PEAK, GAUSSIAN, C0, DISCONTINUOUS, POLY_F7 = range(1, 8)
SIX_FAMILIES = [OSCILLATORY, PRODUCT_PEAK, CORNER_PEAK, GAUSSIAN, C0, DISCONTINUOUS]
NAMES = {1: "oscillatory", 2: "product_peak", 3: "corner_peak", 4: "gaussian", 5: "c0",
         6: "discontinuous", 7: "poly_f7"}

# Sum of a_j per family at d = 8 ("difficulty").  Calibrated once on the CPU
# oracle so that rel_tol = 1e-5 needs between 1e4 and 1e6 evaluated regions,
# then frozen.
DIFFICULTY_D8 = {OSCILLATORY: 9.0, PRODUCT_PEAK: 15.0, CORNER_PEAK: 2.0, GAUSSIAN: 13.0,
                 C0: 4.0, DISCONTINUOUS: 10.0}
# Batch difficulty: sum(a) = BATCH_SCALE * b_family * d / 8.  At 0.35 each of
# the 4096 integrals converges on its own below 2^26 regions (at 0.5 five
# product-peak items at d = 9, 10 and rel_tol < 1e-6 do not) and the
# lock-step batch fits a shared store of 2^28 regions.
BATCH_SCALE = 0.35
# Number of leading coordinates that carry a discontinuity in the seeded
# discontinuous family; the others get u_j = 1 (no cut inside [0,1]).
DISC_CUT_DIMS = 2


def unit_box(d: int):
    return np.zeros(d), np.ones(d)


def family_params(fam: int, d: int, seed: int, difficulty: float | None = None):
    """a ~ U(0,1) rescaled to sum(a) = difficulty, then u ~ U(0,1), in that order."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 1.0, d)
    u = rng.uniform(0.0, 1.0, d)
    if fam != POLY_F7:
        b = DIFFICULTY_D8[fam] if difficulty is None else difficulty
        a = a * (b / a.sum())
    if fam == DISCONTINUOUS:
        # cuts inside [0.3, 1]: a cut near 0 leaves a sliver of support that no
        # node of the initial partition sees
        u = 0.3 + 0.7 * u
        u[DISC_CUT_DIMS:] = 1.0
    return np.concatenate([a, u])


def config1():
    """Gaussian d = 3, a_j = 5, u_j = 1/2 on [0,1]^3, rel_tol 1e-6, 1e5 regions."""
    d = 3
    return dict(family=GAUSSIAN, params=np.concatenate([np.full(d, 5.0), np.full(d, 0.5)]),
                lo=np.zeros(d), hi=np.ones(d), rel_tol=1e-6, abs_tol=1e-16, max_regions=100000)


def config2(taus=(1e-3, 1e-5, 1e-7), reps=1, max_regions=1 << 24):
    """d = 8, six families x tolerances; seed = 1000 * family + rep."""
    d = 8
    out = []
    for fam in SIX_FAMILIES:
        for rep in range(reps):
            p = family_params(fam, d, 1000 * fam + rep)
            for tau in taus:
                out.append(dict(family=fam, params=p, lo=np.zeros(d), hi=np.ones(d), rel_tol=tau,
                                abs_tol=1e-16, max_regions=max_regions,
                                name=f"{NAMES[fam]}_d8_r{rep}_tau{tau:g}"))
    return out


# Sum of a_j of the d = 12 / 16 cases at rel_tol 1e-4, calibrated once on the
# GPU so that each run converges inside a store of 2^27 regions with about
# 1e8 regions at its largest (d = 12: corner peak 2.2e8 regions evaluated,
# 7.9e7 active at the peak; product peak 1.3e8 / 4.3e7; d = 16: corner peak
# 1.0e8 / 3.5e7, product peak 5.1e7 / 2.0e7, where 25 no longer fits), then
# frozen.
DIFFICULTY_C3 = {(CORNER_PEAK, 12): 4.0, (PRODUCT_PEAK, 12): 40.0,
                 (CORNER_PEAK, 16): 2.0, (PRODUCT_PEAK, 16): 20.0}


def config3(dims=(12, 16), tau=1e-4, max_regions=1 << 27):
    """d = 12 and 16: corner peak and product peak, seeded as config 2 with
    the sums of a_j of DIFFICULTY_C3 (region store of 2^27 regions)."""
    out = []
    for d in dims:
        for fam in (CORNER_PEAK, PRODUCT_PEAK):
            p = family_params(fam, d, 1000 * fam + d, DIFFICULTY_C3[(fam, d)])
            out.append(dict(family=fam, params=p, lo=np.zeros(d), hi=np.ones(d), rel_tol=tau,
                            abs_tol=1e-16, max_regions=max_regions, name=f"{NAMES[fam]}_d{d}"))
    return out


def config4(n=4096, seed=4096, scale=BATCH_SCALE):
    """Batch: d_i ~ U{3..10}, family ~ U{Gaussian, oscillatory, product peak},
    a, u seeded (sum(a) = scale * b_family * d / 8), rel_tol_i = 10^U(-7, -3)."""
    rng = np.random.default_rng(seed)
    fams, params, ds, los, his, rts, ats = [], [], [], [], [], [], []
    choices = [GAUSSIAN, OSCILLATORY, PRODUCT_PEAK]
    for _ in range(n):
        d = int(rng.integers(3, 11))
        fam = choices[int(rng.integers(0, 3))]
        a = rng.uniform(0.0, 1.0, d)
        u = rng.uniform(0.0, 1.0, d)
        a = a * (scale * DIFFICULTY_D8[fam] * d / 8.0 / a.sum())
        tau = 10.0 ** rng.uniform(-7.0, -3.0)
        fams.append(fam)
        params.append(np.concatenate([a, u]))
        ds.append(d)
        los.append(np.zeros(d))
        his.append(np.ones(d))
        rts.append(tau)
        ats.append(1e-16)
    return dict(families=fams, params=params, ds=ds, los=los, his=his, rel_tols=rts, abs_tols=ats)


def config5():
    """Gradient: d = 8 Gaussian, a_j ~ U(1,5), u_j ~ U(0,1), seed 8, rel_tol 1e-8."""
    d = 8
    rng = np.random.default_rng(8)
    a = rng.uniform(1.0, 5.0, d)
    u = rng.uniform(0.0, 1.0, d)
    return dict(family=GAUSSIAN, params=np.concatenate([a, u]), lo=np.zeros(d), hi=np.ones(d),
                rel_tol=1e-8, abs_tol=1e-16, max_regions=1 << 27)


def random_regions(d: int, n: int, seed: int, lo=None, hi=None):
    """n random dyadic sub-boxes of [lo, hi] (as the adaptive loop produces):
    per axis a level l_j ~ U{0..5} and a cell index k_j ~ U{0..2^l_j - 1}."""
    rng = np.random.default_rng(seed)
    lo = np.zeros(d) if lo is None else np.asarray(lo, float)
    hi = np.ones(d) if hi is None else np.asarray(hi, float)
    levels = rng.integers(0, 6, size=(n, d))
    k = np.floor(rng.uniform(0, 1, size=(n, d)) * (1 << levels)).astype(np.int64)
    half = (hi - lo) * 0.5
    h = np.ldexp(np.broadcast_to(half, (n, d)), -levels)
    c = lo + (2 * k + 1) * h
    lvl = levels.sum(axis=1).astype(np.int32)
    return c, h, lvl
