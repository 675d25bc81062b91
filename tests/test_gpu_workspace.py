"""Caller-owned workspace (gm_set_workspace): a torch uint8 tensor registered
as the device scratch of gm_integrate, gm_integrate_grad's forward store and
gm_integrate_batch gives the same results as library-owned memory, writes
nothing past the registered size, and a buffer one byte too small is refused
with GM_ENOMEM before anything runs (outputs untouched)."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from paper_2511_01573_amd import gm, workloads as W

pytestmark = pytest.mark.gpu

GUARD = 4096


def _case():
    d = 4
    p = W.family_params(W.GAUSSIAN, d, seed=77)
    lo, hi = W.unit_box(d)
    return d, p, lo, hi


def _registered(nbytes):
    import torch
    buf = torch.empty(nbytes + GUARD, dtype=torch.uint8, device="cuda")
    buf[nbytes:].fill_(0xA5)
    gm.set_workspace(buf[:nbytes])
    return buf


def test_workspace_gives_the_same_run_and_stays_inside():
    import torch
    d, p, lo, hi = _case()
    cap = 1 << 16
    gm.set_workspace(None)
    ref = gm.integrate(W.GAUSSIAN, p, lo, hi, 1e-7, 1e-16, cap)
    ref_stats = gm.last_stats()
    need = gm.workspace_bytes(d, cap, 0)
    assert need > 0
    buf = _registered(need)
    try:
        print("case workspace integrate", flush=True)
        got = gm.integrate(W.GAUSSIAN, p, lo, hi, 1e-7, 1e-16, cap)
        stats = gm.last_stats()
        gI, gE, gg, gst = gm.integrate_grad(W.GAUSSIAN, p, lo, hi, 1e-7, 1e-16, cap)
    finally:
        gm.set_workspace(None)
    torch.cuda.synchronize()
    assert got == ref
    assert stats["regions_evaluated"] == ref_stats["regions_evaluated"]
    assert (gI, gE, gst) == ref
    assert bool((buf[need:] == 0xA5).all())
    # library-owned memory again after deregistration
    assert gm.integrate(W.GAUSSIAN, p, lo, hi, 1e-7, 1e-16, cap) == ref


def test_workspace_too_small_is_refused_with_enomem():
    d, p, lo, hi = _case()
    cap = 1 << 16
    need = gm.workspace_bytes(d, cap, 0)
    buf = _registered(need - 1)
    try:
        L = gm.lib()
        est = C.c_double(-7.0)
        err = C.c_double(-7.0)
        pa = np.ascontiguousarray(p)
        la = np.ascontiguousarray(lo)
        ha = np.ascontiguousarray(hi)
        P = C.POINTER(C.c_double)
        print("case workspace too small", flush=True)
        rc = L.gm_integrate(W.GAUSSIAN, pa.ctypes.data_as(P), d, la.ctypes.data_as(P),
                            ha.ctypes.data_as(P), 1e-7, 1e-16, cap, C.byref(est), C.byref(err),
                            None)
        assert rc == gm.ENOMEM
        assert est.value == -7.0 and err.value == -7.0  # outputs untouched
        with pytest.raises(gm.GMError) as ei:
            gm.integrate(W.GAUSSIAN, p, lo, hi, 1e-7, 1e-16, cap)
        assert ei.value.code == gm.ENOMEM
        # a smaller store fits the same buffer
        I, E, st = gm.integrate(W.GAUSSIAN, p, lo, hi, 1e-3, 1e-16, cap // 2)
        assert st in (gm.OK, gm.MAX_REGIONS)
    finally:
        gm.set_workspace(None)
    del buf


def test_workspace_batch():
    import torch
    rng = np.random.default_rng(3)
    n = 40
    fams, ps, ds, los, his, rts, ats = [], [], [], [], [], [], []
    for i in range(n):
        d = int(rng.integers(3, 8))
        fam = [W.GAUSSIAN, W.OSCILLATORY, W.PRODUCT_PEAK][i % 3]
        fams.append(fam)
        ps.append(W.family_params(fam, d, seed=300 + i, difficulty=0.35 * W.DIFFICULTY_D8[fam]))
        ds.append(d)
        los.append(np.zeros(d))
        his.append(np.ones(d))
        rts.append(10 ** rng.uniform(-7, -4))
        ats.append(1e-16)
    cap = 1 << 20
    args = (fams, ps, ds, los, his, rts, ats, cap)
    gm.set_workspace(None)
    rc0, e0, r0, s0 = gm.integrate_batch(*args)
    need = gm.workspace_bytes(max(ds), cap, 2)
    buf = _registered(need)
    try:
        print("case workspace batch", flush=True)
        rc1, e1, r1, s1 = gm.integrate_batch(*args)
    finally:
        gm.set_workspace(None)
    torch.cuda.synchronize()
    assert rc1 == rc0 and np.array_equal(s1, s0)
    assert np.array_equal(e1, e0) and np.array_equal(r1, r0)
    assert bool((buf[need:] == 0xA5).all())
