"""Parity tolerances between the HIP path and the CPU oracle.

Per region (rule value Q and error estimate err of Sec. 2):
  |Q_gpu - Q_oracle|     <= 1e-13 * max(|Q|, scaleQ),  scaleQ = vol * sum_k |w_k| Sabs_k
  |err_gpu - err_oracle| <= 1e-13 * scaleE,            scaleE = vol * sum_k |w_k - v_k| Sabs_k
(err is a cancelling difference, so its agreement is stated against the
magnitude of the terms it cancels, not against itself.)  Split axis: equal.
Final estimate I: 1e-12 relative.
"""
import numpy as np

Q_TOL = 1e-13
I_TOL = 1e-12


def assert_regions_match(gq, ge, gax, ref, label=""):
    q, e, sq, se = ref["Q"], ref["err"], ref["scaleQ"], ref["scaleE"]
    dq = np.abs(gq - q)
    lim_q = Q_TOL * np.maximum(np.abs(q), sq)
    bad = np.nonzero(~(dq <= lim_q))[0]
    assert bad.size == 0, (label, "Q", bad[:5], gq[bad[:5]], q[bad[:5]])
    de = np.abs(ge - e)
    lim_e = Q_TOL * se
    bad = np.nonzero(~(de <= lim_e))[0]
    assert bad.size == 0, (label, "err", bad[:5], ge[bad[:5]], e[bad[:5]])
    gaxis = gax & 0x7F
    ggeo = (gax >> 7) & 1
    bad = np.nonzero(gaxis != ref["axis"])[0]
    assert bad.size == 0, (label, "axis", bad[:5], gaxis[bad[:5]], ref["axis"][bad[:5]])
    bad = np.nonzero(ggeo != ref["geo"])[0]
    assert bad.size == 0, (label, "geo", bad[:5])
