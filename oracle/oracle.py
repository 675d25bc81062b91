"""ctypes binding for the serial FP64 CPU oracle (``oracle/gm_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.  The
oracle follows Sec. 2 (rule, estimator, split axis), Sec. 3 (breadth-first
loop) and Sec. 4 (test integrands, stopping rule) of arXiv 2511.01573; the
readings taken where the paper is silent are documented in ``gm_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
# the same source built with -fopenmp: the CPU baseline's all-cores variant
# (per-region evaluation in parallel, every reduction serial: the same bits)
LIB_OMP_PATH = os.path.join(HERE, "liboracle_omp.so")
SRC = os.path.join(HERE, "gm_oracle.c")

OSCILLATORY, PRODUCT_PEAK, CORNER_PEAK, GAUSSIAN, C0, DISCONTINUOUS, POLY = range(1, 8)
FAMILY_NAMES = {
    OSCILLATORY: "oscillatory",
    PRODUCT_PEAK: "product_peak",
    CORNER_PEAK: "corner_peak",
    GAUSSIAN: "gaussian",
    C0: "c0",
    DISCONTINUOUS: "discontinuous",
    POLY: "poly",
}
MONOMIAL = 99  # oracle-only test family: prod (x_j - u_j)^(int a_j)
OK, MAX_REGIONS, MAX_ITERS, PRECISION_LIMIT, NONFINITE = 0, 1, 2, 3, 4
EINVAL, ENOMEM = -1, -2
RUNNING = 100
STAT_NAMES = ["iterations", "regions", "evals", "active", "finished", "max_active",
              "geometry", "roundoff"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O3, -ffp-contract=off: no implicit FMA),
    serial and with OpenMP."""
    hdr = os.path.join(HERE, "gm_oracle.h")
    newest = max(os.path.getmtime(SRC), os.path.getmtime(hdr))
    for path, extra in ((LIB_PATH, []), (LIB_OMP_PATH, ["-fopenmp"])):
        if force or not os.path.exists(path) or os.path.getmtime(path) < newest:
            cmd = ["gcc", "-O3", "-std=c11", "-Wall", "-ffp-contract=off", "-fPIC", "-shared"] + \
                extra + ["-o", path, SRC, "-lm"]
            subprocess.check_call(cmd)
    return LIB_PATH


_lib = None
_libs = {}


def use_openmp(on: bool) -> int:
    """Route every following oracle call through the OpenMP build (on) or the
    serial build (off); returns the thread count of the selected build."""
    global _lib
    _lib = _load(LIB_OMP_PATH if on else LIB_PATH)
    return int(_lib.gmo_threads())


def lib():
    global _lib
    if _lib is None:
        _lib = _load(LIB_PATH)
    return _lib


def _load(path):
    if path not in _libs:
        build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        i32p = C.POINTER(C.c_int32)
        i64p = C.POINTER(C.c_int64)
        L.gmo_num_nodes.restype = C.c_int64
        L.gmo_num_nodes.argtypes = [C.c_int]
        L.gmo_constants.argtypes = [C.c_int, dp, dp, dp, dp]
        L.gmo_nodes.argtypes = [C.c_int, dp, dp, dp, ip]
        L.gmo_f.restype = C.c_double
        L.gmo_f.argtypes = [C.c_int, C.c_int, dp, dp]
        L.gmo_df.restype = C.c_double
        L.gmo_df.argtypes = [C.c_int, C.c_int, dp, dp, dp]
        L.gmo_rule.restype = C.c_int
        L.gmo_rule.argtypes = [C.c_int, C.c_int, dp, dp, dp, C.c_int, C.c_double, dp]
        L.gmo_create.restype = C.c_void_p
        L.gmo_create.argtypes = [C.c_int, C.c_int, dp, dp, dp, C.c_double, C.c_double, C.c_int64,
                                 C.c_int, C.c_int, C.c_int, ip]
        L.gmo_step.restype = C.c_int
        L.gmo_step.argtypes = [C.c_void_p]
        L.gmo_run_to_end.restype = C.c_int
        L.gmo_run_to_end.argtypes = [C.c_void_p]
        L.gmo_result.argtypes = [C.c_void_p, dp, dp, ip, i64p]
        L.gmo_escale.restype = C.c_double
        L.gmo_escale.argtypes = [C.c_void_p]
        L.gmo_active_count.restype = C.c_int64
        L.gmo_active_count.argtypes = [C.c_void_p]
        L.gmo_get_active.argtypes = [C.c_void_p, dp, dp, i32p, dp, dp, i32p]
        L.gmo_leaf_count.restype = C.c_int64
        L.gmo_leaf_count.argtypes = [C.c_void_p]
        L.gmo_get_leaves.argtypes = [C.c_void_p, dp, dp, i32p]
        L.gmo_trace_len.restype = C.c_int64
        L.gmo_trace_len.argtypes = [C.c_void_p]
        L.gmo_get_trace.argtypes = [C.c_void_p, i64p, dp]
        L.gmo_free.argtypes = [C.c_void_p]
        L.gmo_quad_leaves.restype = C.c_int
        L.gmo_quad_leaves.argtypes = [C.c_int, C.c_int, dp, C.c_int64, dp, dp, i32p, C.c_double, dp]
        L.gmo_grad_leaves.restype = C.c_int
        L.gmo_grad_leaves.argtypes = [C.c_int, C.c_int, dp, C.c_int64, dp, dp, i32p, C.c_double,
                                      dp]
        L.gmo_quad_leaves_rule.restype = C.c_int
        L.gmo_quad_leaves_rule.argtypes = [C.c_int, C.c_int, dp, C.c_int64, dp, dp, i32p,
                                           C.c_double, C.c_int, dp]
        L.gmo_grad_leaves_rule.restype = C.c_int
        L.gmo_grad_leaves_rule.argtypes = [C.c_int, C.c_int, dp, C.c_int64, dp, dp, i32p,
                                           C.c_double, C.c_int, dp]
        L.gmo_gk_constants.argtypes = [dp, dp, dp]
        L.gmo_gk_num_nodes.restype = C.c_int64
        L.gmo_gk_num_nodes.argtypes = [C.c_int]
        L.gmo_rule_gk.restype = C.c_int
        L.gmo_rule_gk.argtypes = [C.c_int, C.c_int, dp, dp, dp, C.c_int, C.c_double, dp]
        L.gmo_set_rule.restype = C.c_int
        L.gmo_set_rule.argtypes = [C.c_void_p, C.c_int]
        L.gmo_set_err_model.restype = C.c_int
        L.gmo_set_err_model.argtypes = [C.c_void_p, C.c_int]
        L.gmo_num_nodes9.restype = C.c_int64
        L.gmo_num_nodes9.argtypes = [C.c_int]
        L.gmo_constants9.argtypes = [C.c_int, dp, dp, dp]
        L.gmo_nodes9.argtypes = [C.c_int, dp, dp, dp, ip]
        L.gmo_rule9.restype = C.c_int
        L.gmo_rule9.argtypes = [C.c_int, C.c_int, dp, dp, dp, C.c_int, C.c_double, C.c_int, dp]
        L.gmo_set_prune.restype = C.c_int
        L.gmo_set_prune.argtypes = [C.c_void_p, C.c_int]
        L.gmo_pruned.restype = C.c_int
        L.gmo_pruned.argtypes = [C.c_void_p]
        L.gmo_integrate_batch_rule.restype = C.c_int
        L.gmo_integrate_batch_rule.argtypes = [C.c_int, ip, dp, ip, dp, dp, dp, dp, C.c_int64,
                                               C.c_int, C.c_int, C.c_int, C.c_int, dp, dp, ip,
                                               i64p]
        L.gmo_integrate_batch.restype = C.c_int
        L.gmo_integrate_batch.argtypes = [C.c_int, ip, dp, ip, dp, dp, dp, dp, C.c_int64, C.c_int,
                                          C.c_int, dp, dp, ip, i64p]
        L.gmo_threads.restype = C.c_int
        L.gmo_threads.argtypes = []
        _libs[path] = L
    return _libs[path]


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def num_nodes(d: int) -> int:
    return int(lib().gmo_num_nodes(d))


def constants(d: int):
    """(lam, w, v, e) for classes 1..5 as float64 arrays of length 5."""
    lam, w, v, e = (np.zeros(5) for _ in range(4))
    lib().gmo_constants(d, _d(lam)[1], _d(w)[1], _d(v)[1], _d(e)[1])
    return lam, w, v, e


def nodes(d: int, c, h):
    """All nodes of region (c, h) in the oracle's visit order: (x[N, d], cls[N])."""
    n = num_nodes(d)
    x = np.zeros((n, d))
    cls = np.zeros(n, dtype=np.intc)
    c, cp = _d(c)
    h, hp = _d(h)
    lib().gmo_nodes(d, cp, hp, x.ctypes.data_as(C.POINTER(C.c_double)),
                    cls.ctypes.data_as(C.POINTER(C.c_int)))
    return x, cls


def f(fam: int, params, x) -> float:
    x = np.asarray(x, dtype=np.float64)
    d = x.shape[-1]
    p, pp = _d(params)
    assert p.size == 2 * d
    xx, xp = _d(x)
    return float(lib().gmo_f(fam, d, pp, xp))


def df(fam: int, params, x):
    x = np.asarray(x, dtype=np.float64)
    d = x.shape[-1]
    p, pp = _d(params)
    xx, xp = _d(x)
    out = np.zeros(2 * d)
    val = lib().gmo_df(fam, d, pp, xp, _d(out)[1])
    return float(val), out


GENZ_MALIK, GAUSS_KRONROD, DEGREE9 = 0, 1, 2


def num_nodes9(d: int) -> int:
    return int(lib().gmo_num_nodes9(d))


def constants9(d: int):
    """(lam[6], w[8], e[8]) of the degree-9 rule: lam = (0, l2, l3, l4, l5, l6),
    w the weights of classes 1..8, e = w minus the embedded degree-7 weights."""
    lam, w, e = np.zeros(6), np.zeros(8), np.zeros(8)
    lib().gmo_constants9(d, _d(lam)[1], _d(w)[1], _d(e)[1])
    return lam, w, e


def nodes9(d: int, c, h):
    """All nodes of the degree-9 rule on region (c, h) in visit order."""
    n = num_nodes9(d)
    x = np.zeros((n, d))
    cls = np.zeros(n, dtype=np.intc)
    c, cp = _d(c)
    h, hp = _d(h)
    lib().gmo_nodes9(d, cp, hp, x.ctypes.data_as(C.POINTER(C.c_double)),
                     cls.ctypes.data_as(C.POINTER(C.c_int)))
    return x, cls


def gk_constants():
    """(x[15], wk[15], wg[15]) of the tensor-product Gauss-Kronrod rule."""
    x, wk, wg = np.zeros(15), np.zeros(15), np.zeros(15)
    lib().gmo_gk_constants(_d(x)[1], _d(wk)[1], _d(wg)[1])
    return x, wk, wg


def gk_num_nodes(d: int) -> int:
    return int(lib().gmo_gk_num_nodes(d))


def _rule_fn(rule_id: int, err_model: int = 0):
    if rule_id == DEGREE9:
        return lambda fam, d, pp, cp, hp, lvl, vo, op: lib().gmo_rule9(fam, d, pp, cp, hp, lvl, vo,
                                                                       int(err_model), op)
    return lib().gmo_rule_gk if rule_id == GAUSS_KRONROD else lib().gmo_rule


def rule(fam: int, params, c, h, lvl: int = 0, vol_omega: float | None = None, rule_id: int = 0,
         err_model: int = 0):
    """One region (c, h, lvl); returns a dict with Q, err, axis, geo, scales, S, Sabs, D
    (Gauss-Kronrod rule: S[0], S[1] = K and G sums, D = one-axis estimates; degree-9
    rule: eight class sums and also Q7 and the null-rule values n1 = vol |Q9 - Q7|,
    n2 = vol |Q7 - Q5|, n3 = vol |Q5 - Q3|)."""
    c, cp = _d(c)
    h, hp = _d(h)
    d = c.size
    p, pp = _d(params)
    if vol_omega is None:
        # region volume = prod 2h when lvl == 0
        vol_omega = float(np.prod(2.0 * h))
    out = np.zeros(16 + 32)
    rc = _rule_fn(rule_id, err_model)(fam, d, pp, cp, hp, int(lvl), float(vol_omega), _d(out)[1])
    res = {"status": rc, "Q": out[0], "err": out[1], "axis": int(out[2]), "geo": int(out[3]),
           "scaleQ": out[4], "scaleE": out[5]}
    if rule_id == DEGREE9:
        res.update({"Q7": out[6], "n1": out[7], "n2": out[8], "n3": out[9], "S": out[10:18].copy(),
                    "Sabs": out[18:26].copy(), "D": out[26:26 + d].copy()})
    else:
        res.update({"S": out[6:11].copy(), "Sabs": out[11:16].copy(), "D": out[16:16 + d].copy()})
    return res


def rule_many(fam: int, params, c, h, lvl, vol_omega: float, rule_id: int = 0, err_model: int = 0):
    """Rule on a list of regions; c, h: [n, d]; returns dict of arrays."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    h = np.ascontiguousarray(h, dtype=np.float64)
    n, d = c.shape
    p, pp = _d(params)
    out = np.zeros(16 + 32)
    op = _d(out)[1]
    res = {k: np.zeros(n) for k in ("Q", "err", "scaleQ", "scaleE")}
    res["axis"] = np.zeros(n, dtype=np.int32)
    res["geo"] = np.zeros(n, dtype=np.int32)
    res["status"] = np.zeros(n, dtype=np.int32)
    fn = _rule_fn(rule_id, err_model)
    for i in range(n):
        ci = c[i]
        hi = h[i]
        rc = fn(fam, d, pp, ci.ctypes.data_as(C.POINTER(C.c_double)),
                        hi.ctypes.data_as(C.POINTER(C.c_double)), int(lvl[i]), float(vol_omega), op)
        res["status"][i] = rc
        res["Q"][i] = out[0]
        res["err"][i] = out[1]
        res["axis"][i] = int(out[2])
        res["geo"][i] = int(out[3])
        res["scaleQ"][i] = out[4]
        res["scaleE"][i] = out[5]
    return res


class Run:
    """Handle on one adaptive run of the oracle (Sec. 3 loop)."""

    def __init__(self, fam, params, lo, hi, rel_tol, abs_tol=1e-16, max_regions=1 << 20,
                 init_log2=12, max_iters=10000, keep_leaves=False, rule_id=0, prune=False,
                 err_model=0):
        self.fam = fam
        self.params, pp = _d(params)
        self.lo, lp = _d(lo)
        self.hi, hp = _d(hi)
        self.d = self.lo.size
        st = C.c_int(0)
        self.h = lib().gmo_create(fam, self.d, pp, lp, hp, float(rel_tol), float(abs_tol),
                                  int(max_regions), int(init_log2), int(max_iters),
                                  1 if keep_leaves else 0, C.byref(st))
        self.create_status = st.value
        if not self.h:
            raise ValueError(f"oracle rejected arguments (status {st.value})")
        if rule_id and lib().gmo_set_rule(self.h, int(rule_id)) != OK:
            raise ValueError(f"oracle rejected rule {rule_id} at d = {self.d}")
        if err_model and lib().gmo_set_err_model(self.h, int(err_model)) != OK:
            raise ValueError(f"oracle rejected error model {err_model}")
        if prune:
            lib().gmo_set_prune(self.h, 1)
        self.vol_omega = float(np.prod(self.hi - self.lo)) if self.d else 1.0
        v = 1.0
        for j in range(self.d):
            v = v * (self.hi[j] - self.lo[j])
        self.vol_omega = v

    def step(self) -> int:
        return int(lib().gmo_step(self.h))

    def run(self) -> int:
        return int(lib().gmo_run_to_end(self.h))

    def result(self):
        I = C.c_double()
        E = C.c_double()
        st = C.c_int()
        stats = np.zeros(8, dtype=np.int64)
        lib().gmo_result(self.h, C.byref(I), C.byref(E), C.byref(st),
                         stats.ctypes.data_as(C.POINTER(C.c_int64)))
        out = {"I": I.value, "E": E.value, "status": st.value,
               "escale": float(lib().gmo_escale(self.h)), "pruned": bool(lib().gmo_pruned(self.h))}
        out.update({k: int(v) for k, v in zip(STAT_NAMES, stats)})
        return out

    def active(self):
        n = int(lib().gmo_active_count(self.h))
        d = self.d
        c = np.zeros((n, d))
        h = np.zeros((n, d))
        lvl = np.zeros(n, dtype=np.int32)
        Q = np.zeros(n)
        err = np.zeros(n)
        axis = np.zeros(n, dtype=np.int32)
        P = C.POINTER(C.c_double)
        lib().gmo_get_active(self.h, c.ctypes.data_as(P), h.ctypes.data_as(P),
                             lvl.ctypes.data_as(C.POINTER(C.c_int32)), Q.ctypes.data_as(P),
                             err.ctypes.data_as(P), axis.ctypes.data_as(C.POINTER(C.c_int32)))
        return {"c": c, "h": h, "lvl": lvl, "Q": Q, "err": err, "axis": axis}

    def leaves(self):
        n = int(lib().gmo_leaf_count(self.h))
        d = self.d
        c = np.zeros((n, d))
        h = np.zeros((n, d))
        lvl = np.zeros(n, dtype=np.int32)
        P = C.POINTER(C.c_double)
        lib().gmo_get_leaves(self.h, c.ctypes.data_as(P), h.ctypes.data_as(P),
                             lvl.ctypes.data_as(C.POINTER(C.c_int32)))
        return c, h, lvl

    def trace(self):
        n = int(lib().gmo_trace_len(self.h))
        counts = np.zeros((n, 2), dtype=np.int64)
        IE = np.zeros((n, 2))
        lib().gmo_get_trace(self.h, counts.ctypes.data_as(C.POINTER(C.c_int64)),
                            IE.ctypes.data_as(C.POINTER(C.c_double)))
        return counts, IE

    def __del__(self):
        if getattr(self, "h", None):
            lib().gmo_free(self.h)
            self.h = None


def integrate(fam, params, lo, hi, rel_tol, abs_tol=1e-16, max_regions=1 << 20, init_log2=12,
              max_iters=10000, rule_id=0, prune=False, err_model=0):
    r = Run(fam, params, lo, hi, rel_tol, abs_tol, max_regions, init_log2, max_iters,
            rule_id=rule_id, prune=prune, err_model=err_model)
    r.run()
    return r.result()


def quad_leaves(fam, params, c, h, lvl, vol_omega, rule_id=0):
    c, cp = _d(c)
    h, hp = _d(h)
    lvl, lp = _i32(lvl)
    p, pp = _d(params)
    n, d = c.shape
    out = C.c_double()
    rc = lib().gmo_quad_leaves_rule(fam, d, pp, n, cp, hp, lp, float(vol_omega), int(rule_id),
                                    C.byref(out))
    return out.value, rc


def grad_leaves(fam, params, c, h, lvl, vol_omega, rule_id=0):
    c, cp = _d(c)
    h, hp = _d(h)
    lvl, lp = _i32(lvl)
    p, pp = _d(params)
    n, d = c.shape
    out = np.zeros(2 * d)
    rc = lib().gmo_grad_leaves_rule(fam, d, pp, n, cp, hp, lp, float(vol_omega), int(rule_id),
                                    _d(out)[1])
    if rc != OK:
        raise ValueError(f"oracle rejected rule {rule_id}")
    return out


def integrate_grad(fam, params, lo, hi, rel_tol, abs_tol=1e-16, max_regions=1 << 20,
                   init_log2=12, max_iters=10000, rule_id=0, err_model=0):
    """Forward run with leaf retention, then the fixed-tree gradient."""
    r = Run(fam, params, lo, hi, rel_tol, abs_tol, max_regions, init_log2, max_iters,
            keep_leaves=True, rule_id=rule_id, err_model=err_model)
    r.run()
    res = r.result()
    c, h, lvl = r.leaves()
    res["grad"] = grad_leaves(fam, params, c, h, lvl, r.vol_omega, rule_id)
    res["leaves"] = (c, h, lvl)
    res["vol_omega"] = r.vol_omega
    return res


def integrate_batch(fams, params_list, ds, los, his, rel_tols, abs_tols, max_regions_total,
                    init_log2=12, max_iters=10000, rule_id=0, err_model=0):
    n = len(fams)
    fam = np.ascontiguousarray(fams, dtype=np.intc)
    d = np.ascontiguousarray(ds, dtype=np.intc)
    params = np.ascontiguousarray(np.concatenate([np.asarray(p, float) for p in params_list]))
    lo = np.ascontiguousarray(np.concatenate([np.asarray(x, float) for x in los]))
    hi = np.ascontiguousarray(np.concatenate([np.asarray(x, float) for x in his]))
    rt = np.ascontiguousarray(rel_tols, dtype=np.float64)
    at = np.ascontiguousarray(abs_tols, dtype=np.float64)
    est = np.zeros(n)
    err = np.zeros(n)
    st = np.zeros(n, dtype=np.intc)
    its = np.zeros(n, dtype=np.int64)
    P = C.POINTER(C.c_double)
    IP = C.POINTER(C.c_int)
    rc = lib().gmo_integrate_batch_rule(n, fam.ctypes.data_as(IP), params.ctypes.data_as(P),
                                        d.ctypes.data_as(IP), lo.ctypes.data_as(P),
                                        hi.ctypes.data_as(P), rt.ctypes.data_as(P),
                                        at.ctypes.data_as(P), int(max_regions_total),
                                        int(init_log2), int(max_iters), int(rule_id),
                                        int(err_model), est.ctypes.data_as(P),
                                        err.ctypes.data_as(P), st.ctypes.data_as(IP),
                                        its.ctypes.data_as(C.POINTER(C.c_int64)))
    return rc, est, err, st, its
