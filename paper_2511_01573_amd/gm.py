"""Thin ctypes binding of libgm (include/gm.h): argument marshalling only.

Every step of the cubature runs in the HIP kernels behind the C ABI; this
module converts Python/numpy arguments, passes torch's current HIP stream and
turns status codes into results.  It raises if libgm.so is missing: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgm.so")

OSCILLATORY, PRODUCT_PEAK, CORNER_PEAK, GAUSSIAN, C0, DISCONTINUOUS, POLY_F7 = range(1, 8)
FAMILIES = {
    "oscillatory": OSCILLATORY, "product_peak": PRODUCT_PEAK, "corner_peak": CORNER_PEAK,
    "gaussian": GAUSSIAN, "c0": C0, "discontinuous": DISCONTINUOUS, "poly_f7": POLY_F7,
}
OK, MAX_REGIONS, MAX_ITERS, PRECISION_LIMIT, NONFINITE = 0, 1, 2, 3, 4
EINVAL, ENOMEM, EHIP = -1, -2, -3

EXPORTED = [
    "gm_integrate", "gm_integrate_batch", "gm_integrate_grad", "gm_eval_regions",
    "gm_set_workspace", "gm_workspace_bytes", "gm_set_option", "gm_status_string",
    "gm_last_stats", "gm_num_nodes", "gm_last_active", "gm_set_tile", "gm_integrate_noalloc",
]


class GMError(RuntimeError):
    def __init__(self, code: int, text: str):
        super().__init__(f"libgm error {code}: {text}")
        self.code = code


class Stats(C.Structure):
    _fields_ = [
        ("iterations", C.c_int64), ("regions_evaluated", C.c_int64), ("evals", C.c_int64),
        ("max_active", C.c_int64), ("final_active", C.c_int64), ("finished", C.c_int64),
        ("status", C.c_int64), ("lanes_per_region", C.c_int64),
        ("rule_ms", C.c_double), ("reduce_ms", C.c_double), ("classify_ms", C.c_double),
        ("split_ms", C.c_double), ("total_ms", C.c_double), ("rule_launches", C.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libgm.so (built in-tree by paper_2511_01573_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python paper_2511_01573_amd/build.py` (no CPU fallback exists)")
        # One HIP runtime per process: torch ships its own libamdhip64.so.7.  Loading
        # torch first makes libgm bind to that same runtime (same soname), so device
        # pointers and streams are shared; otherwise two HSA runtimes would compete
        # for the device.
        try:
            import torch  # noqa: F401
        except ImportError:  # pragma: no cover - libgm then uses the system runtime
            pass
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        i32p = C.POINTER(C.c_int32)
        L.gm_integrate.restype = C.c_int
        L.gm_integrate.argtypes = [C.c_int, dp, C.c_int, dp, dp, C.c_double, C.c_double,
                                   C.c_int64, dp, dp, C.c_void_p]
        L.gm_integrate_noalloc.restype = C.c_int
        L.gm_integrate_noalloc.argtypes = L.gm_integrate.argtypes
        L.gm_integrate_batch.restype = C.c_int
        L.gm_integrate_batch.argtypes = [C.c_int, ip, dp, ip, dp, dp, dp, dp, C.c_int64, dp, dp,
                                         ip, C.c_void_p]
        L.gm_integrate_grad.restype = C.c_int
        L.gm_integrate_grad.argtypes = [C.c_int, dp, C.c_int, dp, dp, C.c_double, C.c_double,
                                        C.c_int64, dp, dp, dp, C.c_void_p]
        L.gm_eval_regions.restype = C.c_int
        L.gm_eval_regions.argtypes = [C.c_int, dp, C.c_int, dp, dp, C.c_int64, dp, dp, i32p, dp,
                                      dp, i32p, C.c_void_p]
        L.gm_set_workspace.restype = C.c_int
        L.gm_set_workspace.argtypes = [C.c_void_p, C.c_size_t]
        L.gm_workspace_bytes.restype = C.c_size_t
        L.gm_workspace_bytes.argtypes = [C.c_int, C.c_int64, C.c_int]
        L.gm_set_option.restype = C.c_int
        L.gm_set_option.argtypes = [C.c_char_p, C.c_int64]
        L.gm_status_string.restype = C.c_char_p
        L.gm_status_string.argtypes = [C.c_int]
        L.gm_last_stats.restype = C.c_int
        L.gm_last_stats.argtypes = [C.POINTER(Stats)]
        L.gm_num_nodes.restype = C.c_int64
        L.gm_num_nodes.argtypes = [C.c_int]
        L.gm_set_tile.restype = C.c_int
        L.gm_set_tile.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
        L.gm_last_active.restype = C.c_int64
        L.gm_last_active.argtypes = [C.c_int64, C.c_int64, dp, dp, i32p, dp, dp, i32p]
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _stream(stream):
    """HIP stream handle: explicit int/None, else torch's current stream if torch has a GPU."""
    if stream is not None:
        return getattr(stream, "cuda_stream", stream)
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:  # pragma: no cover - torch is optional plumbing
        pass
    return None


def family_id(f) -> int:
    return FAMILIES[f] if isinstance(f, str) else int(f)


def status_string(code: int) -> str:
    return lib().gm_status_string(int(code)).decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise GMError(rc, status_string(rc))
    return rc


def set_option(key: str, value: int) -> None:
    _check(lib().gm_set_option(key.encode(), int(value)))


def last_stats() -> dict:
    s = Stats()
    _check(lib().gm_last_stats(C.byref(s)))
    return s.as_dict()


def set_tile(d: int, family, lanes_per_region: int, grid_blocks: int = 0) -> None:
    """Tile shape of the batched rule kernel for (d, family) (autotuner output)."""
    _check(lib().gm_set_tile(int(d), family_id(family), int(lanes_per_region), int(grid_blocks)))


def num_nodes(d: int) -> int:
    return int(lib().gm_num_nodes(int(d)))


def workspace_bytes(d: int, max_regions: int, mode: int = 0) -> int:
    return int(lib().gm_workspace_bytes(int(d), int(max_regions), int(mode)))


def set_workspace(tensor=None) -> None:
    """Register a caller-owned device buffer (a torch uint8 CUDA tensor) as the
    workspace, or None to return to library-owned memory."""
    if tensor is None:
        _check(lib().gm_set_workspace(None, 0))
    else:
        _check(lib().gm_set_workspace(C.c_void_p(tensor.data_ptr()),
                                      tensor.numel() * tensor.element_size()))


def integrate(family, params, lo, hi, rel_tol, abs_tol=1e-16, max_regions=1 << 22, stream=None):
    """gm_integrate; returns (estimate, error, status)."""
    p, pp = _d(params)
    lo, lp = _d(lo)
    hi, hp = _d(hi)
    d = lo.size
    est = C.c_double()
    err = C.c_double()
    rc = lib().gm_integrate(family_id(family), pp, d, lp, hp, float(rel_tol), float(abs_tol),
                            int(max_regions), C.byref(est), C.byref(err),
                            C.c_void_p(_stream(stream)))
    _check(rc)
    return est.value, err.value, rc


def integrate_noalloc(family, params, lo, hi, rel_tol, abs_tol=1e-16, max_regions=1 << 16,
                      stream=None):
    """gm_integrate_noalloc (no device allocation: the library's fixed 64 MiB
    scratch); returns (estimate, error, status)."""
    p, pp = _d(params)
    lo, lp = _d(lo)
    hi, hp = _d(hi)
    d = lo.size
    est = C.c_double()
    err = C.c_double()
    rc = lib().gm_integrate_noalloc(family_id(family), pp, d, lp, hp, float(rel_tol),
                                    float(abs_tol), int(max_regions), C.byref(est), C.byref(err),
                                    C.c_void_p(_stream(stream)))
    _check(rc)
    return est.value, err.value, rc


def integrate_grad(family, params, lo, hi, rel_tol, abs_tol=1e-16, max_regions=1 << 22,
                   stream=None):
    """gm_integrate_grad; returns (estimate, error, grad[2d], status)."""
    p, pp = _d(params)
    lo, lp = _d(lo)
    hi, hp = _d(hi)
    d = lo.size
    est = C.c_double()
    err = C.c_double()
    g = np.zeros(2 * d)
    rc = lib().gm_integrate_grad(family_id(family), pp, d, lp, hp, float(rel_tol),
                                 float(abs_tol), int(max_regions), C.byref(est), C.byref(err),
                                 _d(g)[1], C.c_void_p(_stream(stream)))
    _check(rc)
    return est.value, err.value, g, rc


def integrate_batch(families, params_list, ds, los, his, rel_tols, abs_tols, max_regions_total,
                    stream=None):
    """gm_integrate_batch; returns (rc, est[n], err[n], status[n])."""
    n = len(families)
    fam = np.ascontiguousarray([family_id(f) for f in families], dtype=np.intc)
    d = np.ascontiguousarray(ds, dtype=np.intc)
    params = np.ascontiguousarray(np.concatenate([np.asarray(x, float) for x in params_list]))
    lo = np.ascontiguousarray(np.concatenate([np.asarray(x, float) for x in los]))
    hi = np.ascontiguousarray(np.concatenate([np.asarray(x, float) for x in his]))
    rt = np.ascontiguousarray(rel_tols, dtype=np.float64)
    at = np.ascontiguousarray(abs_tols, dtype=np.float64)
    est = np.zeros(n)
    err = np.zeros(n)
    st = np.zeros(n, dtype=np.intc)
    P = C.POINTER(C.c_double)
    IP = C.POINTER(C.c_int)
    rc = lib().gm_integrate_batch(n, fam.ctypes.data_as(IP), params.ctypes.data_as(P),
                                  d.ctypes.data_as(IP), lo.ctypes.data_as(P),
                                  hi.ctypes.data_as(P), rt.ctypes.data_as(P),
                                  at.ctypes.data_as(P), int(max_regions_total),
                                  est.ctypes.data_as(P), err.ctypes.data_as(P),
                                  st.ctypes.data_as(IP), C.c_void_p(_stream(stream)))
    _check(rc)
    return rc, est, err, st


def eval_regions(family, params, lo, hi, c, h, lvl, stream=None):
    """gm_eval_regions on host arrays c, h [n, d] and lvl [n]; returns (Q, err, axis)."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    h = np.ascontiguousarray(h, dtype=np.float64)
    lvl = np.ascontiguousarray(lvl, dtype=np.int32)
    n, d = c.shape
    p, pp = _d(params)
    lo, lp = _d(lo)
    hi, hp = _d(hi)
    q = np.zeros(n)
    e = np.zeros(n)
    ax = np.zeros(n, dtype=np.int32)
    P = C.POINTER(C.c_double)
    rc = lib().gm_eval_regions(family_id(family), pp, d, lp, hp, n, c.ctypes.data_as(P),
                               h.ctypes.data_as(P), lvl.ctypes.data_as(C.POINTER(C.c_int32)),
                               q.ctypes.data_as(P), e.ctypes.data_as(P),
                               ax.ctypes.data_as(C.POINTER(C.c_int32)),
                               C.c_void_p(_stream(stream)))
    _check(rc)
    return q, e, ax


def last_active_count() -> int:
    """Size of the last evaluated active set of the previous integrate call."""
    return int(lib().gm_last_active(0, 0, None, None, None, None, None, None))


def last_active(d: int, offset: int = 0, count: int | None = None):
    """Regions [offset, offset + count) of the last evaluated active set of the
    previous integrate call (the whole set by default)."""
    L = lib()
    total = last_active_count()
    n = max(0, min(total - offset, total if count is None else count))
    c = np.zeros((n, d))
    h = np.zeros((n, d))
    lvl = np.zeros(n, dtype=np.int32)
    q = np.zeros(n)
    e = np.zeros(n)
    ax = np.zeros(n, dtype=np.int32)
    P = C.POINTER(C.c_double)
    I32 = C.POINTER(C.c_int32)
    got = L.gm_last_active(offset, n, c.ctypes.data_as(P), h.ctypes.data_as(P),
                           lvl.ctypes.data_as(I32), q.ctypes.data_as(P), e.ctypes.data_as(P),
                           ax.ctypes.data_as(I32))
    if got < 0:
        _check(int(got))
    return {"c": c, "h": h, "lvl": lvl, "Q": q, "err": e, "axis": ax}
