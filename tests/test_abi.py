"""The C ABI library without a GPU: it loads, exports every entry point that
include/gm.h declares, and rejects invalid arguments before touching the
device (no compute call is made here)."""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2511_01573_amd import gm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_api():
    names = declared_functions()
    for n in ["gm_integrate", "gm_integrate_batch", "gm_integrate_grad", "gm_set_workspace",
              "gm_workspace_bytes", "gm_set_option", "gm_status_string", "gm_last_stats"]:
        assert n in names
    assert sorted(gm.EXPORTED) == names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(gm.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings_and_node_count():
    for code in (0, 1, 2, 3, 4, -1, -2):
        assert len(gm.status_string(code)) > 5
    for d in (2, 3, 8, 12, 16):
        assert gm.num_nodes(d) == 2 ** d + 2 * d * d + 2 * d + 1


def test_workspace_registration_checks_alignment():
    """gm_set_workspace only records the buffer (no device access): a pointer
    that is not 256-byte aligned is refused, an aligned one is accepted, and a
    null pointer returns to library-owned memory."""
    L = gm.lib()
    assert L.gm_set_workspace(C.c_void_p(0x10010), 4096) == gm.EINVAL
    assert L.gm_set_workspace(C.c_void_p(0x10000), 4096) == gm.OK
    assert L.gm_set_workspace(None, 0) == gm.OK


def test_workspace_bytes_scales_with_capacity():
    a = gm.workspace_bytes(8, 1 << 20)
    b = gm.workspace_bytes(8, 1 << 21)
    assert 0 < a < b
    # SoA: two ping-pong copies of c, h (16 d bytes each) dominate
    assert b - a >= (1 << 20) * 2 * 16 * 8
    assert gm.workspace_bytes(1, 100) == 0
    assert gm.workspace_bytes(17, 100) == 0


@pytest.mark.parametrize("case", [
    dict(fam=0), dict(fam=8), dict(d=1), dict(d=17), dict(rel_tol=-1e-3),
    dict(rel_tol=float("nan")), dict(abs_tol=float("inf")), dict(rel_tol=0.0, abs_tol=0.0),
    dict(lo_eq_hi=True), dict(nan_param=True), dict(inf_bound=True),
])
def test_integrate_rejects_invalid_arguments(case):
    d = case.get("d", 3)
    lo = np.zeros(max(d, 1))
    hi = np.ones(max(d, 1))
    p = np.ones(2 * max(d, 1))
    if case.get("lo_eq_hi"):
        hi[0] = lo[0]
    if case.get("nan_param"):
        p[1] = np.nan
    if case.get("inf_bound"):
        hi[0] = np.inf
    with pytest.raises(gm.GMError) as ei:
        gm.integrate(case.get("fam", 4), p[:2 * d] if d <= 16 else np.ones(2 * d),
                     lo[:d] if d <= 16 else np.zeros(d), hi[:d] if d <= 16 else np.ones(d),
                     case.get("rel_tol", 1e-3), case.get("abs_tol", 1e-16), stream=0)
    assert ei.value.code == gm.EINVAL


def test_options_validation():
    with pytest.raises(gm.GMError):
        gm.set_option("no_such_option", 1)
    with pytest.raises(gm.GMError):
        gm.set_option("max_iters", 0)
    with pytest.raises(gm.GMError):
        gm.set_option("lanes_per_region", 3)
    with pytest.raises(gm.GMError):
        gm.set_option("init_log2_regions", 31)
    for key, bad in (("rule", 3), ("rule", -1), ("prune", 2), ("timing", 3), ("err_model", 2),
                     ("err_model", -1)):
        with pytest.raises(gm.GMError):
            gm.set_option(key, bad)
    gm.set_option("max_iters", 10000)
    gm.set_option("init_log2_regions", 12)


def test_gauss_kronrod_rule_validates_dimension_before_any_device_work():
    # d = 7 is beyond the tensor-product rule's range: rejected on the host
    gm.set_option("rule", 1)
    try:
        with pytest.raises(gm.GMError) as ei:
            gm.integrate(4, np.ones(14), np.zeros(7), np.ones(7), 1e-6, 1e-16, stream=0)
        assert ei.value.code == gm.EINVAL
        with pytest.raises(gm.GMError) as ei:
            gm.integrate_grad(4, np.ones(6), np.zeros(3), np.ones(3), 1e-6, 1e-16, stream=0)
        assert ei.value.code == gm.EINVAL
    finally:
        gm.set_option("rule", 0)


def test_err_model_option_accepts_both_models():
    gm.set_option("err_model", 1)
    gm.set_option("err_model", 0)


def test_eval_regions_rejects_bad_levels():
    c = np.full((2, 3), 0.5)
    h = np.full((2, 3), 0.5)
    with pytest.raises(gm.GMError):
        gm.eval_regions(4, np.ones(6), np.zeros(3), np.ones(3), c, h, np.array([0, -1]), stream=0)


def test_product_path_has_no_oracle_dependency():
    # the package never imports, links or runs the CPU oracle
    pkg = os.path.join(ROOT, "paper_2511_01573_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                for pat in ("import oracle", "from oracle", "liboracle", "gm_oracle", "gmo_"):
                    assert pat not in src, (f, pat)
