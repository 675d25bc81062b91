"""Build libgm.so (HIP, gfx950) in-tree.

The rule (Genz-Malik degree 7 and 9, Gauss-Kronrod) and adjoint kernels are compiled once per integrand family
(-DGM_RULE_FAMILY=k / -DGM_FAMILY=k) so the objects build in parallel; everything links into
paper_2511_01573_amd/libgm.so.  Flags: FP64 code with no implicit FMA
contraction (-ffp-contract=off; fused multiply-adds are written explicitly),
packed-FP32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libgm.so")
ROOT = os.path.dirname(PKG)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-ffp-contract=off", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
FAMILIES = range(1, 8)
# translation units compiled once per integrand family (template-heavy kernels)
PER_FAMILY = ("gm_rule", "gm_rule9", "gm_adjoint", "gm_gk")


def _units():
    units = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        name = os.path.splitext(os.path.basename(src))[0]
        if name in PER_FAMILY:
            for f in FAMILIES:
                units.append((src, os.path.join(BUILD, f"{name}_f{f}.o"),
                              [f"-DGM_RULE_FAMILY={f}", f"-DGM_FAMILY={f}"]))
        else:
            units.append((src, os.path.join(BUILD, f"{name}.o"), []))
    return units


def _headers_mtime():
    hs = glob.glob(os.path.join(CSRC, "*.hpp")) + [os.path.join(ROOT, "include", "gm.h")]
    return max(os.path.getmtime(h) for h in hs)


def _compile(unit, force):
    src, obj, extra = unit
    if not force and os.path.exists(obj):
        if os.path.getmtime(obj) >= max(os.path.getmtime(src), _headers_mtime()):
            return obj, None
    cmd = [HIPCC] + FLAGS + extra + ["-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (p.stdout + p.stderr).splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        return obj, f"compile failed: {' '.join(cmd)}\n{errs}"
    return obj, None


def _link(objs, lib):
    tmp = lib + ".tmp"
    subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs,
                   check=True)
    shutil.move(tmp, lib)
    return lib


def _compile_all(units, force, jobs):
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda u: _compile(u, force), units))
    errors = [e for _, e in results if e]
    if errors:
        raise RuntimeError("\n\n".join(errors))
    return [o for o, _ in results]


def build(force: bool = True, jobs: int | None = None, check: bool = False) -> str:
    """Compile every HIP translation unit for gfx950 and link libgm.so; with
    check=True also the -DGM_CHECK build libgm_check.so (one compile pool)."""
    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    cunits = _check_units() if check else []
    objs = _compile_all(units + cunits, force, jobs)
    _link(objs[:len(units)], LIB)
    if check:
        _link(objs[len(units):], CHECK_LIB)
    return LIB


# Bounds-check build: every unit compiled with -DGM_CHECK (kernel index checks
# that count violations, gm_common.hpp GM_INB) into libgm_check.so, loaded by
# the bounds-check test in place of libgm.so.
CHECK_BUILD = os.path.join(PKG, "_build_check")
CHECK_LIB = os.path.join(PKG, "libgm_check.so")


def _check_units():
    os.makedirs(CHECK_BUILD, exist_ok=True)
    return [(src, os.path.join(CHECK_BUILD, os.path.basename(obj)), extra + ["-DGM_CHECK"])
            for src, obj, extra in _units()]


def build_check(force: bool = True, jobs: int | None = None) -> str:
    """Compile every unit with -DGM_CHECK and link libgm_check.so."""
    return _link(_compile_all(_check_units(), force, jobs), CHECK_LIB)


# Host-sanitizer check program (tests/libgm_sanitize_main.cpp): the library's
# host-logic units recompiled with AddressSanitizer and UndefinedBehaviorSanitizer
# on their host side only (device code as in libgm.so), linked with the kernel
# objects of build() into one executable.
SAN_UNITS = ("gm_api", "gm_batch", "gm_grad")
SAN_BUILD = os.path.join(PKG, "_build_san")
SAN_EXE = os.path.join(PKG, "gm_host_sanitize")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-g"]


def build_host_sanitize(jobs: int | None = None) -> str:
    """Build the host-sanitizer check program (needs the objects of build())."""
    os.makedirs(SAN_BUILD, exist_ok=True)
    units = []
    for name in SAN_UNITS:
        units.append((os.path.join(CSRC, name + ".hip"), os.path.join(SAN_BUILD, name + ".o"), SAN_FLAGS))
    units.append((os.path.join(ROOT, "tests", "libgm_sanitize_main.cpp"),
                  os.path.join(SAN_BUILD, "libgm_sanitize_main.o"), SAN_FLAGS))
    san_objs = _compile_all(units, True, jobs)
    kernels = [o for _, o, _ in _units()
               if os.path.splitext(os.path.basename(o))[0] not in SAN_UNITS]
    missing = [o for o in kernels if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"build() first: missing {missing[:3]}")
    tmp = SAN_EXE + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}"] + SAN_FLAGS + ["-o", tmp] + san_objs + kernels
    subprocess.run(cmd, check=True)
    shutil.move(tmp, SAN_EXE)
    return SAN_EXE


if __name__ == "__main__":
    force = "--incremental" not in sys.argv
    print(build(force=force, check="--check" in sys.argv))
    if "--host-sanitize" in sys.argv:
        print(build_host_sanitize())
