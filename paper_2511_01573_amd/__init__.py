"""Adaptive Genz-Malik cubature on AMD MI355X (gfx950), FP64.

Method of arXiv 2511.01573 (Sec. 2-4): the breadth-first adaptive loop with a
fully symmetric Genz-Malik rule, embedded-rule error estimate and
fourth-difference split axis, running in hand-written HIP kernels behind the
C ABI in include/gm.h.  `gm` is the ctypes binding; `autograd` wraps the
gradient entry point in a torch.autograd.Function; `workloads` holds the
seeded input generators.
"""
from . import gm  # noqa: F401
from .gm import (GMError, integrate, integrate_batch, integrate_grad, eval_regions,  # noqa: F401
                 set_option, last_stats, status_string)
