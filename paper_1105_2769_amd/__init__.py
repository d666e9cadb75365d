"""MI355X (gfx950) per-particle Axilrod-Teller three-body potential.

The compute path is libmb.so (hand-written HIP, C ABI in include/mb.h);
this package is its thin Python binding.  Torch tensors provide device
memory and streams only.
"""
from ._lib import (KdTree, MBError, Server, eval_direct, eval_direct_deterministic,  # noqa: F401
                   eval_factorized, eval_multitree, farfield_eval, lib, mt_params,
                   normal_quantile, trim, validate)

__all__ = ["MBError", "KdTree", "Server", "eval_direct", "eval_direct_deterministic",
           "eval_factorized", "eval_multitree", "farfield_eval", "mt_params", "normal_quantile",
           "trim", "validate", "lib"]
