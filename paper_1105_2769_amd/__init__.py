"""MI355X (gfx950) per-particle Axilrod-Teller three-body potential.

The compute path is libmb.so (hand-written HIP, C ABI in include/mb.h);
this package is its thin Python binding.  Torch tensors provide device
memory and streams only.
"""
from ._lib import MBError, eval_direct, lib, validate  # noqa: F401

__all__ = ["MBError", "eval_direct", "validate", "lib"]
