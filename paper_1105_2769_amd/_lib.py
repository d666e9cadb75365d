"""ctypes binding of libmb.so (argument marshalling only).

Every function here checks its tensors, passes raw device pointers and the
current HIP stream to the C ABI declared in ``include/mb.h`` and turns a
non-OK status into ``MBError``.  No arithmetic of the method happens here.
If the shared library is missing, loading raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmb.so")

MB_OK = 0
STATUS_NAMES = {
    0: "MB_OK",
    1: "MB_ERR_INVALID",
    2: "MB_ERR_DEGENERATE",
    3: "MB_ERR_OOM",
    4: "MB_ERR_DEVICE",
    5: "MB_ERR_UNSUPPORTED",
}
PREC = {"fp64": 0, "fp32c": 1}


class MBError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
        self.msg = msg


_lib = None

_c_i32 = ctypes.c_int32
_c_i64 = ctypes.c_int64
_c_dbl = ctypes.c_double
_c_vp = ctypes.c_void_p

# name -> (restype, argtypes)
SIGNATURES = {
    "mb_last_error": (ctypes.c_char_p, []),
    "mb_version": (_c_i32, []),
    "mb_validate": (_c_i32, [_c_vp, _c_i64, ctypes.POINTER(_c_dbl), ctypes.POINTER(_c_i32),
                             ctypes.POINTER(_c_dbl), _c_vp]),
    "mb_eval_direct": (_c_i32, [_c_vp, _c_i64, _c_i32, _c_vp, _c_vp]),
    "mb_eval_direct_unchecked": (_c_i32, [_c_vp, _c_i64, _c_i32, _c_vp, _c_vp]),
}


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(status: int) -> None:
    if status != MB_OK:
        raise MBError(status, lib().mb_last_error().decode(errors="replace"))


def stream_of(t) -> _c_vp:
    import torch

    return _c_vp(torch.cuda.current_stream(t.device).cuda_stream)


def _points(x):
    import torch

    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("x must be a CUDA (HIP) torch tensor")
    if x.dtype != torch.float64 or x.dim() != 2 or x.shape[1] != 3:
        raise TypeError("x must be float64 with shape (N, 3)")
    return x.contiguous()


def validate(x) -> tuple[float, bool, tuple]:
    """(min squared pair distance, all coordinates finite, bounding box)."""
    x = _points(x)
    md2 = _c_dbl()
    fin = _c_i32()
    box = (_c_dbl * 6)()
    check(lib().mb_validate(_c_vp(x.data_ptr()), x.shape[0], ctypes.byref(md2), ctypes.byref(fin),
                            box, stream_of(x)))
    return md2.value, bool(fin.value), tuple(box)


def eval_direct(x, prec: str = "fp64", out=None, checked: bool = True):
    """Exhaustive Phi for every point (mb_eval_direct, or the unchecked,
    non-blocking mb_eval_direct_unchecked when checked=False)."""
    import torch

    x = _points(x)
    n = x.shape[0]
    if prec not in PREC:
        raise ValueError(f"prec must be one of {sorted(PREC)}")
    phi = torch.empty(n, dtype=torch.float64, device=x.device) if out is None else out
    if phi.dtype != torch.float64 or phi.numel() != n or not phi.is_contiguous():
        raise TypeError("out must be a contiguous float64 tensor of N elements")
    fn = lib().mb_eval_direct if checked else lib().mb_eval_direct_unchecked
    check(fn(_c_vp(x.data_ptr()), n, PREC[prec], _c_vp(phi.data_ptr()), stream_of(x)))
    return phi
