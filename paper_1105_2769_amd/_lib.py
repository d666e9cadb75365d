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
    6: "MB_ERR_CANCELLED",
}
PREC = {"fp64": 0, "fp32c": 1}
BOUND = {"signed": 0, "two_sided": 1}


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

class MtParams(ctypes.Structure):
    _fields_ = [("eps_rel", ctypes.c_double), ("tau_abs", ctypes.c_double),
                ("alpha", ctypes.c_double), ("m_limit", ctypes.c_int32),
                ("m_min", ctypes.c_int32), ("zeta", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("base_prec", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("bound", ctypes.c_int32), ("order", ctypes.c_int32)]


class MtStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in
                ("visited", "det_prunes", "mc_prunes", "mc_failed", "base_cases", "base_triples",
                 "mc_samples", "max_stack", "rounds")] + \
               [("build_ms", ctypes.c_double), ("traverse_ms", ctypes.c_double),
                ("classify_ms", ctypes.c_double), ("mc_ms", ctypes.c_double),
                ("base_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class FactorStats(ctypes.Structure):
    _fields_ = [("pairmat_ms", ctypes.c_double), ("gemm_ms", ctypes.c_double),
                ("near_ms", ctypes.c_double), ("near_pairs", ctypes.c_int64),
                ("gemm_flops", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in
                ("submitted", "completed", "failed", "fp64_fallbacks", "slices", "units",
                 "mixed_slices", "points_fp64", "peak_reserved")] + \
               [("peak_active", ctypes.c_int32), ("drain_launches", ctypes.c_int32),
                ("triples", ctypes.c_double), ("busy_ms", ctypes.c_double),
                ("stage_ms", ctypes.c_double), ("finalize_ms", ctypes.c_double),
                ("cancelled", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "pad"}


# name -> (restype, argtypes)
SIGNATURES = {
    "mb_last_error": (ctypes.c_char_p, []),
    "mb_version": (_c_i32, []),
    "mb_validate": (_c_i32, [_c_vp, _c_i64, ctypes.POINTER(_c_dbl), ctypes.POINTER(_c_i32),
                             ctypes.POINTER(_c_dbl), _c_vp]),
    "mb_eval_direct": (_c_i32, [_c_vp, _c_i64, _c_i32, _c_vp, _c_vp]),
    "mb_eval_direct_unchecked": (_c_i32, [_c_vp, _c_i64, _c_i32, _c_vp, _c_vp]),
    "mb_eval_direct_noalloc": (_c_i32, [_c_vp, _c_i64, _c_i32, _c_vp, _c_vp]),
    "mb_eval_direct_deterministic": (_c_i32, [_c_vp, _c_i64, _c_vp, _c_i64, _c_vp]),
    "mb_trim": (_c_i32, [_c_vp, ctypes.POINTER(_c_i64)]),
    "mb_build_kdtree": (_c_i32, [_c_vp, _c_i64, _c_i32, _c_vp, ctypes.POINTER(_c_vp)]),
    "mb_free_kdtree": (_c_i32, [_c_vp]),
    "mb_kdtree_info": (_c_i32, [_c_vp, ctypes.POINTER(_c_i64), ctypes.POINTER(_c_i32),
                                ctypes.POINTER(_c_i32), ctypes.POINTER(_c_dbl)]),
    "mb_kdtree_export": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp]),
    "mb_mt_params_default": (None, [ctypes.POINTER(MtParams)]),
    "mb_eval_multitree": (_c_i32, [_c_vp, _c_i64, _c_i32, ctypes.POINTER(MtParams), _c_vp, _c_vp,
                                   _c_vp, ctypes.POINTER(MtStats), _c_vp]),
    "mb_normal_quantile": (_c_dbl, [_c_dbl]),
    "mb_farfield_eval": (_c_i32, [_c_vp, _c_i64, _c_vp, _c_i64, _c_vp, _c_i64, _c_i32, _c_vp,
                                  _c_vp]),
    "mb_eval_factorized": (_c_i32, [_c_vp, _c_i64, _c_i32, _c_i32, _c_dbl, _c_vp,
                                    ctypes.POINTER(FactorStats), _c_vp]),
    "mb_server_create": (_c_i32, [_c_i64, _c_i32, _c_vp, ctypes.POINTER(_c_vp)]),
    "mb_server_submit": (_c_i32, [_c_vp, _c_vp, _c_i64, _c_i32, ctypes.POINTER(_c_i64)]),
    "mb_server_poll": (_c_i32, [_c_vp, _c_i64, _c_vp, ctypes.POINTER(_c_i32)]),
    "mb_server_wait": (_c_i32, [_c_vp, _c_i64, _c_i32, ctypes.POINTER(_c_i32)]),
    "mb_server_latency": (_c_i32, [_c_vp, _c_i64, ctypes.POINTER(_c_dbl)]),
    "mb_server_stats_get": (_c_i32, [_c_vp, ctypes.POINTER(ServerStats)]),
    "mb_server_set_slice_units": (_c_i32, [_c_vp, _c_i64]),
    "mb_server_cancel": (_c_i32, [_c_vp, _c_i64]),
    "mb_server_set_timeout": (_c_i32, [_c_vp, _c_i32]),
    "mb_server_destroy": (_c_i32, [_c_vp]),
    "mb_struct_size": (_c_i64, [ctypes.c_char_p]),
}
HALF = {"fp16": 0, "bf16": 1}


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


def trim(device=None) -> int:
    """Release the library's cached device memory on the current device
    after the current stream's work (mb_trim); returns the bytes released."""
    import torch

    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    released = _c_i64()
    check(lib().mb_trim(_c_vp(torch.cuda.current_stream(dev).cuda_stream), ctypes.byref(released)))
    return released.value


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


def eval_direct_deterministic(x, out=None, scratch_bytes: int = 0):
    """Binary64 exhaustive Phi with a fixed summation order
    (mb_eval_direct_deterministic): bitwise the same on every call."""
    import torch

    x = _points(x)
    n = x.shape[0]
    phi = torch.empty(n, dtype=torch.float64, device=x.device) if out is None else out
    if phi.dtype != torch.float64 or phi.numel() != n or not phi.is_contiguous():
        raise TypeError("out must be a contiguous float64 tensor of N elements")
    check(lib().mb_eval_direct_deterministic(_c_vp(x.data_ptr()), n, _c_vp(phi.data_ptr()),
                                             int(scratch_bytes), stream_of(x)))
    return phi


class KdTree:
    """A device-resident kd-tree (mb_build_kdtree); freed with the object."""

    def __init__(self, x, leaf_size: int = 32):
        x = _points(x)
        self._x = x
        handle = _c_vp()
        check(lib().mb_build_kdtree(_c_vp(x.data_ptr()), x.shape[0], int(leaf_size), stream_of(x),
                                    ctypes.byref(handle)))
        self.handle = handle
        self.leaf_size = int(leaf_size)
        n = _c_i64()
        m = _c_i32()
        d = _c_i32()
        ms = _c_dbl()
        check(lib().mb_kdtree_info(handle, ctypes.byref(n), ctypes.byref(m), ctypes.byref(d),
                                   ctypes.byref(ms)))
        self.n, self.n_nodes, self.max_depth, self.build_ms = n.value, m.value, d.value, ms.value

    def export(self) -> dict:
        import numpy as np

        m = self.n_nodes
        perm = np.zeros(self.n, dtype=np.int32)
        ranges = np.zeros(2 * m, dtype=np.int32)
        children = np.zeros(2 * m, dtype=np.int32)
        bbox = np.zeros(6 * m, dtype=np.float64)
        cen = np.zeros(3 * m, dtype=np.float64)
        ptr = lambda a: _c_vp(a.ctypes.data)  # noqa: E731
        check(lib().mb_kdtree_export(self.handle, ptr(perm), ptr(ranges), ptr(children), ptr(bbox),
                                     ptr(cen)))
        return dict(perm=perm, begin=ranges[0::2], end=ranges[1::2], left=children[0::2],
                    right=children[1::2], lo=bbox.reshape(m, 6)[:, :3], hi=bbox.reshape(m, 6)[:, 3:],
                    centroid=cen.reshape(m, 3))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            lib().mb_free_kdtree(h)
            self.handle = None


def mt_params(**kw) -> MtParams:
    p = MtParams()
    lib().mb_mt_params_default(ctypes.byref(p))
    names = {name for name, _ in MtParams._fields_}
    for key, val in kw.items():
        if key not in names:
            raise TypeError(f"unknown traversal parameter {key!r}")
        if key == "base_prec" and isinstance(val, str):
            val = PREC[val]
        if key == "bound" and isinstance(val, str):
            val = BOUND[val]
        setattr(p, key, val)
    return p


def eval_multitree(x, eps: float = 1e-2, alpha: float = 0.05, leaf_size: int = 32,
                   tree: KdTree | None = None, coverage: bool = False, **kw):
    """Triple-tree Phi (mb_eval_multitree).  Returns (phi, stats[, coverage])."""
    import torch

    x = _points(x)
    n = x.shape[0]
    p = mt_params(eps_rel=eps, alpha=alpha, **kw)
    phi = torch.empty(n, dtype=torch.float64, device=x.device)
    cov = torch.zeros(n, dtype=torch.int64, device=x.device) if coverage else None
    st = MtStats()
    check(lib().mb_eval_multitree(_c_vp(x.data_ptr()), n, int(leaf_size), ctypes.byref(p),
                                  tree.handle if tree is not None else None, _c_vp(phi.data_ptr()),
                                  _c_vp(cov.data_ptr()) if cov is not None else None,
                                  ctypes.byref(st), stream_of(x)))
    if coverage:
        return phi, st.as_dict(), cov
    return phi, st.as_dict()


def farfield_eval(x, y, z, order: int):
    """Far-field expansion at targets x due to source sets y, z (mb_farfield_eval)."""
    import torch

    x, y, z = _points(x), _points(y), _points(z)
    out = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
    check(lib().mb_farfield_eval(_c_vp(x.data_ptr()), x.shape[0], _c_vp(y.data_ptr()), y.shape[0],
                                 _c_vp(z.data_ptr()), z.shape[0], int(order),
                                 _c_vp(out.data_ptr()), stream_of(x)))
    return out


def normal_quantile(alpha_half: float) -> float:
    return float(lib().mb_normal_quantile(float(alpha_half)))


def eval_factorized(x, fmt: str = "fp16", planes: int = 2, r_near: float = 1.5):
    """Phi through the product form on MFMA (mb_eval_factorized); (phi, stats)."""
    import torch

    x = _points(x)
    n = x.shape[0]
    phi = torch.empty(n, dtype=torch.float64, device=x.device)
    st = FactorStats()
    check(lib().mb_eval_factorized(_c_vp(x.data_ptr()), n, HALF[fmt], int(planes), float(r_near),
                                   _c_vp(phi.data_ptr()), ctypes.byref(st), stream_of(x)))
    return phi, st.as_dict()


class Server:
    """A serving loop (mb_server_*): host arrays in, host arrays out.

    ``submit`` copies the points and returns a request id at once; ``poll``
    and ``wait`` report completion; ``result`` fetches Phi (numpy, input
    order) once.  The server finishes all submitted work when closed.
    """

    def __init__(self, hbm_budget_bytes: int = 32 << 30, max_slots: int = 256, stream=None):
        import torch

        s = stream if stream is not None else torch.cuda.current_stream()
        self._srv = _c_vp()
        self._stream = s  # keep the stream alive while the server uses it
        check(lib().mb_server_create(int(hbm_budget_bytes), int(max_slots), _c_vp(s.cuda_stream),
                                     ctypes.byref(self._srv)))
        self._n = {}

    def submit(self, x, prec: str = "fp32c") -> int:
        import numpy as np

        a = np.ascontiguousarray(x, dtype=np.float64)
        if a.ndim != 2 or a.shape[1] != 3:
            raise TypeError("x must have shape (N, 3)")
        rid = _c_i64()
        check(lib().mb_server_submit(self._srv, _c_vp(a.ctypes.data), a.shape[0], PREC[prec],
                                     ctypes.byref(rid)))
        self._n[rid.value] = a.shape[0]
        return rid.value

    def poll(self, rid: int) -> bool:
        done = _c_i32()
        check(lib().mb_server_poll(self._srv, int(rid), None, ctypes.byref(done)))
        return bool(done.value)

    def wait(self, rid: int = -1, timeout_ms: int = -1) -> bool:
        done = _c_i32()
        check(lib().mb_server_wait(self._srv, int(rid), int(timeout_ms), ctypes.byref(done)))
        return bool(done.value)

    def result(self, rid: int):
        import numpy as np

        out = np.empty(self._n[rid], dtype=np.float64)
        done = _c_i32()
        check(lib().mb_server_poll(self._srv, int(rid), _c_vp(out.ctypes.data), ctypes.byref(done)))
        if not done.value:
            raise RuntimeError(f"request {rid} has not finished")
        return out

    def latency(self, rid: int) -> float:
        v = _c_dbl()
        check(lib().mb_server_latency(self._srv, int(rid), ctypes.byref(v)))
        return v.value

    def stats(self) -> dict:
        st = ServerStats()
        check(lib().mb_server_stats_get(self._srv, ctypes.byref(st)))
        return st.as_dict()

    def set_slice_units(self, units: int) -> None:
        check(lib().mb_server_set_slice_units(self._srv, int(units)))

    def cancel(self, rid: int) -> None:
        check(lib().mb_server_cancel(self._srv, int(rid)))

    def set_timeout(self, timeout_ms: int) -> None:
        check(lib().mb_server_set_timeout(self._srv, int(timeout_ms)))

    def close(self) -> None:
        if self._srv:
            check(lib().mb_server_destroy(self._srv))
            self._srv = _c_vp()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
