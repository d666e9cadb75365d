"""Exact per-particle Axilrod-Teller potential on the CPU (oracle).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

``phi(x, idx)`` is the canonical multibody summation of Section 1 for n = 3,
evaluated by the plain triple loop in ``at_oracle.c`` (binary64, compensated
per-particle sums).  ``phi_bruteforce`` is a second, independent formulation
for tiny N: it enumerates *ordered* pairs (j, k), forms each interior angle
with atan2(|u x v|, u . v) and halves the total, so it shares neither the
loop structure nor the cosine formula with the C code.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from .build_oracle import ensure_built

_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(ensure_built())
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_at_phi.restype = ctypes.c_double
        lib.oracle_at_phi.argtypes = [dp, dp, dp]
        lib.oracle_phi.restype = ctypes.c_int
        lib.oracle_phi.argtypes = [dp, ctypes.c_int64, ip, ctypes.c_int64, dp, ctypes.c_int]
        lib.oracle_energy.restype = ctypes.c_int
        lib.oracle_energy.argtypes = [dp, ctypes.c_int64, dp, ctypes.c_int]
        lib.oracle_phi_split.restype = ctypes.c_int
        lib.oracle_phi_split.argtypes = [dp, ctypes.c_int64, ip, ctypes.c_int64, ctypes.c_double,
                                         ctypes.c_int, dp, ctypes.c_int]
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _coords(x) -> np.ndarray:
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if x.ndim != 2 or x.shape[1] != 3:
        raise ValueError("x must have shape (N, 3)")
    return x


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def at_phi(xi, xj, xk) -> float:
    """phi of one triangle (Section 1), by the oracle's C routine."""
    a = [np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(3)) for v in (xi, xj, xk)]
    return float(_load().oracle_at_phi(_dp(a[0]), _dp(a[1]), _dp(a[2])))


def phi(x, idx=None, threads: int = 0) -> np.ndarray:
    """Phi(x_i) for i in idx (all particles when idx is None)."""
    x = _coords(x)
    n = x.shape[0]
    idx = np.arange(n, dtype=np.int64) if idx is None else np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros(idx.shape[0], dtype=np.float64)
    rc = _load().oracle_phi(_dp(x), n, _ip(idx), idx.shape[0], _dp(out), int(threads))
    if rc != 0:
        raise ValueError("oracle_phi: bad arguments")
    return out


def energy(x, threads: int = 0) -> float:
    """E = sum over i < j < k of phi, a loop of its own."""
    x = _coords(x)
    e = np.zeros(1, dtype=np.float64)
    if _load().oracle_energy(_dp(x), x.shape[0], _dp(e), int(threads)) != 0:
        raise ValueError("oracle_energy: bad arguments")
    return float(e[0])


def phi_split(x, r_cut: float, far: bool, idx=None, threads: int = 0) -> np.ndarray:
    """Phi restricted to triangles with all sides >= r_cut (far) or not (near)."""
    x = _coords(x)
    n = x.shape[0]
    idx = np.arange(n, dtype=np.int64) if idx is None else np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros(idx.shape[0], dtype=np.float64)
    rc = _load().oracle_phi_split(_dp(x), n, _ip(idx), idx.shape[0], float(r_cut), int(far),
                                  _dp(out), int(threads))
    if rc != 0:
        raise ValueError("oracle_phi_split: bad arguments")
    return out


def _angle(u: np.ndarray, v: np.ndarray) -> float:
    cr = np.cross(u, v)
    return math.atan2(math.sqrt(float(cr @ cr)), float(u @ v))


def phi_triangle_angles(xi, xj, xk) -> float:
    """phi from interior angles computed with atan2 (independent formula)."""
    xi, xj, xk = (np.asarray(v, dtype=np.float64) for v in (xi, xj, xk))
    ti = _angle(xj - xi, xk - xi)
    tj = _angle(xi - xj, xk - xj)
    tk = _angle(xi - xk, xj - xk)
    rij = math.dist(xi, xj)
    rik = math.dist(xi, xk)
    rjk = math.dist(xj, xk)
    return (1.0 + 3.0 * math.cos(ti) * math.cos(tj) * math.cos(tk)) / (rij * rik * rjk) ** 3


def phi_bruteforce(x) -> np.ndarray:
    """Phi for every particle by full enumeration of ordered pairs (tiny N)."""
    x = _coords(x)
    n = x.shape[0]
    if n > 12:
        raise ValueError("brute force is for tiny N")
    out = np.zeros(n)
    for i in range(n):
        terms = []
        for j in range(n):
            for k in range(n):
                if len({i, j, k}) == 3:
                    terms.append(phi_triangle_angles(x[i], x[j], x[k]))
        out[i] = math.fsum(terms) / 2.0
    return out
