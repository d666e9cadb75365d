"""Seeded synthetic point sets and request traces.

This module only draws inputs: it holds none of the potential's arithmetic,
so both the CPU oracle's tests and the GPU path can take their inputs from it.
Every generator uses ``numpy.random.Generator(PCG64(seed))`` and returns
float64 arrays of shape (N, 3), row-major (x0, y0, z0, x1, ...).

Workloads:
  * ``jittered_lattice`` - n^3 cubic lattice, spacing ``h``, each coordinate
    jittered uniformly in +-``jitter``; for non-cube N the lattice points
    nearest the cube centre are kept (ties broken by z, then y, then x).
    With jitter < h/4 the minimum separation is h - 2*jitter.
  * ``saturated_gaussian_mixture`` - K isotropic Gaussian components with
    uniform means, with sequential rejection of any candidate closer than
    ``min_sep`` to an accepted point (the component is redrawn with it).
  * ``uniform_cube``, ``unit_ball``, ``annulus`` - the three point
    distributions of the paper's experiments (Section 6.2).
  * ``poisson_trace`` - arrival times and sizes of serving requests.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rng",
    "jittered_lattice",
    "saturated_gaussian_mixture",
    "uniform_cube",
    "unit_ball",
    "annulus",
    "poisson_trace",
    "sample_indices",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _lattice_sites(n_points: int, side: int) -> np.ndarray:
    """Integer lattice sites of a side^3 cube, nearest-to-centre first."""
    g = np.arange(side, dtype=np.int64)
    iz, iy, ix = np.meshgrid(g, g, g, indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
    # squared distance to the cube centre, doubled to stay integral
    c = side - 1
    d2 = (2 * ix - c) ** 2 + (2 * iy - c) ** 2 + (2 * iz - c) ** 2
    order = np.lexsort((ix, iy, iz, d2))  # last key is primary
    sel = order[:n_points]
    return np.stack([ix[sel], iy[sel], iz[sel]], axis=1)


def jittered_lattice(n: int, seed: int, spacing: float = 1.0, jitter: float = 0.25) -> np.ndarray:
    """Cubic lattice of N points with uniform per-coordinate jitter."""
    if n < 0:
        raise ValueError("n must be >= 0")
    if n == 0:
        return np.zeros((0, 3), dtype=np.float64)
    side = int(round(n ** (1.0 / 3.0)))
    while side ** 3 < n:
        side += 1
    while side > 1 and (side - 1) ** 3 >= n:
        side -= 1
    sites = _lattice_sites(n, side).astype(np.float64) * spacing
    g = rng(seed)
    return sites + g.uniform(-jitter, jitter, size=(n, 3))


def _cell_keys(cells: np.ndarray) -> np.ndarray:
    off = 1 << 20
    c = cells.astype(np.int64) + off
    return (c[:, 0] << 42) | (c[:, 1] << 21) | c[:, 2]


_OFFSETS = np.array([(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)],
                    dtype=np.int64)


def saturated_gaussian_mixture(n: int, seed: int, components: int = 32, box: float = 100.0,
                               sigma: float = 2.0, min_sep: float = 0.3,
                               batch: int = 65536) -> np.ndarray:
    """Gaussian-mixture points with sequential hard-core rejection.

    Candidates form one sequence, drawn ``batch`` at a time (the components
    of a batch first, then its Gaussian offsets), so ``batch`` is part of
    the generator's definition.  A candidate closer than ``min_sep`` to any
    point accepted before it in the sequence is discarded, and acceptance is
    decided strictly in sequence order; the first ``n`` accepted points are
    returned.
    """
    g = rng(seed)
    means = g.uniform(0.0, box, size=(components, 3))
    acc = np.zeros((0, 3), dtype=np.float64)
    acc_keys = np.zeros(0, dtype=np.int64)  # sorted cell keys of accepted points
    acc_order = np.zeros(0, dtype=np.int64)  # acc index for each sorted key
    sep2 = min_sep * min_sep
    while acc.shape[0] < n:
        comp = g.integers(0, components, size=batch)
        cand = means[comp] + g.normal(0.0, sigma, size=(batch, 3))
        cells = np.floor(cand / min_sep).astype(np.int64)
        ok = np.ones(batch, dtype=bool)
        # conflicts with points accepted in earlier batches
        if acc_keys.size:
            for off in _OFFSETS:
                k = _cell_keys(cells + off)
                lo = np.searchsorted(acc_keys, k, "left")
                hi = np.searchsorted(acc_keys, k, "right")
                cnt = hi - lo
                for t in range(int(cnt.max()) if cnt.size else 0):
                    m = cnt > t
                    idx = acc_order[lo[m] + t]
                    d = cand[m] - acc[idx]
                    close = np.einsum("ij,ij->i", d, d) < sep2
                    sub = np.nonzero(m)[0][close]
                    ok[sub] = False
        # conflicts inside the batch: earlier candidates win if accepted
        bkeys = _cell_keys(cells)
        border = np.argsort(bkeys, kind="stable")
        bsorted = bkeys[border]
        conflicts: dict[int, list[int]] = {}
        for off in _OFFSETS:
            k = _cell_keys(cells + off)
            lo = np.searchsorted(bsorted, k, "left")
            hi = np.searchsorted(bsorted, k, "right")
            cnt = hi - lo
            for t in range(int(cnt.max()) if cnt.size else 0):
                m = np.nonzero(cnt > t)[0]
                other = border[lo[m] + t]
                earlier = other < m
                a_idx, b_idx = m[earlier], other[earlier]
                d = cand[a_idx] - cand[b_idx]
                close = np.einsum("ij,ij->i", d, d) < sep2
                for a, b in zip(a_idx[close].tolist(), b_idx[close].tolist()):
                    conflicts.setdefault(a, []).append(b)
        for a in sorted(conflicts):
            if ok[a] and any(ok[b] for b in conflicts[a]):
                ok[a] = False
        new = cand[ok]
        need = n - acc.shape[0]
        new = new[:need]
        acc = np.concatenate([acc, new], axis=0)
        keys_all = _cell_keys(np.floor(acc / min_sep).astype(np.int64))
        acc_order = np.argsort(keys_all, kind="stable")
        acc_keys = keys_all[acc_order]
    return acc


def uniform_cube(n: int, seed: int) -> np.ndarray:
    """Uniform in the unit cube [0, 1]^3."""
    return rng(seed).uniform(0.0, 1.0, size=(n, 3))


def unit_ball(n: int, seed: int) -> np.ndarray:
    """Uniform in the unit ball (radius by inverse CDF, direction Gaussian)."""
    g = rng(seed)
    v = g.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = g.uniform(0.0, 1.0, size=n) ** (1.0 / 3.0)
    return v * r[:, None]


def annulus(n: int, seed: int, r_in: float = 0.9, r_out: float = 1.0) -> np.ndarray:
    """Uniform in the spherical shell r_in <= r <= r_out (radii are a choice)."""
    g = rng(seed)
    v = g.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    u = g.uniform(0.0, 1.0, size=n)
    r = (r_in ** 3 + u * (r_out ** 3 - r_in ** 3)) ** (1.0 / 3.0)
    return v * r[:, None]


def poisson_trace(n_requests: int, seed: int, rate_hz: float = 200.0,
                  n_min: int = 64, n_max: int = 8192) -> tuple[np.ndarray, np.ndarray]:
    """Arrival times (s) with exponential gaps and log-uniform request sizes."""
    g = rng(seed)
    gaps = g.exponential(1.0 / rate_hz, size=n_requests)
    t = np.cumsum(gaps)
    sizes = np.rint(np.exp(g.uniform(math.log(n_min), math.log(n_max), size=n_requests)))
    return t, sizes.astype(np.int64)


def sample_indices(n: int, m: int, seed: int) -> np.ndarray:
    """m distinct particle indices in [0, n), sorted."""
    return np.sort(rng(seed).choice(n, size=min(m, n), replace=False)).astype(np.int64)
