"""Philox4x32-10 counter-based generator (oracle side).

TEST INFRASTRUCTURE ONLY.

Written from the published definition (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11): a 4 x 32-bit counter
and a 2 x 32-bit key go through 10 rounds.  Each round multiplies counter
words 0 and 2 by the constants 0xD2511F53 and 0xCD9E8D57 into 64-bit
products, and the new counter is (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0).
Between rounds the key is bumped by the Weyl constants 0x9E3779B9 and
0xBB67AE85 (mod 2^32).

The Monte Carlo step draws its random tuples from this generator; the GPU
library carries its own implementation of the same definition.  The
mapping from a sample to (counter, key) and from output words to indices is
fixed in ``multitree.mc_draw``.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """One block: ctr = 4 uint32 words, key = 2 uint32 words -> 4 uint32 words."""
    c0, c1, c2, c3 = (int(v) & MASK for v in ctr)
    k0, k1 = (int(v) & MASK for v in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def philox4x32_10_np(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """Vectorized form: ctr (M, 4) and key (M, 2) uint32 arrays -> (M, 4) uint32."""
    ctr = np.asarray(ctr, dtype=np.uint64) & MASK
    key = np.asarray(key, dtype=np.uint64) & MASK
    c0, c1, c2, c3 = (ctr[:, i].copy() for i in range(4))
    k0, k1 = key[:, 0].copy(), key[:, 1].copy()
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    mask = np.uint64(MASK)
    sh = np.uint64(32)
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(W0)) & mask
            k1 = (k1 + np.uint64(W1)) & mask
        p0 = m0 * c0  # < 2^64, exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> sh, p0 & mask
        hi1, lo1 = p1 >> sh, p1 & mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=1).astype(np.uint32)
