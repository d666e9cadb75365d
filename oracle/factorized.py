"""The factorized (matrix-product) form of the per-particle sum - oracle side.

TEST INFRASTRUCTURE ONLY.

With squared sides a = r_ij^2, b = r_ik^2, c = r_jk^2 the law of cosines turns
the Axilrod-Teller potential (Section 1) into

    phi = (abc)^(-3/2) + 3/8 (abc)^(-5/2) (a+b-c)(a-b+c)(-a+b+c),

and expanding the cubic gives ten monomials r_ij^e1 r_ik^e2 r_jk^e3.  The
paper restricts its method to potentials that are products of pairwise
functions (Section 1, the product-form equation); each monomial is one, so
per particle

    Phi_i = 1/2 sum_t c_t sum_{j,k} M_e1[i,j] M_e2[i,k] M_e3[j,k]
          = 1/2 sum_t c_t sum_j M_e1[i,j] (M_e2 M_e3)[i,j],

with M_e[u,v] = r_uv^e and zero diagonals (which enforce j != i, k != i,
j != k).  Swapping e1 and e2 swaps the dummy indices j and k, so the ten
monomials collapse to six sums:

    (e1, e2, e3)      coefficient
    (-3, -3, -3)      1 - 3/4 = 1/4
    ( 1, -5, -5)      2 * (-3/8)      (also (-5, 1, -5))
    (-5, -5,  1)      -3/8
    (-1, -3, -5)      2 * 3/8         (also (-3, -1, -5))
    (-1, -5, -3)      2 * 3/8         (also (-5, -1, -3))
    (-3, -5, -1)      2 * 3/8         (also (-5, -3, -1))

Near field.  Entries with r < r_near are set to zero in every M, so the
product form sums exactly the triples whose three sides are all >= r_near;
the other triples (at least one side < r_near) are added exactly.  The two
parts together are the full sum.
"""
from __future__ import annotations

import numpy as np

from . import direct

TERMS = (
    ((-3, -3, -3), 0.25),
    ((1, -5, -5), -0.75),
    ((-5, -5, 1), -0.375),
    ((-1, -3, -5), 0.75),
    ((-1, -5, -3), 0.75),
    ((-3, -5, -1), 0.75),
)


def pair_matrix(x: np.ndarray, e: int, r_near: float = 0.0) -> np.ndarray:
    d = x[:, None, :] - x[None, :, :]
    r = np.sqrt(np.einsum("ijd,ijd->ij", d, d))
    keep = r >= max(r_near, 0.0)
    np.fill_diagonal(keep, False)
    m = np.zeros_like(r)
    m[keep] = r[keep] ** e
    return m


def term_sums(x: np.ndarray, r_near: float = 0.0) -> list[np.ndarray]:
    """The six per-particle sums T_t(i) = sum_j M_e1[i,j] (M_e2 M_e3)[i,j]."""
    x = np.asarray(x, dtype=np.float64)
    mats = {e: pair_matrix(x, e, r_near) for e in (-5, -3, -1, 1)}
    out = []
    for (e1, e2, e3), _c in TERMS:
        out.append(np.einsum("ij,ij->i", mats[e1], mats[e2] @ mats[e3]))
    return out


def phi_far(x: np.ndarray, r_near: float = 0.0) -> np.ndarray:
    """Phi over triples with all three sides >= r_near, by the product form."""
    t = term_sums(x, r_near)
    return 0.5 * sum(c * ti for ((_, c), ti) in zip(TERMS, t))


def phi(x: np.ndarray, r_near: float = 0.0) -> np.ndarray:
    """Product form for the far triples plus exact near triples."""
    x = np.asarray(x, dtype=np.float64)
    far = phi_far(x, r_near)
    if r_near <= 0.0:
        return far
    return far + direct.phi_split(x, r_near, far=False)
