"""Three-body far-field expansion of order p (Section 3.2) - oracle side.

TEST INFRASTRUCTURE ONLY.

For a point x of node P1 and two other nodes P2, P3 with centres c2, c3,
the contribution of P2 x P3 to x is

    Phi(x; P2 x P3) = sum over y in P2, z in P3 of phi(x, y, z).

Section 3.2 expands each pairwise factor of a product potential in the
displacements y - c2 and z - c3 and truncates at total order p (the
truncated three-body far-field expansion); for a product of pairwise
functions the kept terms are exactly the monomials (y - c2)^a (z - c3)^b
with |a| + |b| <= p of the joint Taylor series, so the truncated expansion
is the degree-p Taylor polynomial of phi(x, c2 + u, c3 + v) in (u, v),
summed over the points:

    Phi_p(x) = sum_{|a| + |b| <= p} C_ab(x) M_a(P2) M_b(P3),
    M_a(P)   = sum over y in P of (y - c)^a       (moments of the node),
    C_ab(x)  = Taylor coefficient of u^a v^b.

The Axilrod-Teller phi is not one product of pairwise functions but a sum
of ten (the law-of-cosines expansion); the expansion is linear, so this is
the sum of the per-term expansions.  x is kept exact: at p = 0 the
expansion is |P2| |P3| phi(x, c2, c3), and at x = c1 it is the monopole
|P2| |P3| phi(c1, c2, c3) of Section 4.  The evaluation cost per point grows
as O(p^6) (Section 3.2).

The Taylor coefficients are computed by plain truncated polynomial
arithmetic in the six variables (u, v), with phi written through squared
distances a = |x - c2 - u|^2, b = |x - c3 - v|^2, c = |c2 + u - c3 - v|^2:
phi = (abc)^(-3/2) + 3/8 (abc)^(-5/2) (a + b - c)(a - b + c)(-a + b + c).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

NV = 6  # variables: u (3), v (3)


def monomials(p: int) -> list[tuple[int, ...]]:
    """Exponent tuples of the monomials in NV variables of total degree <= p."""
    out = []
    for d in range(p + 1):
        for c in itertools.combinations_with_replacement(range(NV), d):
            e = [0] * NV
            for i in c:
                e[i] += 1
            out.append(tuple(e))
    return out


class Poly:
    """A polynomial in (u, v) truncated at total degree p: {exponents: coefficient}."""

    def __init__(self, p: int, terms=None):
        self.p = p
        self.t = {k: v for k, v in (terms or {}).items() if sum(k) <= p}

    @staticmethod
    def const(p, c):
        return Poly(p, {(0,) * NV: float(c)})

    def c0(self) -> float:
        return self.t.get((0,) * NV, 0.0)

    def __add__(self, o):
        o = o if isinstance(o, Poly) else Poly.const(self.p, o)
        r = dict(self.t)
        for k, v in o.t.items():
            r[k] = r.get(k, 0.0) + v
        return Poly(self.p, r)

    __radd__ = __add__

    def __neg__(self):
        return Poly(self.p, {k: -v for k, v in self.t.items()})

    def __sub__(self, o):
        return self + (-(o if isinstance(o, Poly) else Poly.const(self.p, o)))

    def __rsub__(self, o):
        return (-self) + o

    def __mul__(self, o):
        if not isinstance(o, Poly):
            return Poly(self.p, {k: v * o for k, v in self.t.items()})
        r = {}
        for k1, v1 in self.t.items():
            for k2, v2 in o.t.items():
                k = tuple(a + b for a, b in zip(k1, k2))
                if sum(k) <= self.p:
                    r[k] = r.get(k, 0.0) + v1 * v2
        return Poly(self.p, r)

    __rmul__ = __mul__

    def pow(self, e: float):
        """self^e by the binomial series about the constant term (which must be > 0)."""
        s0 = self.c0()
        d = (self - s0) * (1.0 / s0)  # no constant term
        out = Poly.const(self.p, 1.0)
        term = Poly.const(self.p, 1.0)
        coef = 1.0
        for k in range(1, self.p + 1):
            term = term * d
            coef *= (e - (k - 1)) / k
            out = out + term * coef
        return out * (s0 ** e)


def _sqdist(p: int, d: np.ndarray, su: int, sv: int) -> Poly:
    """|d + su u + sv v|^2 as a polynomial (su, sv in {-1, 0, 1})."""
    r = Poly.const(p, float(d @ d))
    for i in range(3):
        for s, off in ((su, 0), (sv, 3)):
            if s == 0:
                continue
            e = [0] * NV
            e[off + i] = 1
            r = r + Poly(p, {tuple(e): 2.0 * s * d[i]})
            e2 = [0] * NV
            e2[off + i] = 2
            r = r + Poly(p, {tuple(e2): 1.0})
        if su != 0 and sv != 0:
            e = [0] * NV
            e[i] = 1
            e[3 + i] = 1
            r = r + Poly(p, {tuple(e): 2.0 * su * sv})
    return r


def taylor_coefficients(x, c2, c3, p: int) -> Poly:
    """Degree-p Taylor polynomial of phi(x, c2 + u, c3 + v) in (u, v)."""
    x, c2, c3 = (np.asarray(v, dtype=np.float64) for v in (x, c2, c3))
    a = _sqdist(p, x - c2, -1, 0)     # |x - (c2 + u)|^2
    b = _sqdist(p, x - c3, 0, -1)     # |x - (c3 + v)|^2
    c = _sqdist(p, c2 - c3, 1, -1)    # |(c2 + u) - (c3 + v)|^2
    abc = a * b * c
    pp = (a + b - c) * (a - b + c) * (c + b - a)
    return abc.pow(-1.5) + abc.pow(-2.5) * pp * 0.375


def moments(pts, c, p: int) -> dict:
    """M_a = sum over the points of (y - c)^a for |a| <= p (3 variables)."""
    d = np.asarray(pts, dtype=np.float64) - np.asarray(c, dtype=np.float64)
    out = {}
    for deg in range(p + 1):
        for comb in itertools.combinations_with_replacement(range(3), deg):
            e = [0, 0, 0]
            for i in comb:
                e[i] += 1
            out[tuple(e)] = float(np.prod(d ** np.array(e), axis=1).sum())
    return out


def farfield(x, p2_pts, p3_pts, p: int, c2=None, c3=None) -> float:
    """Phi_p(x; P2 x P3): the truncated expansion about the centroids (or c2, c3)."""
    p2_pts = np.asarray(p2_pts, dtype=np.float64)
    p3_pts = np.asarray(p3_pts, dtype=np.float64)
    c2 = p2_pts.mean(0) if c2 is None else np.asarray(c2, dtype=np.float64)
    c3 = p3_pts.mean(0) if c3 is None else np.asarray(c3, dtype=np.float64)
    poly = taylor_coefficients(x, c2, c3, p)
    m2 = moments(p2_pts, c2, p)
    m3 = moments(p3_pts, c3, p)
    total = 0.0
    for k, v in poly.t.items():
        total += v * m2[k[:3]] * m3[k[3:]]
    return total


def exact(x, p2_pts, p3_pts) -> float:
    """Phi(x; P2 x P3) by the plain double sum (cosines from dot products)."""
    from .multitree import at_phi_np

    y = np.asarray(p2_pts, dtype=np.float64)[:, None, :]
    z = np.asarray(p3_pts, dtype=np.float64)[None, :, :]
    xx = np.broadcast_to(np.asarray(x, dtype=np.float64), (y.shape[0], z.shape[1], 3))
    return float(at_phi_np(xx, np.broadcast_to(y, xx.shape), np.broadcast_to(z, xx.shape)).sum())
