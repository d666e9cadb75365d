"""Pins of the three-body far-field expansion oracle (Section 3.2), no GPU.

  * p = 0 is |P2| |P3| phi(x, c2, c3), and at x = c1 the monopole of
    Section 4;
  * nodes of single points: every order is exact;
  * the Taylor coefficients agree with finite differences of phi
    (first and second derivatives), an independent route;
  * the truncation error falls as p grows on separated nodes (p = 0..4);
  * about the centroids the first-order term vanishes (first moments are
    zero), about other centres it does not and then p = 1 is closer than
    p = 0;
  * homogeneity: scaling every point by s scales each order by s^-9.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import direct as oracle_direct
from oracle import farfield as ff


def three_nodes(seed, sep=6.0, width=1.0, n2=20, n3=15):
    """A point near c1 and two boxes of points around c2, c3, where the three
    centres are a randomly rotated triangle with sides sep * (1, 1.2, 1.4)."""
    rng = workloads.rng(seed)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    a, b, cc = sep, 1.2 * sep, 1.4 * sep  # sides c1c2, c1c3, c2c3
    cos1 = (a * a + b * b - cc * cc) / (2 * a * b)
    tri = np.array([[0.0, 0, 0], [a, 0, 0], [b * cos1, b * math.sqrt(1 - cos1 ** 2), 0]])
    c = tri @ q.T + rng.normal(size=3)
    x = rng.uniform(-width / 2, width / 2, size=3) + c[0]
    p2 = rng.uniform(-width / 2, width / 2, size=(n2, 3)) + c[1]
    p3 = rng.uniform(-width / 2, width / 2, size=(n3, 3)) + c[2]
    return x, p2, p3, c


def test_order_zero_is_the_monopole():
    x, p2, p3, c = three_nodes(1)
    c2, c3 = p2.mean(0), p3.mean(0)
    want = len(p2) * len(p3) * oracle_direct.at_phi(x, c2, c3)
    assert ff.farfield(x, p2, p3, 0) == pytest.approx(want, rel=1e-13)
    c1 = np.array([0.3, -0.2, 0.1]) + c[0]
    assert ff.farfield(c1, p2, p3, 0) == pytest.approx(
        len(p2) * len(p3) * oracle_direct.at_phi(c1, c2, c3), rel=1e-13)


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_single_point_nodes_are_exact(p):
    x, p2, p3, _ = three_nodes(2)
    y, z = p2[:1], p3[:1]
    assert ff.farfield(x, y, z, p) == pytest.approx(ff.exact(x, y, z), rel=1e-12)


def test_coefficients_match_finite_differences():
    x, p2, p3, _ = three_nodes(3, sep=3.0)
    c2, c3 = p2.mean(0), p3.mean(0)
    poly = ff.taylor_coefficients(x, c2, c3, 2)

    def f(w):
        return oracle_direct.at_phi(x, c2 + w[:3], c3 + w[3:])

    h = 1e-4
    f0 = f(np.zeros(6))
    assert poly.c0() == pytest.approx(f0, rel=1e-14)
    for i in range(6):
        e = np.zeros(6)
        e[i] = h
        g = (f(e) - f(-e)) / (2 * h)
        key = tuple(1 if k == i else 0 for k in range(6))
        assert poly.t[key] == pytest.approx(g, rel=1e-6, abs=1e-9 * abs(f0))
        for j in range(i, 6):
            e2 = np.zeros(6)
            e2[j] = h
            d2 = (f(e + e2) - f(e - e2) - f(-e + e2) + f(-e - e2)) / (4 * h * h)
            key = [0] * 6
            key[i] += 1
            key[j] += 1
            coef = poly.t.get(tuple(key), 0.0)
            # Taylor coefficient of u_i u_j is d2 / 2 on the diagonal, d2 off it
            want = d2 / 2 if i == j else d2
            assert coef == pytest.approx(want, rel=1e-4, abs=1e-6 * abs(f0))


def test_error_falls_with_order():
    # the truncation error is not monotone in p for every configuration (a
    # low order can cancel by luck) but it falls geometrically overall
    ratios, last = [], []
    for seed in range(10, 30):
        x, p2, p3, _ = three_nodes(seed, sep=7.0, width=1.2)
        ex = ff.exact(x, p2, p3)
        err = [abs(ff.farfield(x, p2, p3, p) - ex) / abs(ex) for p in range(5)]
        ratios.append(err[4] / err[0])
        last.append(err[4])
    assert np.median(ratios) < 0.05
    assert max(last) < 2e-3


def test_first_order_vanishes_about_centroids_only():
    x, p2, p3, _ = three_nodes(7, sep=6.0)
    assert ff.farfield(x, p2, p3, 1) == pytest.approx(ff.farfield(x, p2, p3, 0), rel=1e-13)
    # about shifted centres the first-order term is non-zero and helps
    c2 = p2.mean(0) + np.array([0.3, -0.2, 0.25])
    c3 = p3.mean(0) + np.array([-0.25, 0.2, 0.3])
    ex = ff.exact(x, p2, p3)
    e0 = abs(ff.farfield(x, p2, p3, 0, c2, c3) - ex)
    e1 = abs(ff.farfield(x, p2, p3, 1, c2, c3) - ex)
    assert e1 < 0.5 * e0


@pytest.mark.parametrize("p", [0, 2, 3])
def test_homogeneity(p):
    x, p2, p3, _ = three_nodes(8)
    s = 2.0 ** 3
    a = ff.farfield(x, p2, p3, p)
    b = ff.farfield(s * x, s * p2, s * p3, p)
    assert b == pytest.approx(a * s ** -9, rel=1e-12)
