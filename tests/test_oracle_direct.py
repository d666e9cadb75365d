"""Pins of the exact-sum oracle (Section 1) against facts fixed by the
mathematics: closed-form triangles, an independent brute force, the energy
identity, invariances and the degenerate sizes."""
import math

import numpy as np
import pytest

import workloads
from oracle import direct


def test_equilateral_closed_form():
    # every angle 60 deg: 1 + 3/8 = 11/8, over d^9
    for d in (1.0, 2.0, 0.7):
        s = math.sqrt(3.0) / 2.0
        got = direct.at_phi([0, 0, 0], [d, 0, 0], [d / 2, d * s, 0])
        assert got == pytest.approx(11.0 / (8.0 * d ** 9), rel=1e-14)


def test_right_angle_closed_form():
    # right angle at x_i: cos t_i = 0, phi = 1 / (r_ij r_ik r_jk)^3
    xi, xj, xk = [0, 0, 0], [3.0, 0, 0], [0, 4.0, 0]
    assert direct.at_phi(xi, xj, xk) == pytest.approx(1.0 / (3.0 * 4.0 * 5.0) ** 3, rel=1e-14)
    # the right angle may sit at any vertex
    assert direct.at_phi(xj, xi, xk) == pytest.approx(1.0 / (3.0 * 4.0 * 5.0) ** 3, rel=1e-14)


def test_collinear_closed_form():
    # collinear: cosines +1, +1, -1 -> 1 - 3 = -2
    got = direct.at_phi([0, 0, 0], [1.0, 0, 0], [-2.5, 0, 0])
    assert got == pytest.approx(-2.98542274052478e-3, rel=1e-12)
    assert got == pytest.approx(-2.0 / (1.0 * 2.5 * 3.5) ** 3, rel=1e-14)


def test_phi_symmetric_and_invariant():
    g = np.random.default_rng(0)
    for _ in range(20):
        p = g.normal(size=(3, 3))
        v = direct.at_phi(*p)
        for perm in ((1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0)):
            assert direct.at_phi(*p[list(perm)]) == pytest.approx(v, rel=1e-13)
        # rigid motion
        q, _ = np.linalg.qr(g.normal(size=(3, 3)))
        t = g.normal(size=3)
        assert direct.at_phi(*(p @ q.T + t)) == pytest.approx(v, rel=1e-11, abs=1e-13 * abs(v))
        # scaling by 2^k multiplies phi by 2^(-9k) exactly
        assert direct.at_phi(*(p * 4.0)) == v * 2.0 ** -18


def test_small_n():
    assert direct.phi(np.zeros((0, 3))).shape == (0,)
    assert np.all(direct.phi(np.array([[0.0, 0, 0]])) == 0.0)
    assert np.all(direct.phi(np.array([[0.0, 0, 0], [1.0, 0, 0]])) == 0.0)
    p = np.array([[0.0, 0, 0], [1.0, 0.2, 0], [0.3, 1.1, 0.4]])
    v = direct.at_phi(*p)
    np.testing.assert_allclose(direct.phi(p), [v, v, v], rtol=1e-15)


@pytest.mark.parametrize("n,seed", [(4, 1), (5, 2), (6, 3), (8, 4)])
def test_bruteforce_independent_formula(n, seed):
    x = workloads.rng(seed).normal(size=(n, 3))
    np.testing.assert_allclose(direct.phi(x), direct.phi_bruteforce(x), rtol=1e-12)


def test_energy_identity():
    x = workloads.jittered_lattice(216, seed=5)
    assert direct.phi(x).sum() == pytest.approx(3.0 * direct.energy(x), rel=1e-13)


def test_permutation_equivariance():
    x = workloads.jittered_lattice(120, seed=6)
    p = workloads.rng(7).permutation(120)
    np.testing.assert_allclose(direct.phi(x[p]), direct.phi(x)[p], rtol=1e-13)


def test_scaling_exact():
    x = workloads.jittered_lattice(64, seed=8)
    np.testing.assert_array_equal(direct.phi(x * 2.0), direct.phi(x) * 2.0 ** -9)


def test_sampled_equals_all():
    x = workloads.jittered_lattice(100, seed=9)
    idx = np.array([0, 7, 50, 99])
    np.testing.assert_array_equal(direct.phi(x, idx), direct.phi(x)[idx])


def test_split_sums_add_up():
    x = workloads.jittered_lattice(125, seed=10)
    far = direct.phi_split(x, 1.5, True)
    near = direct.phi_split(x, 1.5, False)
    np.testing.assert_allclose(far + near, direct.phi(x), rtol=1e-13)
    assert np.all(np.abs(near) > 0)


def test_lattice_generator():
    x = workloads.jittered_lattice(512, seed=1)
    assert x.shape == (512, 3)
    d = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)) + np.eye(512) * 9
    assert d.min() >= 0.5
    assert np.all(np.abs(x - np.rint(x)) <= 0.25)
    assert workloads.jittered_lattice(1000, 3).shape == (1000, 3)


def test_factorized_identity_matches_direct():
    # the law-of-cosines product form is an identity: same sum, FP64
    from oracle import factorized

    for n, seed in ((7, 1), (40, 2)):
        x = workloads.rng(seed).normal(size=(n, 3)) * 2.0
        np.testing.assert_allclose(factorized.phi(x), direct.phi(x), rtol=1e-11)
    x = workloads.jittered_lattice(216, seed=3)
    ref = direct.phi(x)
    for r_near in (0.0, 1.5, 2.5):
        np.testing.assert_allclose(factorized.phi(x, r_near), ref, rtol=1e-12)
        np.testing.assert_allclose(factorized.phi_far(x, r_near),
                                   direct.phi_split(x, r_near, far=True), rtol=1e-10,
                                   atol=1e-14 * np.abs(ref).max())


def test_factorized_coefficients_equilateral():
    # equilateral triangle: the six sums reproduce 11/8 d^-9 for each vertex
    from oracle import factorized

    s = np.sqrt(3.0) / 2.0
    x = np.array([[0, 0, 0], [2.0, 0, 0], [1.0, 2 * s, 0]])
    np.testing.assert_allclose(factorized.phi(x), [11 / 8 / 2 ** 9] * 3, rtol=1e-14)
