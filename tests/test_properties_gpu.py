"""Property tests on random small point sets (hypothesis): the exhaustive
sum (N from 3 to 64) on every path against the binary64 oracle, and the
symmetries of Phi - permutation equivariance, invariance under rotation and
translation, and homogeneity of degree -9 under scaling by 2^k; the
triple-tree traversal (N up to 300, any leaf size) exact at eps = 0 and
within its deterministic bound (alpha = 0, Theorem 5.1) at every point for
eps > 0, with every triple covered exactly once.

Error scale: a particle's bar is relative to M_i = sum over its triangles of
|phi| (the size of the terms being summed; Phi_i itself may cancel):
1e-12 M_i for the binary64 paths, 1e-6 M_i for FP32C.  M_i is computed here
in numpy only to size the bar, never as an expected value."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import workloads
from oracle import direct as oracle

pytestmark = pytest.mark.gpu

SETTINGS = settings(max_examples=25, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.function_scoped_fixture])


def points(kind, n, seed):
    if kind == "lattice":
        return workloads.jittered_lattice(n, seed=seed)
    if kind == "cube":
        return workloads.uniform_cube(n, seed=seed)
    return workloads.unit_ball(n, seed=seed)


def magnitude(x):
    """M_i = sum over j < k (j, k != i) of |phi(x_i, x_j, x_k)|."""
    n = x.shape[0]
    d = x[:, None, :] - x[None, :, :]
    r2 = np.einsum("ijc,ijc->ij", d, d)
    np.fill_diagonal(r2, 1.0)
    r = np.sqrt(r2)
    m = np.zeros(n)
    for i in range(n):
        ci = np.einsum("jc,kc->jk", d[:, i, :], d[:, i, :]) / np.outer(r[:, i], r[:, i])  # cos at i
        a, b, c = r[i][:, None], r[i][None, :], r
        cj = (a ** 2 + c ** 2 - b ** 2) / (2 * a * c)  # cos at j
        ck = (b ** 2 + c ** 2 - a ** 2) / (2 * b * c)  # cos at k
        phi = (1 + 3 * ci * cj * ck) / (a * b * c) ** 3
        mask = np.triu(np.ones((n, n), bool), 1)
        mask[i, :] = mask[:, i] = False
        m[i] = np.abs(phi[mask]).sum()
    return m


def gpu(x, path, cuda):
    import torch

    import paper_1105_2769_amd as mb

    xt = torch.from_numpy(np.ascontiguousarray(x)).to(cuda)
    if path == "det":
        return mb.eval_direct_deterministic(xt).cpu().numpy()
    return mb.eval_direct(xt, prec=path).cpu().numpy()


TOL = {"fp64": 1e-12, "det": 1e-12, "fp32c": 1e-6}
sets = st.tuples(st.sampled_from(["lattice", "cube", "ball"]), st.integers(3, 64),
                 st.integers(0, 2 ** 31 - 1))


@SETTINGS
@given(case=sets)
def test_every_path_matches_oracle(case, cuda):
    kind, n, seed = case
    x = points(kind, n, seed)
    print(f"properties: oracle {kind} N={n} seed={seed}", flush=True)
    ref = oracle.phi(x)
    mag = magnitude(x)
    for path, tol in TOL.items():
        err = np.abs(gpu(x, path, cuda) - ref)
        assert np.all(err <= tol * mag), (path, float(np.max(err / mag)))


@SETTINGS
@given(case=sets, k=st.integers(-3, 3), data=st.data())
def test_symmetries(case, k, data, cuda):
    kind, n, seed = case
    x = points(kind, n, seed)
    print(f"properties: symmetries {kind} N={n} seed={seed} k={k}", flush=True)
    g = workloads.rng(seed ^ 0x5EED)
    mag = magnitude(x)
    for path in ("fp64", "det"):
        base = gpu(x, path, cuda)
        # permutation equivariance
        p = g.permutation(n)
        assert np.all(np.abs(gpu(x[p], path, cuda) - base[p]) <= 1e-13 * mag[p])
        # rotation (orthogonal factor of a Gaussian matrix) and translation
        q, _ = np.linalg.qr(g.standard_normal((3, 3)))
        assert np.all(np.abs(gpu(x @ q.T, path, cuda) - base) <= 1e-11 * mag)
        shift = np.array(data.draw(st.tuples(*[st.floats(-8, 8)] * 3)))
        assert np.all(np.abs(gpu(x + shift, path, cuda) - base) <= 1e-10 * mag)
        # Phi(2^k x) = 2^(-9k) Phi(x): every pair term scales by a power of two
        s = 2.0 ** k
        assert np.all(np.abs(gpu(x * s, path, cuda) * s ** 9 - base) <= 1e-14 * mag)


@SETTINGS
@given(kind=st.sampled_from(["lattice", "cube", "ball"]), n=st.integers(3, 300),
       seed=st.integers(0, 2 ** 31 - 1), leaf=st.sampled_from([1, 2, 5, 16, 32]),
       eps=st.sampled_from([0.0, 1e-2, 0.1]))
def test_traversal_properties(kind, n, seed, leaf, eps, cuda):
    import torch

    import paper_1105_2769_amd as mb

    x = points(kind, n, seed)
    print(f"properties: traversal {kind} N={n} seed={seed} leaf={leaf} eps={eps}", flush=True)
    ref = oracle.phi(x)
    mag = magnitude(x)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(cuda)
    phi, st_, cov = mb.eval_multitree(xt, eps=eps, alpha=0.0, leaf_size=leaf, coverage=True,
                                      base_prec="fp64")
    bar = eps * np.abs(ref) + 1e-12 * mag
    ratio = np.abs(phi.cpu().numpy() - ref) / bar
    assert np.all(cov.cpu().numpy() == (n - 1) * (n - 2) // 2)
    assert np.all(ratio <= 1.0), float(ratio.max())
