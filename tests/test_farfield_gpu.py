"""The far-field expansion of Section 3.2 on the GPU against the CPU oracle.

mb_farfield_eval (the routine the traversal applies per point) is compared
value by value with oracle.farfield for orders 0, 1 and 2 on separated
source sets; the traversal with order 1 or 2 keeps its decisions (the prune
test does not depend on the order), its exact coverage and its eps bound.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import direct as oracle_direct
from oracle import farfield as oracle_ff

pytestmark = pytest.mark.gpu


def dev(x, cuda):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).to(cuda)


def source_sets(seed, sep=6.0, width=1.0, nx=40, ny=25, nz=18):
    rng = workloads.rng(seed)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    c = np.array([[0.0, 0, 0], [sep, 0, 0], [0.4 * sep, 1.1 * sep, 0]]) @ q.T
    x = rng.uniform(-width / 2, width / 2, size=(nx, 3)) + c[0]
    y = rng.uniform(-width / 2, width / 2, size=(ny, 3)) + c[1]
    z = rng.uniform(-width / 2, width / 2, size=(nz, 3)) + c[2]
    return x, y, z


@pytest.mark.parametrize("order", [0, 1, 2])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_farfield_eval_matches_oracle(order, seed, cuda):
    import paper_1105_2769_amd as mb

    x, y, z = source_sets(seed)
    got = mb.farfield_eval(dev(x, cuda), dev(y, cuda), dev(z, cuda), order).cpu().numpy()
    want = np.array([oracle_ff.farfield(xi, y, z, order) for xi in x])
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=0.0)
    # and the expansion is close to the exact sums it stands for
    ex = np.array([oracle_ff.exact(xi, y, z) for xi in x])
    rel = np.abs(got - ex) / np.abs(ex)
    assert rel.max() < (0.1 if order < 2 else 0.02)


def test_farfield_eval_errors(cuda):
    import paper_1105_2769_amd as mb

    x, y, z = source_sets(4)
    with pytest.raises(mb.MBError) as e:
        mb.farfield_eval(dev(x, cuda), dev(y, cuda), dev(z, cuda), 3)
    assert e.value.status == 5


def blobs(n_per, centers, seed):
    parts = [workloads.jittered_lattice(n_per, seed=seed + q) + np.asarray(c, float)
             for q, c in enumerate(centers)]
    return np.concatenate(parts)


def test_traversal_orders_keep_decisions_and_bound(cuda):
    import paper_1105_2769_amd as mb

    centers = [(0, 0, 0), (60, 0, 0), (0, 60, 0), (0, 0, 60), (60, 60, 0), (60, 0, 60),
               (0, 60, 60), (60, 60, 60)]
    x = blobs(216, centers, seed=60)
    n = x.shape[0]
    ref = oracle_direct.phi(x)
    runs = {}
    for order in (0, 1, 2):
        print(f"order {order}", flush=True)
        phi, st, cov = mb.eval_multitree(dev(x, cuda), eps=0.05, alpha=0.0, leaf_size=16,
                                         coverage=True, base_prec="fp64", order=order)
        rel = np.abs(phi.cpu().numpy() - ref) / np.abs(ref)
        print(order, st, "max", rel.max(), "mean", rel.mean(), flush=True)
        assert np.all(cov.cpu().numpy() == math.comb(n - 1, 2))
        assert rel.max() <= 0.05
        runs[order] = (st, rel)
    for order in (1, 2):
        for key in ("det_prunes", "base_triples", "visited"):
            assert runs[order][0][key] == runs[0][0][key]
    assert runs[0][0]["det_prunes"] > 0
