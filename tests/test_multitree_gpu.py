"""The HIP kd-tree and triple-tree traversal against the CPU oracle.

Tree: bit-exact permutation, node ranges and boxes (index and min/max
work), centroids to rounding.  Traversal: with eps = 0 and alpha = 0 it
reduces to the exhaustive sum; every point is credited exactly C(N-1, 2)
tuples; with alpha = 0 every point meets eps (Theorem 5.1); with alpha > 0
at least a 1 - alpha fraction does (Theorem 5.2)."""
import math

import numpy as np
import pytest

import workloads
from oracle import direct as oracle_direct
from oracle import kdtree as oracle_kdtree

pytestmark = pytest.mark.gpu


def dev(x, cuda):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).to(cuda)


def clustered(n_per, centers, seed, spread=1.0):
    """Jittered-lattice blobs (spacing 1.0) translated to the given centers."""
    parts = [workloads.jittered_lattice(n_per, seed=seed + q) * spread + np.asarray(c)
             for q, c in enumerate(centers)]
    return np.concatenate(parts)


CENTERS8 = [(0, 0, 0), (40, 0, 0), (0, 40, 0), (0, 0, 40), (40, 40, 0), (40, 0, 40), (0, 40, 40),
            (40, 40, 40)]


@pytest.mark.parametrize("case", ["lattice1000_32", "mixture3000_32", "uniform777_8", "lattice64_32",
                                  "tiny5_1", "lattice300_7"])
def test_tree_matches_oracle(case, cuda):
    import paper_1105_2769_amd as mb

    x = {"lattice1000_32": lambda: workloads.jittered_lattice(1000, 3),
         "mixture3000_32": lambda: workloads.saturated_gaussian_mixture(3000, 5, components=6,
                                                                         box=40.0),
         "uniform777_8": lambda: workloads.uniform_cube(777, 4),
         "lattice64_32": lambda: workloads.jittered_lattice(64, 5),
         "tiny5_1": lambda: workloads.uniform_cube(5, 6),
         "lattice300_7": lambda: workloads.jittered_lattice(300, 7)}[case]()
    leaf = int(case.split("_")[1])
    print(f"tree {case}", flush=True)
    t = mb.KdTree(dev(x, cuda), leaf)
    g = t.export()
    o = oracle_kdtree.build_kdtree(x, leaf)
    assert t.n_nodes == o.n_nodes
    np.testing.assert_array_equal(g["perm"], o.perm)
    np.testing.assert_array_equal(g["begin"], o.begin)
    np.testing.assert_array_equal(g["end"], o.end)
    np.testing.assert_array_equal(g["left"], o.left)
    np.testing.assert_array_equal(g["right"], o.right)
    np.testing.assert_array_equal(g["lo"], o.lo)
    np.testing.assert_array_equal(g["hi"], o.hi)
    np.testing.assert_allclose(g["centroid"], o.centroid, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("n,leaf", [(3, 32), (20, 32), (130, 8), (513, 32), (700, 16)])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32c", 1e-5)])
def test_eps0_is_exhaustive(n, leaf, prec, tol, cuda):
    import paper_1105_2769_amd as mb

    x = workloads.jittered_lattice(n, seed=20 + n)
    ref = oracle_direct.phi(x)
    print(f"eps0 n={n} leaf={leaf} {prec}", flush=True)
    phi, st, cov = mb.eval_multitree(dev(x, cuda), eps=0.0, alpha=0.0, leaf_size=leaf,
                                     coverage=True, base_prec=prec)
    got = phi.cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=tol, atol=tol * np.abs(ref).max())
    assert np.all(cov.cpu().numpy() == (n - 1) * (n - 2) // 2)
    assert st["det_prunes"] == 0 and st["mc_prunes"] == 0
    # nothing pruned: the base cases hold every triple exactly once, and the
    # statistics counters (summed per workgroup on the device) say so
    assert st["base_triples"] == n * (n - 1) * (n - 2) // 6
    assert st["visited"] >= st["base_cases"] > 0


def test_small_n(cuda):
    import paper_1105_2769_amd as mb

    for n in (1, 2):
        phi, st = mb.eval_multitree(dev(workloads.uniform_cube(n, 1), cuda), leaf_size=8)
        assert np.all(phi.cpu().numpy() == 0.0)


def test_deterministic_guarantee(cuda):
    # eight separated blobs: far triples of blobs are pruned by the bound
    import paper_1105_2769_amd as mb

    x = clustered(216, CENTERS8, seed=30)
    n = x.shape[0]
    idx = workloads.sample_indices(n, 96, seed=31)
    ref = oracle_direct.phi(x, idx)
    for eps in (0.1, 1e-2):
        print(f"deterministic eps={eps}", flush=True)
        phi, st, cov = mb.eval_multitree(dev(x, cuda), eps=eps, alpha=0.0, leaf_size=16,
                                         coverage=True, base_prec="fp64")
        rel = np.abs(phi.cpu().numpy()[idx] - ref) / np.abs(ref)
        print(eps, st, rel.max())
        assert st["det_prunes"] > 0
        assert rel.max() <= eps
        assert np.all(cov.cpu().numpy() == (n - 1) * (n - 2) // 2)


def test_absolute_and_hybrid_guarantee(cuda):
    # absolute (eps = 0, tau > 0) and hybrid (both) bounds, deterministic:
    # every point within eps |Phi| + tau (Definitions 2.1 and 2.3)
    import paper_1105_2769_amd as mb

    x = clustered(216, CENTERS8, seed=30)
    n = x.shape[0]
    idx = workloads.sample_indices(n, 96, seed=31)
    ref = oracle_direct.phi(x, idx)
    scale = float(np.abs(ref).max())
    for eps, tau in ((0.0, 1e-2 * scale), (1e-2, 1e-3 * scale)):
        print(f"eps={eps} tau={tau:.3e}", flush=True)
        phi, st, cov = mb.eval_multitree(dev(x, cuda), eps=eps, tau_abs=tau, alpha=0.0,
                                         leaf_size=16, coverage=True, base_prec="fp64")
        err = np.abs(phi.cpu().numpy()[idx] - ref)
        print(st, float((err / (eps * np.abs(ref) + tau)).max()))
        assert st["det_prunes"] > 0
        assert np.all(err <= eps * np.abs(ref) + tau)
        assert np.all(cov.cpu().numpy() == (n - 1) * (n - 2) // 2)


def test_partial_chunks(cuda):
    # a round chunk far below the stack size: rounds pop part of the stack,
    # and the result keeps its guarantee and its exact coverage
    import paper_1105_2769_amd as mb

    x = clustered(216, CENTERS8, seed=30)
    n = x.shape[0]
    idx = workloads.sample_indices(n, 96, seed=31)
    ref = oracle_direct.phi(x, idx)
    runs = {}
    for chunk in (64, 1 << 20):
        phi, st, cov = mb.eval_multitree(dev(x, cuda), eps=1e-2, alpha=0.0, leaf_size=16,
                                         coverage=True, base_prec="fp64", chunk=chunk)
        rel = np.abs(phi.cpu().numpy()[idx] - ref) / np.abs(ref)
        print(chunk, st, rel.max())
        assert rel.max() <= 1e-2
        assert np.all(cov.cpu().numpy() == (n - 1) * (n - 2) // 2)
        runs[chunk] = st
    assert runs[64]["rounds"] > runs[1 << 20]["rounds"]


def test_monte_carlo_guarantee(cuda):
    import paper_1105_2769_amd as mb

    x = clustered(512, CENTERS8[:6], seed=40, spread=1.0)
    n = x.shape[0]
    idx = workloads.sample_indices(n, 128, seed=41)
    ref = oracle_direct.phi(x, idx)
    eps, alpha = 1e-2, 0.05
    # zeta 4 (the library default is 128) so that the Monte Carlo prune runs
    # on node triples of this size
    phi, st, cov = mb.eval_multitree(dev(x, cuda), eps=eps, alpha=alpha, leaf_size=32,
                                     coverage=True, seed=7, zeta=4.0)
    rel = np.abs(phi.cpu().numpy()[idx] - ref) / np.abs(ref)
    frac = float(np.mean(rel <= eps))
    print("mc", st, "fraction within eps", frac, "max", rel.max())
    assert st["mc_prunes"] > 0
    # every point of a pruned node triple drew at least m_min = 30 samples
    assert st["mc_samples"] >= 30 * st["mc_prunes"]
    assert frac >= 1 - alpha
    assert np.all(cov.cpu().numpy() == (n - 1) * (n - 2) // 2)


def test_tree_reuse_same_result(cuda):
    import paper_1105_2769_amd as mb

    x = clustered(125, CENTERS8[:4], seed=50)
    xt = dev(x, cuda)
    t = mb.KdTree(xt, 16)
    a, _ = mb.eval_multitree(xt, eps=1e-2, alpha=0.0, leaf_size=16, tree=t, base_prec="fp64")
    b, _ = mb.eval_multitree(xt, eps=1e-2, alpha=0.0, leaf_size=16, base_prec="fp64")
    np.testing.assert_allclose(a.cpu().numpy(), b.cpu().numpy(), rtol=1e-12)


def test_errors(cuda):
    import paper_1105_2769_amd as mb

    x = workloads.jittered_lattice(100, 1)
    d = x.copy()
    d[7] = d[3]
    with pytest.raises(mb.MBError) as e:
        mb.eval_multitree(dev(d, cuda), leaf_size=8)
    assert e.value.status == 2
    t = mb.KdTree(dev(x, cuda), 8)
    with pytest.raises(mb.MBError):
        mb.eval_multitree(dev(workloads.jittered_lattice(50, 1), cuda), tree=t)


@pytest.mark.parametrize("alpha", [0.0, 0.05])
def test_magnitude_bound_on_sign_indefinite_mixture(alpha, cuda):
    # The Gaussian-mixture generator at N = 8192: 12 % of the points have
    # Phi < 0, so the paper's running lower bound stays negative and prunes
    # nothing; the magnitude statistic prunes most of the work and every
    # sampled point stays within eps (against the CPU oracle).
    import paper_1105_2769_amd as mb

    x = workloads.saturated_gaussian_mixture(8192, seed=3)
    n = x.shape[0]
    idx = workloads.sample_indices(n, 48, seed=33)
    ref = oracle_direct.phi(x, idx)
    assert np.mean(ref < 0) > 0.0
    eps = 1e-2
    phi, st, cov = mb.eval_multitree(dev(x, cuda), eps=eps, alpha=alpha, leaf_size=32,
                                     coverage=True, bound="magnitude", seed=11)
    rel = np.abs(phi.cpu().numpy()[idx] - ref) / np.abs(ref)
    frac_exh = st["base_triples"] / (n * (n - 1) * (n - 2) / 6)
    print(f"magnitude alpha={alpha}: {st} within eps {np.mean(rel <= eps):.3f} max {rel.max():.2e} "
          f"exhaustive fraction {frac_exh:.3f}")
    assert st["det_prunes"] > 0 and frac_exh < 0.5
    assert np.mean(rel <= eps) >= 1 - max(alpha, 0.0) and (alpha > 0 or rel.max() <= eps)
    assert np.all(cov.cpu().numpy() == (n - 1) * (n - 2) // 2)
    # the paper's signed statistic on the same points: exact, nothing pruned
    _, st2 = mb.eval_multitree(dev(x, cuda), eps=eps, alpha=0.0, leaf_size=32)
    assert st2["base_triples"] / (n * (n - 1) * (n - 2) / 6) > 0.9


@pytest.mark.parametrize("bound", ["signed", "magnitude"])
def test_eps0_exact_either_bound(bound, cuda):
    import paper_1105_2769_amd as mb

    x = workloads.saturated_gaussian_mixture(1500, seed=8)
    ref = oracle_direct.phi(x)
    phi, st, cov = mb.eval_multitree(dev(x, cuda), eps=0.0, alpha=0.0, leaf_size=16,
                                     coverage=True, bound=bound, base_prec="fp64")
    # binary64 rounding, measured against the largest |Phi| for the points
    # whose Phi nearly cancels to zero
    np.testing.assert_allclose(phi.cpu().numpy(), ref, rtol=1e-11, atol=1e-14 * np.abs(ref).max())
    assert np.all(cov.cpu().numpy() == (1500 - 1) * (1500 - 2) // 2)


def test_mixture_262144_oracle_samples(cuda):
    """Full-size parity: the N = 262144 saturated Gaussian mixture at the
    settings the benchmark times (relative eps 1e-2, alpha 0.05, leaf 32,
    FP32C base cases, magnitude bound), against the oracle's Phi at 64
    seeded-sampled points stored in tests/golden (Theorem 5.2: at least a
    1 - alpha fraction within eps)."""
    import json
    import os

    import paper_1105_2769_amd as mb

    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "c3_direct_samples.json")))
    n = g["n"]
    print(f"mixture n={n}: generating", flush=True)
    x = workloads.saturated_gaussian_mixture(n, seed=3)
    idx = np.array(g["indices"])
    ref = np.array([float(v) for v in g["phi"]])
    print(f"mixture n={n}: traversal", flush=True)
    phi, st = mb.eval_multitree(dev(x, cuda), eps=1e-2, alpha=0.05, leaf_size=32,
                                bound="magnitude", base_prec="fp32c")
    rel = np.abs(phi.cpu().numpy()[idx] - ref) / np.abs(ref)
    frac = float(np.mean(rel <= 1e-2))
    print("mixture", st, "fraction within eps", frac, "max", rel.max(), flush=True)
    assert frac >= 0.95
    assert st["det_prunes"] > 0 and st["mc_prunes"] > 0
    assert 0 < st["base_triples"] < n * (n - 1) * (n - 2) // 6
