"""Parity of the factorized (MFMA) form with the CPU oracle.

Bars: relative error <= 1e-6 per particle for the two-plane FP16 and BF16
forms with the near-field split (r_near = 1.5 on the unit lattice), which
is the accuracy the product form has to reach to replace the exhaustive
sum; the one-plane forms are checked only against looser, documented bars.
"""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import direct as oracle_direct
from oracle import factorized as oracle_factorized

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def run(x, cuda, **kw):
    import torch

    import paper_1105_2769_amd as mb

    print(f"factorized N={x.shape[0]} {kw}", flush=True)
    phi, st = mb.eval_factorized(torch.from_numpy(np.ascontiguousarray(x)).to(cuda), **kw)
    return phi.cpu().numpy(), st


@pytest.mark.parametrize("fmt,planes,tol", [("fp16", 2, 1e-6), ("bf16", 2, 1e-6), ("fp16", 3, 1e-7),
                                            ("bf16", 3, 1e-7), ("fp16", 1, 1e-4), ("bf16", 1, 2e-3)])
def test_lattice_all_particles(fmt, planes, tol, cuda):
    x = workloads.jittered_lattice(1000, seed=4)
    ref = oracle_direct.phi(x)
    got, st = run(x, cuda, fmt=fmt, planes=planes, r_near=1.5)
    rel = np.abs(got - ref) / np.abs(ref)
    print(f"{fmt} planes={planes}: max rel {rel.max():.3e}")
    assert rel.max() <= tol
    assert st["near_pairs"] > 0


@pytest.mark.parametrize("n", [3, 4, 50, 127, 128, 129, 300])
def test_ragged_and_tiny(n, cuda):
    x = workloads.jittered_lattice(n, seed=60 + n)
    ref = oracle_direct.phi(x)
    got, _ = run(x, cuda, fmt="fp16", planes=2, r_near=1.5)
    np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-6 * np.abs(ref).max())


def test_no_near_split_matches_oracle_product_form(cuda):
    # r_near = 0: everything goes through the matrices; the oracle's FP64
    # product form (pinned against the direct sum in the CPU tests) is the bar
    x = workloads.jittered_lattice(343, seed=7)
    ref = oracle_factorized.phi(x, 0.0)
    got, st = run(x, cuda, fmt="fp16", planes=3, r_near=0.0)
    assert st["near_pairs"] == 0
    np.testing.assert_allclose(got, ref, rtol=2e-6)


def test_uniform_cube_scaled(cuda):
    # non-lattice input; r_near scales with the data
    x = workloads.uniform_cube(400, seed=8) * 7.0
    ref = oracle_direct.phi(x)
    got, _ = run(x, cuda, fmt="fp16", planes=2, r_near=1.2)
    rel = np.abs(got - ref) / np.abs(ref)
    assert np.median(rel) <= 1e-6


def test_errors(cuda):
    import paper_1105_2769_amd as mb

    x = workloads.jittered_lattice(100, seed=1)
    for kw in ({"planes": 0}, {"planes": 4}, {"r_near": -1.0}):
        with pytest.raises(mb.MBError):
            run(x, cuda, **kw)
    with pytest.raises(KeyError):
        run(x, cuda, fmt="fp8")
    for n in (0, 1, 2):
        got, _ = run(workloads.jittered_lattice(max(n, 1), 1)[:n], cuda)
        assert np.all(got == 0.0)


@pytest.mark.parametrize("fmt", ["fp16", "bf16"])
def test_c4_sampled(fmt, cuda):
    path = os.path.join(HERE, "golden", "c4_direct_samples.json")
    if not os.path.exists(path):
        pytest.skip("stored oracle values for the N = 16384 lattice not generated")
    g = json.load(open(path))
    x = workloads.jittered_lattice(g["n"], seed=4)
    idx = np.array(g["indices"])
    ref = np.array([float(v) for v in g["phi"]])
    got, st = run(x, cuda, fmt=fmt, planes=2, r_near=1.5)
    rel = np.abs(got[idx] - ref) / np.abs(ref)
    print(f"C4 {fmt}: max rel {rel.max():.3e} gemm {st['gemm_ms']:.1f} ms")
    assert rel.max() <= 1e-6
