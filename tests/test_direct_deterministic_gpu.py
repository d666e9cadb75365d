"""The fixed-order exhaustive sum (mb_eval_direct_deterministic).

Against the binary64 oracle at 1e-12 relative per particle, as the atomic
binary64 path; against itself bitwise: repeated calls, a call on a second
stream while other work occupies the GPU, and the same split into stripes
give identical bits."""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import direct as oracle

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-12


def det(x, cuda, scratch_bytes=0):
    import torch

    import paper_1105_2769_amd as mb

    print(f"deterministic N={x.shape[0]} scratch={scratch_bytes}", flush=True)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(cuda)
    return mb.eval_direct_deterministic(xt, scratch_bytes=scratch_bytes).cpu().numpy()


@pytest.mark.parametrize("n", [3, 4, 63, 64, 65, 129, 257, 700])
def test_matches_oracle_ragged(n, cuda):
    x = workloads.jittered_lattice(n, seed=300 + n)
    ref = oracle.phi(x)
    got = det(x, cuda)
    np.testing.assert_allclose(got, ref, rtol=TOL, atol=TOL * np.abs(ref).max())


def test_c1_all_particles(cuda):
    x = workloads.jittered_lattice(512, seed=1)
    ref = oracle.phi(x)
    rel = np.abs(det(x, cuda) - ref) / np.abs(ref)
    print(f"C1 deterministic: max rel err {rel.max():.3e}")
    assert rel.max() <= TOL


def test_uniform_cube_signed_terms(cuda):
    x = workloads.uniform_cube(300, seed=3)
    ref = oracle.phi(x)
    got = det(x, cuda)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("n,scratch", [(1000, 0), (3000, 0), (3000, 1), (3000, 16 << 20)])
def test_bitwise_repeatable(n, scratch, cuda):
    x = workloads.uniform_cube(n, seed=7 + n)
    first = det(x, cuda, scratch)
    for _ in range(3):
        again = det(x, cuda, scratch)
        assert np.array_equal(first.view(np.uint64), again.view(np.uint64))


def test_stripes_agree_with_one_pass(cuda):
    # scratch_bytes = 1: one J block per stripe (47 stripes at N = 3000)
    x = workloads.uniform_cube(3000, seed=11)
    one = det(x, cuda, 0)
    many = det(x, cuda, 1)
    np.testing.assert_allclose(many, one, rtol=1e-13, atol=1e-13 * np.abs(one).max())


def test_same_bits_under_concurrent_load(cuda):
    # the atomic path's sums of the same points run on the default stream
    # while the fixed-order sum runs on a second one, so the units are
    # scheduled differently from a call on an idle GPU
    import torch

    import paper_1105_2769_amd as mb

    x = workloads.uniform_cube(4000, seed=5)
    idle = det(x, cuda)
    xt = torch.from_numpy(x).to(cuda)
    big = torch.from_numpy(workloads.uniform_cube(12000, seed=6)).to(cuda)
    side = torch.cuda.Stream(device=cuda)
    torch.cuda.synchronize()
    print("deterministic under load", flush=True)
    mb.eval_direct(big, prec="fp64", checked=False)
    with torch.cuda.stream(side):
        busy = mb.eval_direct_deterministic(xt)
    mb.eval_direct(big, prec="fp64", checked=False)
    torch.cuda.synchronize()
    assert np.array_equal(idle.view(np.uint64), busy.cpu().numpy().view(np.uint64))


def test_close_to_atomic_path(cuda):
    import torch

    import paper_1105_2769_amd as mb

    x = workloads.jittered_lattice(5000, seed=9)
    got = det(x, cuda)
    atomic = mb.eval_direct(torch.from_numpy(x).to(cuda), prec="fp64").cpu().numpy()
    np.testing.assert_allclose(got, atomic, rtol=1e-13, atol=1e-14 * np.abs(atomic).max())


def test_c2_sampled(cuda):
    g = json.load(open(os.path.join(HERE, "golden", "c2_direct_samples.json")))
    x = workloads.jittered_lattice(g["n"], seed=2)
    idx = np.array(g["indices"])
    ref = np.array([float(v) for v in g["phi"]])
    got = det(x, cuda)[idx]
    rel = np.abs(got - ref) / np.abs(ref)
    print(f"C2 deterministic: max rel err {rel.max():.3e}")
    assert rel.max() <= TOL


def test_errors(cuda):
    import torch

    import paper_1105_2769_amd as mb

    x = workloads.uniform_cube(50, seed=1)
    x[7] = np.nan
    with pytest.raises(mb.MBError) as e:
        det(x, cuda)
    assert e.value.status == 1
    x = workloads.uniform_cube(50, seed=1)
    x[9] = x[3]
    with pytest.raises(mb.MBError) as e:
        det(x, cuda)
    assert e.value.status == 2
    two = det(workloads.uniform_cube(2, seed=1), cuda)
    assert np.array_equal(two, np.zeros(2))
    empty = mb.eval_direct_deterministic(torch.zeros((0, 3), dtype=torch.float64, device=cuda))
    assert empty.numel() == 0
