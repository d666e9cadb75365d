"""Parity of the HIP exhaustive sum (mb_eval_direct) with the CPU oracle.

Tolerances: relative error <= 1e-12 per particle for binary64 and <= 1e-5
for the binary32-compensated path (both against the binary64 oracle)."""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import direct as oracle

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {"fp64": 1e-12, "fp32c": 1e-5}


def run(x, prec, cuda):
    import torch

    import paper_1105_2769_amd as mb

    print(f"direct {prec} N={x.shape[0]}", flush=True)
    return mb.eval_direct(torch.from_numpy(np.ascontiguousarray(x)).to(cuda), prec=prec).cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_c1_all_particles(prec, cuda):
    x = workloads.jittered_lattice(512, seed=1)
    ref = oracle.phi(x)
    got = run(x, prec, cuda)
    rel = np.abs(got - ref) / np.abs(ref)
    print(f"C1 {prec}: max rel err {rel.max():.3e}")
    assert rel.max() <= TOL[prec]


@pytest.mark.parametrize("n", [3, 4, 5, 63, 64, 65, 127, 128, 129, 191, 257, 700, 1000])
@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_ragged_sizes(n, prec, cuda):
    x = workloads.jittered_lattice(n, seed=100 + n)
    ref = oracle.phi(x)
    got = run(x, prec, cuda)
    np.testing.assert_allclose(got, ref, rtol=TOL[prec], atol=TOL[prec] * np.abs(ref).max())


def test_uniform_cube_signed_terms(cuda):
    # uniform points: many near-degenerate triangles, sums of mixed sign
    x = workloads.uniform_cube(300, seed=3)
    ref = oracle.phi(x)
    got = run(x, "fp64", cuda)
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


def test_empty_and_tiny(cuda):
    for n in (0, 1, 2):
        x = workloads.jittered_lattice(n, seed=1) if n else np.zeros((0, 3))
        got = run(x, "fp64", cuda)
        assert got.shape == (n,) and np.all(got == 0.0)


def test_errors(cuda):
    import paper_1105_2769_amd as mb

    x = workloads.jittered_lattice(100, seed=1)
    bad = x.copy()
    bad[17, 1] = np.nan
    with pytest.raises(mb.MBError) as e:
        run(bad, "fp64", cuda)
    assert e.value.status == 1
    dup = x.copy()
    dup[40] = dup[3]
    with pytest.raises(mb.MBError) as e:
        run(dup, "fp64", cuda)
    assert e.value.status == 2
    with pytest.raises(ValueError):
        run(x, "fp16", cuda)


def test_validate_reports_min_distance(cuda):
    import torch

    import paper_1105_2769_amd as mb

    x = workloads.jittered_lattice(300, seed=4)
    d2 = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1) + np.eye(300) * 1e9
    md2, fin, box = mb.validate(torch.from_numpy(x).to(cuda))
    assert fin and md2 == pytest.approx(d2.min(), rel=1e-15)
    np.testing.assert_array_equal(box, np.concatenate([x.min(0), x.max(0)]))
    y = x - 3.0  # negative coordinates too
    _, _, box = mb.validate(torch.from_numpy(y).to(cuda))
    np.testing.assert_array_equal(box, np.concatenate([y.min(0), y.max(0)]))


def test_scaling_and_translation(cuda):
    x = workloads.jittered_lattice(343, seed=11)
    base = run(x, "fp64", cuda)
    np.testing.assert_allclose(run(x * 2.0, "fp64", cuda), base * 2.0 ** -9, rtol=1e-13)
    np.testing.assert_allclose(run(x + 1000.0, "fp64", cuda), base, rtol=1e-9)


def test_fp32c_falls_back_to_fp64_on_wide_range(cuda):
    # two lattice clusters 1e5 apart: extent / closest pair > 2^16, so the
    # binary32 path hands over to binary64 and meets the binary64 bar
    a = workloads.jittered_lattice(125, seed=12)
    x = np.concatenate([a, workloads.jittered_lattice(125, seed=13) + 1e5])
    ref = oracle.phi(x)
    got = run(x, "fp32c", cuda)
    rel = np.abs(got - ref) / np.abs(ref)
    print(f"fallback case: max rel err {rel.max():.3e}")
    assert rel.max() <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_c2_sampled(prec, cuda):
    g = json.load(open(os.path.join(HERE, "golden", "c2_direct_samples.json")))
    x = workloads.jittered_lattice(g["n"], seed=2)
    idx = np.array(g["indices"])
    assert np.array_equal(idx, workloads.sample_indices(g["n"], 64, seed=g["sample_seed"]))
    ref = np.array([float(v) for v in g["phi"]])
    got = run(x, prec, cuda)[idx]
    rel = np.abs(got - ref) / np.abs(ref)
    print(f"C2 {prec}: max rel err {rel.max():.3e} mean {rel.mean():.3e}")
    assert rel.max() <= TOL[prec]


@pytest.mark.parametrize("n,seed", [(4096, 2), (32768, 2)])
def test_fp32c_every_particle_within_1e6(n, seed, cuda):
    # Every particle of the binary32 path against the binary64 path, which the
    # oracle pins to 1e-12 on the same points (C1, C2 samples above).  The
    # near-field refinement is what brings the worst (smallest-|Phi|, surface)
    # particles under the bar.
    x = workloads.jittered_lattice(n, seed=seed)
    f64 = run(x, "fp64", cuda)
    f32 = run(x, "fp32c", cuda)
    rel = np.abs(f32 - f64) / np.abs(f64)
    print(f"N={n}: fp32c vs fp64 max rel {rel.max():.3e} at phi {f64[np.argmax(rel)]:.4g}")
    assert rel.max() <= 1e-6


def test_fp32c_falls_back_for_close_pairs(cuda):
    # uniform random points have pairs far closer than the mean spacing; the
    # thin triangles they make lose bits in binary32, so FP32C hands over to
    # binary64 and meets the binary64 bar
    x = workloads.uniform_cube(3000, seed=12) * 20.0
    f64 = run(x, "fp64", cuda)
    f32 = run(x, "fp32c", cuda)
    rel = np.abs(f32 - f64) / np.abs(f64)
    print(f"uniform N=3000: fp32c vs fp64 max rel {rel.max():.3e}")
    assert rel.max() <= 1e-12
