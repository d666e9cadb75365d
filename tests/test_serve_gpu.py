"""The serving loop on the GPU: results, admission, batching, completion.

Bars: each result equals the one-shot exhaustive sum of the same precision
to 1e-12 relative (the two differ only in the order of binary64 atomic
additions), and the oracle to 1e-12 (binary64 requests) or 1e-6 (binary32
requests).  "Alone equals mixed" is checked with small slices so that
requests share slices.
"""
import numpy as np
import pytest

import workloads
from oracle import direct as oracle_direct

pytestmark = pytest.mark.gpu


def server(**kw):
    import paper_1105_2769_amd as mb

    return mb.Server(**kw)


def chunk_bytes(n):
    """Device bytes of one request's chunk: 24 N (points) + 8 N (Phi) + 8 N
    (near-field magnitudes) + the larger (i, j) table of the two tile types,
    each part rounded up to 256.  The binary64 table is the larger one: I and
    J blocks of 64 points, (a, w) per pair in 8 bytes each."""
    up = lambda b: (b + 255) // 256 * 256
    blocks = -(-n // 64)
    return up(24 * n) + 2 * up(8 * n) + up(blocks * blocks * 64 * 64 * 2 * 8)


def one_shot(x, prec, cuda):
    import torch

    import paper_1105_2769_amd as mb

    return mb.eval_direct(torch.from_numpy(x).to(cuda), prec).cpu().numpy()


def oracle_check(x, got, tol, n_sample=48, seed=0):
    n = x.shape[0]
    if n <= 700:
        ref = oracle_direct.phi(x)
        np.testing.assert_allclose(got, ref, rtol=tol)
    else:
        idx = workloads.sample_indices(n, n_sample, seed)
        np.testing.assert_allclose(got[idx], oracle_direct.phi(x, idx), rtol=tol)


SIZES = [100, 333, 64, 1000, 2500, 777, 3, 129]


def test_alone_equals_mixed(cuda):
    pts = [workloads.jittered_lattice(n, seed=1_000_000 + r) for r, n in enumerate(SIZES)]
    print("serving: alone", flush=True)
    alone = []
    with server() as srv:
        for x in pts:
            rid = srv.submit(x)
            assert srv.wait(rid, 60_000)
            alone.append(srv.result(rid))
    print("serving: mixed", flush=True)
    with server() as srv:
        srv.set_slice_units(7)
        ids = [srv.submit(x) for x in pts]
        assert srv.wait(-1, 120_000)
        mixed = [srv.result(r) for r in ids]
        st = srv.stats()
    assert st["mixed_slices"] > 0
    assert st["completed"] == len(pts) and st["failed"] == 0
    for x, a, m in zip(pts, alone, mixed):
        np.testing.assert_allclose(m, a, rtol=1e-12)
        np.testing.assert_allclose(m, one_shot(x, "fp32c", cuda), rtol=1e-12)
        oracle_check(x, m, 1e-6)


def test_fp64_and_fp32c_requests_together(cuda):
    pts = [workloads.jittered_lattice(n, seed=70 + n) for n in (200, 450, 650)]
    with server() as srv:
        srv.set_slice_units(5)
        ids = [srv.submit(x, "fp64" if k % 2 == 0 else "fp32c") for k, x in enumerate(pts)]
        assert srv.wait(-1, 60_000)
        res = [srv.result(r) for r in ids]
    for k, (x, got) in enumerate(zip(pts, res)):
        oracle_check(x, got, 1e-12 if k % 2 == 0 else 1e-6)


def test_fp64_fallback_on_wide_range(cuda):
    # two clusters 1e5 apart: bounding box / closest pair > 2^16
    a = workloads.jittered_lattice(150, seed=3)
    x = np.concatenate([a, a[:100] + 1.0e5])
    with server() as srv:
        rid = srv.submit(x, "fp32c")
        assert srv.wait(rid, 60_000)
        got = srv.result(rid)
        assert srv.stats()["fp64_fallbacks"] == 1
    oracle_check(x, got, 1e-10)


def test_degenerate_tiny_and_invalid(cuda):
    import paper_1105_2769_amd as mb

    good = workloads.jittered_lattice(300, seed=9)
    bad = good.copy()
    bad[17] = bad[201]
    with server() as srv:
        ids = {"good": srv.submit(good), "bad": srv.submit(bad)}
        tiny = [srv.submit(np.zeros((n, 3))) for n in (0, 1, 2)]
        for k, n in enumerate((0, 1, 2)):
            assert srv.poll(tiny[k])
            assert np.all(srv.result(tiny[k]) == 0.0)  # n < 3: the empty sum
        with pytest.raises(mb.MBError):
            srv.submit(np.full((10, 3), np.nan))
        assert srv.wait(-1, 60_000)
        with pytest.raises(mb.MBError) as e:
            srv.result(ids["bad"])
        assert e.value.status == 2
        oracle_check(good, srv.result(ids["good"]), 1e-6)
        with pytest.raises(mb.MBError):
            srv.result(ids["good"])  # fetched once
        st = srv.stats()
    assert st["failed"] == 1 and st["completed"] == 4


def test_budget_admission(cuda):
    import paper_1105_2769_amd as mb

    n = 600
    need = chunk_bytes(n)
    with server(hbm_budget_bytes=need - 1) as srv:
        with pytest.raises(mb.MBError) as e:
            srv.submit(workloads.jittered_lattice(n, seed=1))
        assert e.value.status == 3
    pts = [workloads.jittered_lattice(n, seed=20 + r) for r in range(4)]
    with server(hbm_budget_bytes=need, max_slots=8) as srv:
        ids = [srv.submit(x) for x in pts]
        assert srv.wait(-1, 60_000)
        st = srv.stats()
        res = [srv.result(r) for r in ids]
    assert st["peak_active"] == 1 and st["peak_reserved"] <= need
    for x, got in zip(pts, res):
        np.testing.assert_allclose(got, one_shot(x, "fp32c", cuda), rtol=1e-12)


def test_budget_counts_whole_chunks(cuda):
    # A budget between one and two request chunks admits one request at a
    # time: a binary32 request keeps its whole chunk (sized for either tile
    # type) reserved until it is released, so the live chunks never exceed
    # the budget.
    import paper_1105_2769_amd as mb

    n = 600
    need = chunk_bytes(n)
    budget = need + need // 2
    pts = [workloads.jittered_lattice(n, seed=40 + r) for r in range(4)]
    with server(hbm_budget_bytes=budget, max_slots=8) as srv:
        ids = [srv.submit(x) for x in pts]
        assert srv.wait(-1, 60_000)
        st = srv.stats()
        res = [srv.result(r) for r in ids]
    assert st["peak_active"] == 1 and st["peak_reserved"] == need <= budget
    assert st["fp64_fallbacks"] == 0  # binary32 requests
    for x, got in zip(pts, res):
        np.testing.assert_allclose(got, one_shot(x, "fp32c", cuda), rtol=1e-12)


def test_many_small_requests_none_lost(cuda):
    g = workloads.rng(11)
    sizes = g.integers(3, 300, size=60)
    pts = [workloads.jittered_lattice(int(n), seed=500 + k) for k, n in enumerate(sizes)]
    with server(max_slots=7) as srv:
        srv.set_slice_units(3)
        ids = [srv.submit(x) for x in pts]
        assert srv.wait(-1, 120_000)
        st = srv.stats()
        res = [srv.result(r) for r in ids]
    assert st["completed"] == len(pts) and st["failed"] == 0
    assert st["peak_active"] <= 7
    for x, got in zip(pts, res):
        np.testing.assert_allclose(got, one_shot(x, "fp32c", cuda), rtol=1e-12)


def test_poisson_arrivals_latency(cuda):
    import time

    t, sizes = workloads.poisson_trace(40, seed=5, rate_hz=400.0, n_max=2048)
    pts = [workloads.jittered_lattice(int(n), seed=1_000_000 + r) for r, n in enumerate(sizes)]
    with server() as srv:
        t0 = time.perf_counter()
        ids = []
        for ta, x in zip(t, pts):
            while time.perf_counter() - t0 < ta:
                time.sleep(1e-4)
            ids.append(srv.submit(x))
        assert srv.wait(-1, 120_000)
        lat = np.array([srv.latency(r) for r in ids])
        res = [srv.result(r) for r in ids]
    assert np.all(lat > 0) and np.all(np.isfinite(lat))
    print(f"p50 {np.percentile(lat, 50) * 1e3:.2f} ms  p99 {np.percentile(lat, 99) * 1e3:.2f} ms")
    for k in (0, len(pts) // 2, len(pts) - 1):
        oracle_check(pts[k], res[k], 1e-6)


def test_full_trace_4096_requests(cuda):
    """Full-size parity of the serving loop: the 4096-request Poisson trace
    (200 requests/s, N log-uniform in [64, 8192], seed 5) replayed in real
    time through a server configured as the benchmark's, with every result
    finite and 8 seeded-sampled requests checked against the oracle."""
    import time

    t, sizes = workloads.poisson_trace(4096, seed=5, rate_hz=200.0, n_min=64, n_max=8192)
    pts = [workloads.jittered_lattice(int(n), seed=1_000_000 + r) for r, n in enumerate(sizes)]
    print("trace: replaying 4096 requests", flush=True)
    with server(hbm_budget_bytes=64 << 30, max_slots=512) as srv:
        t0 = time.perf_counter()
        ids = []
        for ta, x in zip(t, pts):
            while time.perf_counter() - t0 < ta:
                time.sleep(5e-4)
            ids.append(srv.submit(x))
        assert srv.wait(-1, 120_000)
        lat = np.array([srv.latency(r) for r in ids])
        res = [srv.result(r) for r in ids]
    assert np.all(lat > 0) and np.all(np.isfinite(lat))
    assert all(np.all(np.isfinite(v)) and v.shape == (x.shape[0],) for v, x in zip(res, pts))
    print(f"trace: p50 {np.percentile(lat, 50) * 1e3:.2f} ms  p99 "
          f"{np.percentile(lat, 99) * 1e3:.2f} ms", flush=True)
    for k in workloads.sample_indices(len(pts), 8, seed=56):
        oracle_check(pts[k], res[k], 1e-6, n_sample=16, seed=int(k))


def test_many_streams_do_not_stall_the_drain(cuda):
    """Regression: with many streams in the process, HIP maps several of
    them to one hardware queue.  The drain kernel, launched cooperatively,
    runs from a queue of its own, so the server's publishing copies and
    staging kernels never wait behind it: a 256-request burst (about
    7e10 triples) finishes within 6 s, against about 30 ms per request when
    a plain launch shared the publishing stream's queue, and matches the
    one-shot sums."""
    import time

    import torch

    extra = [torch.cuda.Stream(device=cuda) for _ in range(12)]  # noqa: F841
    g = workloads.rng(21)
    sizes = g.integers(64, 3000, size=256)
    pts = [workloads.jittered_lattice(int(n), seed=900 + k) for k, n in enumerate(sizes)]
    print("serving: 256 requests with 12 extra streams", flush=True)
    with server(max_slots=64) as srv:
        t0 = time.perf_counter()
        ids = [srv.submit(x) for x in pts]
        assert srv.wait(-1, 60_000)
        took = time.perf_counter() - t0
        st = srv.stats()
        res = [srv.result(r) for r in ids]
    print(f"burst of 256 requests: {took:.2f} s, {st['drain_launches']} drain launches", flush=True)
    assert st["completed"] == len(pts) and st["failed"] == 0
    assert took < 6.0
    for x, got in zip(pts[:16], res[:16]):
        np.testing.assert_allclose(got, one_shot(x, "fp32c", cuda), rtol=1e-12)
