"""Cancellation and time limits of serving requests (mb_server_cancel,
mb_server_set_timeout).

A cancelled or timed-out request ends with MB_ERR_CANCELLED, stops early,
and gives its slot back: requests queued behind it run and match the oracle
(1e-6, binary32 requests) or the one-shot sum (1e-12)."""
import time

import numpy as np
import pytest

import workloads
from oracle import direct as oracle_direct

pytestmark = pytest.mark.gpu

CANCELLED = 6


def server(**kw):
    import paper_1105_2769_amd as mb

    return mb.Server(**kw)


def one_shot(x, cuda):
    import torch

    import paper_1105_2769_amd as mb

    return mb.eval_direct(torch.from_numpy(x).to(cuda), "fp32c").cpu().numpy()


def oracle_check(x, got, tol=1e-6):
    np.testing.assert_allclose(got, oracle_direct.phi(x), rtol=tol)


def test_cancel_queued_running_and_finished(cuda):
    import paper_1105_2769_amd as mb

    big = workloads.jittered_lattice(20000, seed=61)
    small = [workloads.jittered_lattice(n, seed=62 + k) for k, n in enumerate((300, 500, 200))]
    print("serving: full run of the large request", flush=True)
    with server(max_slots=1) as srv:
        full = srv.submit(big)
        assert srv.wait(full, 120_000)
        t_full = srv.latency(full)
    print(f"serving: cancellations (full run {t_full * 1e3:.0f} ms)", flush=True)
    with server(max_slots=1) as srv:
        a = srv.submit(big)  # holds the only slot
        b = srv.submit(small[0])  # queued behind it
        c = srv.submit(small[1])  # cancelled while queued
        srv.cancel(c)
        time.sleep(0.05)  # a is staging or running
        srv.cancel(a)
        assert srv.wait(-1, 120_000)
        for rid in (a, c):
            with pytest.raises(mb.MBError) as e:
                srv.result(rid)
            assert e.value.status == CANCELLED and "cancelled" in e.value.msg
        assert srv.latency(a) < 0.5 * t_full
        oracle_check(small[0], srv.result(b))  # admitted once a gave its slot back
        d = srv.submit(small[2])
        assert srv.wait(d, 60_000)
        srv.cancel(d)  # already finished: no effect
        oracle_check(small[2], srv.result(d))
        with pytest.raises(mb.MBError) as e:
            srv.cancel(10_000)
        assert e.value.status == 1
        st = srv.stats()
    assert st["cancelled"] == 2 and st["failed"] == 2 and st["completed"] == 2


def test_timeout(cuda):
    import paper_1105_2769_amd as mb

    big = workloads.jittered_lattice(20000, seed=71)
    small = workloads.jittered_lattice(400, seed=72)
    print("serving: time limit", flush=True)
    with server() as srv:
        srv.set_timeout(20)
        a = srv.submit(big)
        assert srv.wait(a, 60_000)
        with pytest.raises(mb.MBError) as e:
            srv.result(a)
        assert e.value.status == CANCELLED and "timed out" in e.value.msg
        assert srv.latency(a) < 0.5
        srv.set_timeout(0)
        b = srv.submit(small)
        assert srv.wait(b, 60_000)
        oracle_check(small, srv.result(b))
        st = srv.stats()
    assert st["cancelled"] == 1 and st["completed"] == 1


def test_limit_is_the_one_at_submission(cuda):
    # a request keeps the limit in force when it was submitted, whatever the
    # server's limit is by the time its scheduler thread takes it in; and a
    # short limit set after a long one ends its request at its own deadline,
    # not behind the earlier request's later one
    import paper_1105_2769_amd as mb

    big = workloads.jittered_lattice(20000, seed=73)
    print("serving: limits fixed at submission", flush=True)
    with server() as srv:
        srv.set_timeout(60_000)
        a = srv.submit(big)
        srv.set_timeout(20)
        b = srv.submit(big)
        srv.set_timeout(0)
        assert srv.wait(-1, 120_000)
        np.testing.assert_allclose(srv.result(a), one_shot(big, cuda), rtol=1e-12)
        with pytest.raises(mb.MBError) as e:
            srv.result(b)
        assert e.value.status == CANCELLED and "timed out after 20 ms" in e.value.msg
        assert srv.latency(b) < srv.latency(a)
        st = srv.stats()
    assert st["cancelled"] == 1 and st["completed"] == 1


def test_random_cancels_rest_correct(cuda):
    import paper_1105_2769_amd as mb

    g = workloads.rng(5)
    sizes = g.integers(3, 2000, size=40)
    pts = [workloads.jittered_lattice(int(n), seed=800 + k) for k, n in enumerate(sizes)]
    print("serving: random cancellations", flush=True)
    with server(max_slots=4) as srv:
        srv.set_slice_units(16)
        ids = [srv.submit(x) for x in pts]
        chosen = {ids[k] for k in g.choice(len(ids), 12, replace=False)}
        for rid in ids:
            if rid in chosen:
                srv.cancel(rid)
        assert srv.wait(-1, 120_000)
        results = {}
        for rid in ids:
            try:
                results[rid] = srv.result(rid)
            except mb.MBError as e:
                # only a request that was cancelled ends this way; one whose
                # last unit had run when the cancellation landed completes
                assert rid in chosen and e.status == CANCELLED
        st = srv.stats()
    assert st["completed"] + st["failed"] == len(ids)
    assert st["failed"] == st["cancelled"] == len(ids) - len(results) >= 1
    for x, rid in zip(pts, ids):
        if rid in results:
            np.testing.assert_allclose(results[rid], one_shot(x, cuda), rtol=1e-12)
