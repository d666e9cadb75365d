"""The server driven from several threads at once.

The binding's ctypes calls release the interpreter lock, so the calls of the
client threads overlap inside the library while its scheduler thread runs
the requests: four clients submit, poll, wait, cancel, fetch and change the
slice size; a monitor reads the counters throughout; one thread sets a 5 ms
time limit around a large request while the others submit (so any request
submitted in that window may end timed out).  Checks: every request ends
with its result or MB_ERR_CANCELLED, the same points submitted twice give
the same Phi to 1e-12 of the largest |Phi| (only the order of binary64
additions differs), and the counters add up.  This is the dynamic check of
the lock discipline that the compile-time analysis (test_serve_locks.py)
checks statically.
"""
import threading
import time

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

CANCELLED = 6


def test_concurrent_clients(cuda):
    import paper_1105_2769_amd as mb

    errors = []
    counts = {"submitted": 0, "cancelled": 0}
    lock = threading.Lock()
    stop = threading.Event()

    def guarded(fn):
        def run(*args):
            try:
                fn(*args)
            except BaseException as e:  # reported by the main thread
                errors.append(e)
        return run

    def ended(srv, rid):
        """Phi of a finished request, or None if it was cancelled."""
        try:
            return srv.result(rid)
        except mb.MBError as e:
            assert e.status == CANCELLED, (rid, e.status, e.msg)
            return None

    def client(srv, cid):
        g = workloads.rng(900 + cid)
        for r in range(10):
            n, m = (int(v) for v in g.integers(3, 1200, size=2))
            x = workloads.jittered_lattice(n, seed=2000 + 50 * cid + r)
            y = workloads.jittered_lattice(m, seed=3000 + 50 * cid + r)
            a, b, c = srv.submit(x, "fp64"), srv.submit(x, "fp64"), srv.submit(y, "fp32c")
            srv.cancel(c)
            if r % 3 == 1:
                srv.set_slice_units(8 + 8 * (r % 5))
            while not srv.poll(a):
                time.sleep(2e-4)
            assert srv.wait(b, 60_000) and srv.wait(c, 60_000)
            pa, pb, pc = ended(srv, a), ended(srv, b), ended(srv, c)
            if pa is not None and pb is not None:
                np.testing.assert_allclose(pa, pb, rtol=0, atol=1e-12 * np.abs(pa).max())
                assert srv.latency(a) >= 0.0
            with lock:
                counts["submitted"] += 3
                counts["cancelled"] += sum(p is None for p in (pa, pb, pc))

    def limiter(srv):
        x = workloads.jittered_lattice(8000, seed=7)  # about 35 ms of binary64 work
        srv.set_timeout(5)
        rid = srv.submit(x, "fp64")
        srv.set_timeout(0)
        assert srv.wait(rid, 60_000)
        with lock:
            counts["submitted"] += 1
            counts["cancelled"] += ended(srv, rid) is None

    def monitor(srv):
        while not stop.is_set():
            st = srv.stats()
            assert st["completed"] + st["failed"] <= st["submitted"]
            time.sleep(1e-3)

    print("serving: concurrent clients", flush=True)
    with mb.Server(hbm_budget_bytes=4 << 30, max_slots=8) as srv:
        mon = threading.Thread(target=guarded(monitor), args=(srv,))
        workers = [threading.Thread(target=guarded(client), args=(srv, c)) for c in range(4)]
        workers.append(threading.Thread(target=guarded(limiter), args=(srv,)))
        mon.start()
        for t in workers:
            t.start()
        for t in workers:
            t.join(120)
        stop.set()
        mon.join(10)
        assert not any(t.is_alive() for t in workers + [mon]), "a client thread did not end"
        if errors:
            raise errors[0]
        assert srv.wait(-1, 60_000)
        st = srv.stats()
    print(f"serving: {st['submitted']} requests, {st['cancelled']} cancelled, "
          f"{st['drain_launches']} drain launches", flush=True)
    assert st["submitted"] == counts["submitted"] == 4 * 10 * 3 + 1
    assert st["completed"] + st["failed"] == st["submitted"]
    assert st["failed"] == st["cancelled"] == counts["cancelled"]
