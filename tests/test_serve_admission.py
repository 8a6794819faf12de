"""Admission rule of the server (host logic, CPU only)."""
import collections

import numpy as np

from paper_2408_11331_amd.serve import Request, admit


def req(n, k=4, deg=4):
    rp = np.arange(0, deg * (n + 1), deg, dtype=np.int64)[: n + 1]
    return Request(rp, np.zeros(int(rp[-1]), np.int32), np.zeros((k, n), np.int32), None)


def test_fifo_within_budget_and_kind():
    q = collections.deque([req(100), req(100_000), req(200), req(300)])
    fp = [r.footprint() for r in q]
    picked, held = admit(q, budget=fp[0] + fp[2] + 10, in_use=0, large_n=50_000,
                         want_large=False, max_batch=8)
    assert picked == [q[0], q[2]] and held == fp[0] + fp[2]


def test_large_requests_go_one_at_a_time():
    q = collections.deque([req(60_000), req(70_000)])
    picked, _ = admit(q, budget=1 << 40, in_use=0, large_n=50_000, want_large=True, max_batch=8)
    assert picked == [q[0]]


def test_head_of_line_blocks_when_full():
    q = collections.deque([req(100), req(5000), req(100)])
    fp0 = q[0].footprint()
    picked, _ = admit(q, budget=fp0 + q[1].footprint() - 1, in_use=0, large_n=50_000,
                      want_large=False, max_batch=8)
    assert picked == [q[0]]  # the second does not fit; the third waits behind it
    picked, _ = admit(q, budget=fp0, in_use=fp0, large_n=50_000, want_large=False, max_batch=8)
    assert picked == []


def test_oversize_request_runs_alone_when_idle():
    q = collections.deque([req(10_000)])
    picked, held = admit(q, budget=1, in_use=0, large_n=50_000, want_large=False, max_batch=8)
    assert picked == [q[0]] and held == q[0].footprint()
    picked, _ = admit(q, budget=1, in_use=5, large_n=50_000, want_large=False, max_batch=8)
    assert picked == []


def test_max_batch():
    q = collections.deque([req(10) for _ in range(20)])
    picked, _ = admit(q, budget=1 << 40, in_use=0, large_n=50_000, want_large=False, max_batch=5)
    assert len(picked) == 5


class FakeBackend:
    """Stands in for the GPU: copies the initial consensus as the answer."""

    def __init__(self, delay=0.002):
        self.delay = delay
        self.calls = []

    def make_stream(self):
        return None

    def solve(self, reqs, large, stream):
        import time
        self.calls.append((large, len(reqs)))
        time.sleep(self.delay * len(reqs))
        for r in reqs:
            r.out = np.arange(r.n, dtype=np.int32) if r.init is None else r.init.copy()
            r.stats = {"n": r.n}


def test_server_threads_drain_a_mixed_stream():
    from paper_2408_11331_amd.serve import run_served
    pool = [req(100), req(300), req(60_000), req(200, k=2)]
    be = FakeBackend()
    reqs, summ = run_served(pool, rate=2000.0, count=200, seed=1, wait_s=30.0,
                            budget_bytes=8 << 20, large_n=50_000, max_batch=16, backend=be)
    assert summ["solves"] == 200 and all(r.out is not None and r.error is None for r in reqs)
    assert any(large for large, _ in be.calls) and any(not large for large, _ in be.calls)
    assert max(c for large, c in be.calls if not large) > 1  # requests were batched


def test_server_reports_backend_errors():
    from paper_2408_11331_amd.serve import run_served

    class Broken(FakeBackend):
        def solve(self, reqs, large, stream):
            raise RuntimeError("boom")

    reqs, _ = run_served([req(50)], rate=1000.0, count=5, seed=2, wait_s=10.0, backend=Broken())
    assert all(r.error and "boom" in r.error for r in reqs)
