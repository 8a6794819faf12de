"""Admission rule and worker threads of the server (host logic, CPU only)."""
import collections

import numpy as np

from paper_2408_11331_amd.serve import Entry, Pool, Request, admit, entry_from_arrays


def entry(index, n, k=4, ws=None):
    e = Entry(index, n, k, 4 * n, 10, n, 8 * (n + 1) + 16 * n + 4 * n * k, 0)
    e.bound = ws if ws is not None else 1000 + 10 * n
    return e


def q_of(entries, picks):
    return collections.deque(Request(j) for j in picks)


def cost(e):
    return e.workspace() + 4 * e.n


def test_entry_figures_from_arrays():
    n, k = 50, 3
    rp = np.arange(0, 2 * (n + 1), 2, dtype=np.int64)
    col = np.zeros(int(rp[-1]), np.int32)
    lab = np.zeros((k, n), np.int32)
    lab[1, 7] = 9
    init = np.arange(n, dtype=np.int32) % 5
    e = entry_from_arrays(2, rp, col, lab, init)
    assert (e.n, e.k, e.nnz, e.max_label, e.clusters) == (n, k, 100, 9, 5)
    assert e.input_bytes == 8 * 51 + 4 * 100 + 4 * n * k + 4 * n
    assert entry_from_arrays(0, rp, col, lab, None).clusters == n


def test_fifo_within_budget_and_kind():
    E = [entry(0, 100), entry(1, 100_000), entry(2, 200), entry(3, 300)]
    q = q_of(E, [0, 1, 2, 3])
    # one or two requests: the workspace of the largest, the outputs of all
    g02 = max(E[0].workspace(), E[2].workspace()) + 4 * (E[0].n + E[2].n)
    picked, g = admit(q, E, budget=g02 + 10, in_use=0, large_n=50_000, want_large=False,
                      max_batch=8)
    assert picked == [q[0], q[2]] and g == g02  # the fourth would not fit


def test_batched_calls_take_the_batch_workspace():
    E = [entry(j, 100) for j in range(4)]
    q = q_of(E, [0, 1, 2, 3])
    seen = []

    def bws(reqs):
        seen.append(len(reqs))
        return 777
    picked, g = admit(q, E, budget=1 << 40, in_use=0, large_n=50_000, want_large=False,
                      max_batch=8, batch_ws=bws)
    assert len(picked) == 4 and seen == [3, 4] and g == 777 + 4 * 400


def test_measured_workspace_replaces_the_bound():
    e = entry(0, 100, ws=5000)
    assert e.workspace() == 5000
    e.measured = 1200
    assert e.workspace() == 1200


def test_large_requests_go_one_at_a_time():
    E = [entry(0, 60_000), entry(1, 70_000)]
    q = q_of(E, [0, 1])
    picked, _ = admit(q, E, budget=1 << 40, in_use=0, large_n=50_000, want_large=True,
                      max_batch=8)
    assert picked == [q[0]]


def test_head_of_line_blocks_when_full():
    E = [entry(0, 100), entry(1, 5000), entry(2, 100)]
    q = q_of(E, [0, 1, 2])
    c0 = cost(E[0])
    picked, _ = admit(q, E, budget=c0 + 10, in_use=0, large_n=50_000, want_large=False,
                      max_batch=8)
    assert picked == [q[0]]  # the second does not fit; the third waits behind it
    picked, _ = admit(q, E, budget=c0, in_use=1, large_n=50_000, want_large=False,
                      max_batch=8)
    assert picked == []


def test_oversize_request_runs_alone_when_idle():
    E = [entry(0, 10_000)]
    q = q_of(E, [0])
    picked, g = admit(q, E, budget=1, in_use=0, large_n=50_000, want_large=False, max_batch=8)
    assert picked == [q[0]] and g == cost(E[0])
    picked, _ = admit(q, E, budget=1, in_use=5, large_n=50_000, want_large=False, max_batch=8)
    assert picked == []


def test_max_batch():
    E = [entry(0, 10)]
    q = q_of(E, [0] * 20)
    picked, _ = admit(q, E, budget=1 << 40, in_use=0, large_n=50_000, want_large=False,
                      max_batch=5)
    assert len(picked) == 5


class FakeBackend:
    """Stands in for the GPU: returns the vertex ids as the answer and keeps
    a made-up retained workspace per stream."""

    def __init__(self, pool, delay=0.002):
        self.pool, self.delay = pool, delay
        self.calls = []
        self.keep = {}

    def make_stream(self):
        return object()

    def held(self, stream):
        return self.keep.get(id(stream), 0)

    def batch_ws(self, reqs):
        return 100 * len(reqs)

    def solve(self, reqs, stream):
        import time
        self.calls.append(len(reqs))
        time.sleep(self.delay * len(reqs))
        for r in reqs:
            n = self.pool.entries[r.entry].n
            r.out = np.arange(n, dtype=np.int32)
            r.stats = {"n": n}
        self.keep[id(stream)] = max(self.held(stream), 50 * len(reqs))


def test_server_threads_drain_a_mixed_stream():
    from paper_2408_11331_amd.serve import run_served
    pool = Pool.of_entries([entry(0, 100), entry(1, 300), entry(2, 60_000), entry(3, 200, k=2)])
    be = FakeBackend(pool)
    reqs, summ = run_served(pool, [1, 1, 1, 1], rate=2000.0, count=200, seed=1, wait_s=30.0,
                            budget_bytes=64 << 20, large_n=50_000, max_batch=16, backend=be)
    assert summ["solves"] == 200 and all(r.out is not None and r.error is None for r in reqs)
    assert all(r.out.size == pool.entries[r.entry].n for r in reqs)
    assert max(be.calls) > 2  # requests were batched
    assert summ["retained_bytes"] == sum(be.keep.values())
    assert summ["peak_accounted_bytes"] <= summ["budget_bytes"]


def test_budget_is_never_exceeded_by_the_accounting():
    from paper_2408_11331_amd.serve import run_served
    E = [entry(j, 100 + 50 * j, ws=4000) for j in range(6)]
    pool = Pool.of_entries(E)
    be = FakeBackend(pool, delay=0.001)
    budget = pool.resident_bytes + 3 * 4000 + 50_000
    reqs, summ = run_served(pool, [1] * 6, rate=5000.0, count=150, seed=4, wait_s=30.0,
                            budget_bytes=budget, max_batch=64, small_workers=3,
                            large_workers=1, backend=be)
    assert summ["solves"] == 150 and summ["peak_accounted_bytes"] <= budget


def test_server_reports_backend_errors():
    from paper_2408_11331_amd.serve import run_served
    pool = Pool.of_entries([entry(0, 50)])

    class Broken(FakeBackend):
        def solve(self, reqs, stream):
            raise RuntimeError("boom")

    reqs, _ = run_served(pool, [1], rate=1000.0, count=5, seed=2, wait_s=10.0,
                         backend=Broken(pool), warm=False)
    assert all(r.error and "boom" in r.error for r in reqs)


def test_failed_warm_up_raises():
    import pytest

    from paper_2408_11331_amd.serve import Server
    pool = Pool.of_entries([entry(0, 50)])

    class Broken(FakeBackend):
        def solve(self, reqs, stream):
            raise RuntimeError("no device")

    with pytest.raises(RuntimeError, match="warm-up failed"):
        Server(pool, backend=Broken(pool))
