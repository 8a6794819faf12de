"""Admission rule and worker threads of the server (host logic, CPU only)."""
import collections

import numpy as np

from paper_2408_11331_amd.serve import Entry, Pool, Request, admit, entry_from_arrays


def entry(index, n, k=4, ws=None, t_single=None, t_batch=None):
    e = Entry(index, n, k, 4 * n, 10, n, 8 * (n + 1) + 16 * n + 4 * n * k, 0)
    e.bound = ws if ws is not None else 1000 + 10 * n
    e.t_single, e.t_batch = t_single, t_batch
    return e


def q_of(entries, picks):
    q = collections.deque(Request(j) for j in picks)
    for t, r in enumerate(q):
        r.arrival = float(t)
    return q


def cost(e):
    return e.workspace() + 4 * e.n


KW = dict(large_n=50_000, want_large=False, max_batch=8)


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


def test_oldest_request_of_the_kind_alone_without_timings():
    E = [entry(0, 100_000), entry(1, 100), entry(2, 200)]
    q = q_of(E, [0, 1, 2])
    picked, g, rec, batched = admit(q, E, budget=1 << 40, in_use=0, retained=0,
                                    batch_ws=lambda r: 1, **KW)
    assert picked == [q[1]] and g == cost(E[1]) and not rec and not batched
    picked, _, _, _ = admit(q, E, budget=1 << 40, in_use=0, retained=0, large_n=50_000,
                            want_large=True, max_batch=8)
    assert picked == [q[0]]


def test_batched_calls_take_the_batch_workspace():
    E = [entry(j, 100, t_single=1.0, t_batch=1.5) for j in range(4)]
    q = q_of(E, [0, 1, 2, 3])
    seen = []

    def bws(reqs):
        seen.append(len(reqs))
        return 777
    picked, g, _, batched = admit(q, E, budget=1 << 40, in_use=0, retained=0, batch_ws=bws,
                                  **KW)
    assert sorted(r.entry for r in picked) == [0, 1, 2, 3] and batched
    assert seen == [4] and g == 777 + 4 * 400


def test_batch_joins_only_while_it_beats_solving_one_by_one():
    from paper_2408_11331_amd.serve import choose_batch
    # tiny entries batch for their time alone; the head batches slowly
    E = [entry(0, 5000, t_single=1.0, t_batch=6.0), entry(1, 1000, t_single=0.6, t_batch=0.5)]
    q = q_of(E, [0] + [1] * 5)
    assert choose_batch(list(q), E, 64) == []  # 6.0 > 1.0 + 5 * 0.6
    q = q_of(E, [0] + [1] * 9)
    got = choose_batch(list(q), E, 64)
    assert len(got) == 10 and q[0] in got      # 6.0 <= 1.0 + 9 * 0.6
    # shared by four workers, the batch must beat a quarter of the time alone
    q = q_of(E, [0] + [1] * 30)
    assert choose_batch(list(q), E, 64, workers=4) == []   # 6.0 * 4 > 1.0 + 30 * 0.6
    q = q_of(E, [0] + [1] * 40)
    assert len(choose_batch(list(q), E, 64, workers=4)) == 41
    # a head that is never batched is solved alone
    E[0].t_batch = None
    assert choose_batch(list(q), E, 64) == []
    # the head's own cheap batch: tiny ones only, head first
    q = q_of(E, [1, 1, 0, 1])
    got = choose_batch(list(q), E, 64)
    assert len(got) == 3 and q[0] in got and q[2] not in got


def test_max_batch():
    E = [entry(0, 10, t_single=1.0, t_batch=1.0)]
    q = q_of(E, [0] * 20)
    picked, _, _, batched = admit(q, E, budget=1 << 40, in_use=0, retained=0,
                                  batch_ws=lambda r: 1, large_n=50_000, want_large=False,
                                  max_batch=5)
    assert len(picked) == 5 and batched and q[0] in picked


def test_batch_that_does_not_fit_shrinks_to_the_oldest():
    E = [entry(0, 100, t_single=1.0, t_batch=1.0)]
    q = q_of(E, [0, 0, 0])
    budget = cost(E[0]) + 10
    picked, g, _, batched = admit(q, E, budget=budget, in_use=0, retained=0,
                                  batch_ws=lambda r: 10 ** 9, **KW)
    assert picked == [q[0]] and g == cost(E[0]) and not batched


def test_measured_workspace_replaces_the_bound():
    e = entry(0, 100, ws=5000)
    assert e.workspace() == 5000
    e.measured = 1200
    assert e.workspace() == 1200


def test_head_of_line_blocks_when_full():
    E = [entry(0, 5000), entry(1, 100)]
    q = q_of(E, [0, 1])
    picked, _, _, _ = admit(q, E, budget=cost(E[0]) - 1, in_use=0, retained=0, **KW)
    assert picked == []  # the oldest does not fit; the one behind it waits


def test_oversize_request_runs_alone_when_idle():
    E = [entry(0, 10_000)]
    q = q_of(E, [0])
    picked, g, rec, _ = admit(q, E, budget=1, in_use=5, retained=0, idle=True, **KW)
    assert picked == [q[0]] and g == cost(E[0]) and not rec
    picked, _, _, _ = admit(q, E, budget=1, in_use=5, retained=0, idle=False, **KW)
    assert picked == []


def test_blocked_request_reclaims_idle_workspace():
    E = [entry(0, 1000, ws=5000), entry(1, 10)]
    q = q_of(E, [0, 1])
    need = cost(E[0])
    # resident 100 + retained 9000: does not fit in 100 + need + 10 while
    # calls are in flight; with none, it is taken alone and the retained
    # workspace released
    picked, _, _, _ = admit(q, E, budget=100 + need + 10, in_use=9100, retained=9000, **KW)
    assert picked == []
    picked, g, rec, _ = admit(q, E, budget=100 + need + 10, in_use=9100, retained=9000,
                              idle=True, **KW)
    assert picked == [q[0]] and g == need and rec


def test_requests_after_a_blocked_one_wait():
    E = [entry(0, 10, t_single=1.0, t_batch=1.0)]
    q = q_of(E, [0, 0, 0])
    picked, _, _, _ = admit(q, E, budget=1 << 40, in_use=0, retained=0, batch_ws=lambda r: 1,
                            before=2.0, **KW)
    assert picked == [q[0], q[1]]
    picked, _, _, _ = admit(q, E, budget=1 << 40, in_use=0, retained=0, before=0.0, **KW)
    assert picked == []


class FakeBackend:
    """Stands in for the GPU: returns the vertex ids as the answer and keeps
    a made-up retained workspace."""

    def __init__(self, pool, delay=0.002):
        self.pool, self.delay = pool, delay
        self.calls = []
        self.kept = 0

    def make_stream(self):
        return object()

    def held(self):
        return self.kept

    def batch_ws(self, reqs):
        return 100 * len(reqs)

    def solve(self, reqs, stream, batched=False):
        import time
        self.calls.append((len(reqs), batched))
        time.sleep(self.delay * len(reqs))
        for r in reqs:
            n = self.pool.entries[r.entry].n
            r.out = np.arange(n, dtype=np.int32)
            r.stats = {"n": n}
        self.kept = max(self.kept, 150 * len(reqs))

    def release(self):
        self.kept = 0


def test_server_threads_drain_a_mixed_stream():
    from paper_2408_11331_amd.serve import run_served
    pool = Pool.of_entries([entry(0, 100, t_single=1.0, t_batch=0.5),
                            entry(1, 300, t_single=1.0, t_batch=0.8), entry(2, 60_000),
                            entry(3, 200, k=2)])
    be = FakeBackend(pool)
    reqs, summ = run_served(pool, [1, 1, 1, 1], rate=2000.0, count=200, seed=1, wait_s=30.0,
                            budget_bytes=64 << 20, large_n=50_000, max_batch=16, backend=be)
    assert summ["solves"] == 200 and all(r.out is not None and r.error is None for r in reqs)
    assert all(r.out.size == pool.entries[r.entry].n for r in reqs)
    assert any(b and c > 1 for c, b in be.calls)  # requests were batched
    assert summ["retained_bytes"] == be.kept
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


def test_large_request_under_memory_pressure_is_served():
    """A request that fits only once every other call has ended and the
    retained workspace is released is still served (requests that arrive
    after it wait meanwhile: see test_requests_after_a_blocked_one_wait)."""
    from paper_2408_11331_amd.serve import run_served
    E = [entry(j, 100, ws=100) for j in range(4)] + [entry(4, 60_000, ws=0)]
    pool = Pool.of_entries(E)
    big = 4 * 60_000
    budget = pool.resident_bytes + big + 300
    E[4].bound = big - 4 * 60_000 + 200  # with its outputs: big + 200
    be = FakeBackend(pool, delay=0.001)
    reqs, summ = run_served(pool, [1, 1, 1, 1, 1], rate=3000.0, count=120, seed=8,
                            wait_s=30.0, budget_bytes=budget, max_batch=8, backend=be)
    assert summ["solves"] == 120 and all(r.error is None for r in reqs)
    assert summ["reclaims"] >= 1 and summ["peak_accounted_bytes"] <= budget


def test_server_reports_backend_errors():
    from paper_2408_11331_amd.serve import run_served
    pool = Pool.of_entries([entry(0, 50)])

    class Broken(FakeBackend):
        def solve(self, reqs, stream, batched=False):
            raise RuntimeError("boom")

    reqs, _ = run_served(pool, [1], rate=1000.0, count=5, seed=2, wait_s=10.0,
                         backend=Broken(pool), warm=False)
    assert all(r.error and "boom" in r.error for r in reqs)


def test_failed_warm_up_raises():
    import pytest

    from paper_2408_11331_amd.serve import Server
    pool = Pool.of_entries([entry(0, 50)])

    class Broken(FakeBackend):
        def solve(self, reqs, stream, batched=False):
            raise RuntimeError("no device")

    with pytest.raises(RuntimeError, match="warm-up failed"):
        Server(pool, backend=Broken(pool))
