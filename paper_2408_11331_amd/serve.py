"""Consensus-solve serving with continuous batching on one GPU.

A pool of problems (a graph, k partitions, an initial consensus) is
registered once: its arrays are uploaded and stay resident in device
memory, and each entry is timed once on the multi-workgroup path
(``mcc_consensus``) and, if it is small enough, alone in the persistent
batched launch (``mcc_consensus_batch``, one workgroup per instance).
Requests name a pool entry and arrive at any time.  Worker threads, each
with its own HIP stream, take requests from one admission queue in arrival
order: "small" workers take the oldest small request and, when it pays,
the other waiting small requests with it in one batched launch — a batched
call lasts about as long as its slowest instance, so requests join the
call while that stays below the time solving them one by one would take;
otherwise the request is solved alone.  "Large" workers solve large
requests one at a time.  Calls on different workers' streams overlap on the
GPU, so requests that arrive while others are being solved start at once.

Admission keeps device memory within a budget: the resident pool, the
workspace the library keeps between calls (shared by the workers' streams;
the library reports it, ``mcc_workspace_held``), and for each call in
flight its whole workspace and outputs, counted as if none of the retained
workspace could be reused.  A call's workspace is taken from the library's own sizing
(``mcc_workspace_bound``, ``mcc_batch_workspace_bytes``) until a solve of
the same entry has reported its exact figure (``workspace_bytes``).

Every result is exactly the result ``mcc_consensus`` gives for the request
alone: batching changes where a solve runs, not what it computes.  This
module only schedules: all computation happens in libmcc.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import List, Optional

import numpy as np


@dataclasses.dataclass(eq=False)
class Entry:
    """One registered problem: host arrays, their resident device copies and
    what the admission needs to know about them."""
    index: int
    n: int
    k: int
    nnz: int
    max_label: int
    clusters: int          # distinct initial cluster ids (n for singletons)
    input_bytes: int       # resident device bytes
    bound: int             # workspace bound of one solve (library sizing)
    measured: int = 0      # exact workspace of a finished solve, once known
    dev: Optional[dict] = None
    t_single: Optional[float] = None  # seconds, alone on the multi-workgroup path
    t_batch: Optional[float] = None   # seconds, alone in a batched launch (None: never batched)

    def workspace(self) -> int:
        return self.measured or self.bound


@dataclasses.dataclass(eq=False)  # requests compare by identity (queue removal)
class Request:
    entry: int
    rid: int = 0
    arrival: float = 0.0         # perf_counter at submission
    started: float = 0.0
    done_at: float = 0.0
    out: Optional[np.ndarray] = None
    stats: Optional[dict] = None
    error: Optional[str] = None
    event: threading.Event = dataclasses.field(default_factory=threading.Event)


def entry_from_arrays(index, row_ptr, col, labels, init):
    """Admission figures of a problem given as host arrays (no upload)."""
    n = int(row_ptr.size - 1)
    k = int(labels.shape[0])
    nnz = int(col.size)
    max_label = int(labels.max()) if labels.size else 0
    clusters = int(np.unique(init).size) if init is not None else n
    input_bytes = 8 * (n + 1) + 4 * nnz + 4 * n * k + (4 * n if init is not None else 0)
    return Entry(index, n, k, nnz, max_label, clusters, input_bytes, 0)


class Pool:
    """Problems uploaded once and kept resident on the device."""

    def __init__(self, instances, flags: int = 0, device: str = "cuda", calibrate: bool = True,
                 batch_n_max: int = 16384, batch_ratio_max: float = 4.0):
        import torch

        import paper_2408_11331_amd as mcc
        self.flags = flags
        self.entries: List[Entry] = []
        T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        for j, inst in enumerate(instances):
            e = entry_from_arrays(j, inst.row_ptr, inst.col, inst.labels, inst.init)
            e.bound = mcc.workspace_bound(e.n, e.nnz, e.k, e.max_label, e.clusters, flags)
            e.dev = {"row_ptr": T(inst.row_ptr), "col": T(inst.col), "labels": T(inst.labels),
                     "init": None if inst.init is None else T(inst.init)}
            self.entries.append(e)
        torch.cuda.synchronize()
        self.resident_bytes = sum(e.input_bytes for e in self.entries)
        if calibrate:
            self.calibrate(batch_n_max, batch_ratio_max)

    def calibrate(self, batch_n_max: int = 16384, batch_ratio_max: float = 4.0,
                  max_rounds: int = 0):
        """Time every entry alone on the multi-workgroup path and, if it has
        at most batch_n_max vertices and 256 partitions, two copies of it in
        one batched launch (after one untimed call of each that sets the
        path up).  An entry is batched only if two copies take no longer
        than 1.5 times one copy (else the launch hands it back to the
        multi-workgroup path one copy after the other) and at most
        batch_ratio_max times its time alone."""
        import torch

        import paper_2408_11331_amd as mcc

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            return time.perf_counter() - t

        for e in self.entries:
            d = e.dev
            e.t_single = timed(lambda: mcc.consensus(d["row_ptr"], d["col"], d["labels"],
                                                     d["init"], max_rounds=max_rounds,
                                                     flags=self.flags))
            e.t_batch = None
            if e.n <= batch_n_max and e.k <= 256:
                t1 = timed(lambda: mcc.consensus_batch([d], max_rounds=max_rounds,
                                                       flags=self.flags))
                t2 = timed(lambda: mcc.consensus_batch([d, d], max_rounds=max_rounds,
                                                       flags=self.flags))
                if t2 <= 1.5 * t1 and t2 <= batch_ratio_max * e.t_single:
                    e.t_batch = t2

    @classmethod
    def of_entries(cls, entries: List[Entry], flags: int = 0) -> "Pool":
        """A pool of admission figures only (nothing uploaded), for a
        backend that does not read device arrays."""
        p = cls.__new__(cls)
        p.flags, p.entries = flags, list(entries)
        p.resident_bytes = sum(e.input_bytes for e in p.entries)
        return p

    def __len__(self):
        return len(self.entries)


def choose_batch(mine, entries, max_batch: int, workers: int = 1):
    """The requests to solve with the oldest one, mine[0], in one batched
    call, or [] if it should be solved alone.  A batched call lasts about as
    long as its slowest instance and holds one of `workers` workers that
    would otherwise share the requests: among the waiting requests that may
    be batched, taken in increasing batched time, the longest run that
    includes mine[0] and whose slowest batched time stays within the sum of
    their times alone divided by `workers`."""
    head = mine[0]
    if entries[head.entry].t_batch is None:
        return []
    cand = sorted((r for r in mine if entries[r.entry].t_batch is not None),
                  key=lambda r: entries[r.entry].t_batch)[:max_batch]
    if head not in cand:  # more than max_batch requests are cheaper than the head
        cand = cand[:max_batch - 1] + [head]
        cand.sort(key=lambda r: entries[r.entry].t_batch)
    best, alone, has_head = [], 0.0, False
    for m, r in enumerate(cand, 1):
        e = entries[r.entry]
        alone += e.t_single
        has_head = has_head or r is head
        if has_head and m >= 2 and e.t_batch * workers <= alone:
            best = cand[:m]
    return best


def admit(queue, entries, budget: int, in_use: int, retained: int, large_n: int,
          want_large: bool, max_batch: int, batch_ws=None, idle: bool = False,
          before: float = float("inf"), workers: int = 1):
    """Pick the call one worker (of `workers` of its kind) makes now: the
    oldest request of its kind that arrived before `before`, with the
    requests ``choose_batch`` joins to it when the worker batches (``batch_ws(reqs)`` gives the workspace
    of a batched call; None: never batch).  The call's workspace and outputs
    must fit next to `in_use` (of which `retained` is idle workspace the
    library keeps): a batch that does not fit shrinks to the oldest request
    alone, and a request that does not fit alone waits (requests behind it
    wait too), unless no call is in flight (`idle`): then it is taken alone,
    after the retained workspace is released if there is any (`reclaim`) —
    also when it needs more than the whole budget.  Pure function of its
    arguments.  Returns (requests, bytes the call may add, reclaim,
    batched)."""
    mine = []
    for r in queue:
        if r.arrival >= before:
            break  # the queue is in arrival order
        if (entries[r.entry].n > large_n) == want_large:
            mine.append(r)
    if not mine:
        return [], 0, False, False
    head = mine[0]
    g1 = entries[head.entry].workspace() + 4 * entries[head.entry].n
    if in_use + g1 > budget:
        if idle:
            return [head], g1, retained > 0, False
        return [], 0, False, False
    if not want_large and batch_ws is not None and max_batch > 1:
        group = choose_batch(mine, entries, max_batch, workers)
        if group:
            g = batch_ws(group) + sum(4 * entries[r.entry].n for r in group)
            if in_use + g <= budget:
                return group, g, False, True
    return [head], g1, False, False


class GpuBackend:
    """Solves admitted requests with libmcc on the worker's own HIP stream,
    from the pool's resident arrays."""

    def __init__(self, pool: Pool, max_rounds: int = 0):
        import torch

        import paper_2408_11331_amd as mcc
        mcc.lib()
        self.torch, self.mcc, self.pool, self.max_rounds = torch, mcc, pool, max_rounds

    def make_stream(self):
        return self.torch.cuda.Stream()  # default priority

    def held(self) -> int:
        return self.mcc.workspace_held()

    def release(self) -> None:
        """Free the library's idle workspace (no call may be in flight)."""
        self.mcc.release_workspace()

    def batch_ws(self, reqs: List[Request]) -> int:
        return self.mcc.batch_workspace_bytes([self.pool.entries[r.entry].dev for r in reqs])

    def solve(self, reqs: List[Request], stream, batched: bool = False) -> None:
        """Solve (in one batched call, or one by one), fill each request's
        out and stats."""
        torch, mcc = self.torch, self.mcc
        entries = self.pool.entries
        with torch.cuda.stream(stream):
            outs = [torch.empty(entries[r.entry].n, dtype=torch.int32, device="cuda")
                    for r in reqs]
        if batched:
            probs = [entries[r.entry].dev for r in reqs]
            _, stats, codes, info = mcc.consensus_batch(probs, max_rounds=self.max_rounds,
                                                        flags=self.pool.flags, stream=stream,
                                                        outs=outs)
            for r, c, st in zip(reqs, codes, stats):
                if c != 0:
                    r.error = mcc.lib().mcc_strerror(c).decode()
                r.stats = st
        else:
            for r, o in zip(reqs, outs):
                d = entries[r.entry].dev
                _, st = mcc.consensus(d["row_ptr"], d["col"], d["labels"], d["init"],
                                      max_rounds=self.max_rounds, flags=self.pool.flags,
                                      stream=stream, out=o)
                r.stats = st
                e = entries[r.entry]
                e.measured = max(e.measured, st["workspace_bytes"])
        with torch.cuda.stream(stream):
            host = [o.cpu() for o in outs]  # synchronous copies on the worker's stream
        for r, h in zip(reqs, host):
            r.out = h.numpy()


class Server:
    """Admission queue plus worker threads that own one stream each.

    Each worker first warms up (``_warm``), so that the first requests pay
    no set-up; the constructor returns once every worker is ready."""

    def __init__(self, pool: Pool, budget_bytes: int = 64 << 30, large_n: int = 50_000,
                 max_batch: int = 512, small_workers: int = 4, large_workers: int = 2,
                 max_rounds: int = 0, backend=None, warm: bool = True):
        self.pool = pool
        self.backend = backend if backend is not None else GpuBackend(pool, max_rounds)
        self.budget = int(budget_bytes)
        if pool.resident_bytes > self.budget:
            raise ValueError("the resident pool alone exceeds the budget")
        self.large_n = int(large_n)
        self.max_batch = int(max_batch)
        self.queue = collections.deque()
        self.lock = threading.Lock()
        # workers wait on their kind's condition: an arrival wakes one worker
        # of its kind; a finished call (memory, idle state) wakes them all
        self.kind_cv = {False: threading.Condition(self.lock), True: threading.Condition(self.lock)}
        self.running = True
        self.completed: List[Request] = []
        self.retained = 0       # workspace the library keeps on the device (its figure)
        self.growth = {}        # worker -> bytes its call in flight may add
        self.blocked = {}       # worker -> arrival of its request waiting for memory
        self.peak_in_use = 0
        self.batches = 0        # calls made
        self.batched_calls = 0  # of which batched launches
        self.reclaims = 0
        self.threads = []
        kinds = [False] * small_workers + [True] * large_workers
        self.kinds = kinds
        ready = threading.Barrier(len(kinds) + 1)
        for w, large in enumerate(kinds):
            self.growth[w] = 0
            self.blocked[w] = None
            self.threads.append(threading.Thread(target=self._worker, args=(w, large, warm, ready),
                                                 daemon=True))
        self.warm_errors: List[str] = []
        self.warm_lock = threading.Lock()
        for t in self.threads:
            t.start()
        ready.wait()
        if self.warm_errors:
            self.close()
            raise RuntimeError("worker warm-up failed: " + "; ".join(self.warm_errors))

    def in_use(self) -> int:
        """Bytes accounted for: resident pool, retained workspaces, calls in
        flight (caller holds the lock)."""
        return self.pool.resident_bytes + self.retained + sum(self.growth.values())

    # -- client side ----------------------------------------------------------
    def submit(self, entry: int, rid: int = 0) -> Request:
        req = Request(entry, rid=rid)
        req.arrival = time.perf_counter()
        with self.lock:
            self.queue.append(req)
            self.kind_cv[self.pool.entries[entry].n > self.large_n].notify()
        return req

    def _wake_all(self):  # caller holds the lock
        for c in self.kind_cv.values():
            c.notify_all()

    def close(self):
        with self.lock:
            self.running = False
            self._wake_all()
        for t in self.threads:
            t.join()

    # -- workers ----------------------------------------------------------------
    def _warm(self, w: int, large: bool, stream):
        """One solve of an entry of the worker's kind (the largest for large
        workers, so that the workspace kept between calls is sized for any
        request; the smallest for small ones) and, for small workers, one
        batched call (it sets up the batched launch's graph)."""
        entries = self.pool.entries
        mine = [e for e in entries if (e.n > self.large_n) == large]
        if not mine:
            return
        e = max(mine, key=lambda x: x.n) if large else min(mine, key=lambda x: x.n)
        # one warm-up at a time: the later ones reuse the workspace the first
        # left, so warming up takes no more memory than one request does
        with self.warm_lock:
            self.backend.solve([Request(e.index)], stream)
            if not large and e.t_batch is not None:
                self.backend.solve([Request(e.index) for _ in range(3)], stream, batched=True)
            with self.lock:
                self.retained = self.backend.held()

    def _worker(self, w: int, large: bool, warm: bool, ready):
        stream = self.backend.make_stream()
        entries = self.pool.entries
        bws = None if large else self.backend.batch_ws
        try:
            if warm:
                self._warm(w, large, stream)
        except Exception as e:
            with self.lock:
                self.warm_errors.append(f"worker {w}: {type(e).__name__}: {e}")
            ready.wait()
            return
        ready.wait()
        inf = float("inf")
        cv = self.kind_cv[large]
        while True:
            with self.lock:
                while True:
                    # a request another worker holds back for memory goes first:
                    # take nothing that arrived after it
                    before = min((t for v, t in self.blocked.items()
                                  if v != w and t is not None), default=inf)
                    idle = not any(self.growth.values())
                    picked, growth, reclaim, batched = admit(
                        self.queue, entries, self.budget, self.in_use(),
                        self.retained, self.large_n, large, self.max_batch, bws,
                        idle=idle, before=before,
                        workers=self.kinds.count(large))
                    if picked:
                        if self.blocked[w] is not None:  # others may take later requests now
                            self.blocked[w] = None
                            self._wake_all()
                        if reclaim:
                            self.backend.release()
                            self.retained = 0
                            self.reclaims += 1
                        break
                    head = next((r for r in self.queue
                                 if (entries[r.entry].n > self.large_n) == large), None)
                    if not self.running and head is None:
                        return
                    self.blocked[w] = head.arrival if head is not None and \
                        head.arrival < before else None
                    cv.wait()
                for r in picked:
                    self.queue.remove(r)
                self.growth[w] = growth
                self.peak_in_use = max(self.peak_in_use, self.in_use())
                self.batches += 1
                self.batched_calls += 1 if batched else 0
            t0 = time.perf_counter()
            for r in picked:
                r.started = t0
            held = None
            try:
                self.backend.solve(picked, stream, batched)
                held = self.backend.held()
            except Exception as e:  # reported per request, the server keeps going
                for r in picked:
                    r.error = f"{type(e).__name__}: {e}"
            t1 = time.perf_counter()
            with self.lock:
                self.growth[w] = 0
                if held is not None:
                    self.retained = held
                for r in picked:
                    r.done_at = t1
                    self.completed.append(r)
                    r.event.set()
                self._wake_all()


def latency_summary(reqs: List[Request]) -> dict:
    lat = np.array([r.done_at - r.arrival for r in reqs])
    span = max(r.done_at for r in reqs) - min(r.arrival for r in reqs)
    return {"solves": len(reqs), "solves_per_s": len(reqs) / span if span > 0 else float("inf"),
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}


def poisson_arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def request_stream(weights, rate: float, count: int, seed: int):
    """Entries (drawn with the given weights) and arrival offsets (s)."""
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    p = np.asarray(weights, np.float64)
    picks = rng.choice(len(p), size=count, p=p / p.sum())
    return picks, poisson_arrivals(rate, count, seed)


def run_served(pool: Pool, weights, rate: float, count: int, seed: int = 0,
               wait_s: float = 600.0, **server_kw):
    """Replay `count` requests with Poisson arrivals at `rate` per second
    through a Server; returns (requests, summary)."""
    picks, times = request_stream(weights, rate, count, seed)
    srv = Server(pool, **server_kw)
    reqs = []
    t0 = time.perf_counter()
    for p, at in zip(picks, times):
        delay = t0 + at - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        reqs.append(srv.submit(int(p), rid=int(p)))
    deadline = time.perf_counter() + wait_s
    for r in reqs:
        if not r.event.wait(max(0.0, deadline - time.perf_counter())):
            raise TimeoutError(f"request for entry {r.entry} not served within {wait_s} s")
    srv.close()
    summ = latency_summary(reqs)
    summ.update(batches=srv.batches, batched_calls=srv.batched_calls, reclaims=srv.reclaims, peak_accounted_bytes=srv.peak_in_use,
                retained_bytes=srv.retained, budget_bytes=srv.budget,
                resident_bytes=pool.resident_bytes)
    return reqs, summ


def run_one_at_a_time(pool: Pool, weights, rate: float, count: int, seed: int = 0,
                      max_rounds: int = 0):
    """The plain path on the same arrivals: one mcc_consensus at a time, in
    arrival order, on one stream, from the same resident arrays."""
    import torch

    import paper_2408_11331_amd as mcc
    picks, times = request_stream(weights, rate, count, seed)
    small = min(pool.entries, key=lambda x: x.n).dev
    mcc.consensus(small["row_ptr"], small["col"], small["labels"], small["init"],
                  max_rounds=max_rounds, flags=pool.flags)  # warm-up, as the server's workers
    reqs = []
    t0 = time.perf_counter()
    for p, at in zip(picks, times):
        now = time.perf_counter()
        if now < t0 + at:
            time.sleep(t0 + at - now)
        e = pool.entries[int(p)]
        r = Request(int(p), rid=int(p))
        r.arrival = t0 + at
        d = e.dev
        out, st = mcc.consensus(d["row_ptr"], d["col"], d["labels"], d["init"],
                                max_rounds=max_rounds, flags=pool.flags)
        r.out, r.stats = out.cpu().numpy(), st
        r.done_at = time.perf_counter()
        reqs.append(r)
    torch.cuda.synchronize()
    return reqs, latency_summary(reqs)
