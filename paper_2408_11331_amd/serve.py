"""Consensus-solve serving with continuous batching on one GPU.

Requests (a graph, k partitions, an optional initial consensus) arrive at
any time.  Small requests (a few thousand vertices, where one workgroup per
instance is the right size) are solved in batches by the persistent
batched kernel (``mcc_consensus_batch``); larger ones by the multi-workgroup
single-instance path (``mcc_consensus``).  Several workers, each with its
own HIP stream, pull from one admission queue: while one batch or solve is
on the device the next one is admitted and launched on another stream, so
work from requests that arrived at different times overlaps on the GPU.
Admission is bounded by an HBM budget: a request is taken only when its
device footprint fits next to everything in flight.

Every result is exactly the result ``mcc_consensus`` gives for the request
alone: batching changes where a solve runs, not what it computes.

This module only schedules: all computation happens in libmcc.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import List, Optional

import numpy as np


@dataclasses.dataclass(eq=False)  # requests compare by identity (queue removal)
class Request:
    row_ptr: np.ndarray          # int64 [n + 1]
    col: np.ndarray              # int32 [nnz]
    labels: np.ndarray           # int32 [k, n]
    init: Optional[np.ndarray]   # int32 [n] or None (singletons)
    rid: int = 0
    arrival: float = 0.0         # perf_counter at submission
    started: float = 0.0
    done_at: float = 0.0
    out: Optional[np.ndarray] = None
    stats: Optional[dict] = None
    error: Optional[str] = None
    event: threading.Event = dataclasses.field(default_factory=threading.Event)

    @property
    def n(self) -> int:
        return int(self.row_ptr.size - 1)

    @property
    def k(self) -> int:
        return int(self.labels.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.col.size)

    def footprint(self) -> int:
        """Device bytes held while the request is in flight: its inputs and
        output, the vertex-major label rows, per-vertex state and a table
        allowance."""
        n, k, nnz = self.n, self.k, self.nnz
        return 8 * (n + 1) + 4 * nnz + 8 * n * k + 48 * n + 16 * n * k // 4 + (1 << 16)


def admit(queue, budget: int, in_use: int, large_n: int, want_large: bool, max_batch: int):
    """Pick the requests one worker takes now (FIFO among the requests of
    its kind whose footprint still fits the budget).  Pure function of its
    arguments: returns (picked requests, bytes they hold)."""
    picked, held = [], 0
    for r in queue:
        if (r.n > large_n) != want_large:
            continue
        fp = r.footprint()
        if in_use + held + fp > budget:
            if not picked and in_use == 0 and held == 0:
                # a request larger than the whole budget runs alone
                picked.append(r)
                held += fp
            break
        picked.append(r)
        held += fp
        if want_large or len(picked) >= max_batch:
            break
    return picked, held


class GpuBackend:
    """Solves admitted requests with libmcc on the worker's own HIP stream."""

    def __init__(self, max_rounds: int = 0):
        import torch
        import paper_2408_11331_amd as mcc
        mcc.lib()
        self.torch, self.mcc, self.max_rounds = torch, mcc, max_rounds

    def make_stream(self):
        return self.torch.cuda.Stream()  # default priority

    def _upload(self, r: Request):
        T = lambda a: self.torch.from_numpy(np.ascontiguousarray(a)).cuda()
        return {"row_ptr": T(r.row_ptr), "col": T(r.col), "labels": T(r.labels),
                "init": None if r.init is None else T(r.init)}

    def solve(self, reqs: List[Request], large: bool, stream) -> None:
        torch, mcc = self.torch, self.mcc
        with torch.cuda.stream(stream):
            if large:
                for r in reqs:
                    d = self._upload(r)
                    out, st = mcc.consensus(d["row_ptr"], d["col"], d["labels"], d["init"],
                                            max_rounds=self.max_rounds, stream=stream)
                    r.out, r.stats = out.cpu().numpy(), st
            else:
                # the batch's requests concatenated in one upload
                pb = mcc.pack_batch(reqs)
                mcc.consensus_batch_packed(pb, max_rounds=self.max_rounds, stream=stream)
                out = pb.out.cpu().numpy()
                for j, r in enumerate(reqs):
                    c = pb.status[j]
                    if c != 0:
                        r.error = mcc.lib().mcc_strerror(c).decode()
                    o = int(pb.v_off[j])
                    r.out, r.stats = out[o:o + r.n], pb.stats[j].as_dict()
            stream.synchronize()


class Server:
    """Admission queue plus worker threads that own one stream each."""

    def __init__(self, budget_bytes: int = 16 << 30, large_n: int = 8192,
                 max_batch: int = 256, small_workers: int = 2, large_workers: int = 3,
                 max_rounds: int = 0, backend=None):
        self.backend = backend if backend is not None else GpuBackend(max_rounds)
        self.budget = int(budget_bytes)
        self.large_n = int(large_n)
        self.max_batch = int(max_batch)
        self.queue = collections.deque()
        self.cv = threading.Condition()
        self.in_use = 0
        self.running = True
        self.completed: List[Request] = []
        self.peak_in_use = 0
        self.batches = 0
        self.threads = []
        for j in range(small_workers):
            self.threads.append(threading.Thread(target=self._worker, args=(False,), daemon=True))
        for j in range(large_workers):
            self.threads.append(threading.Thread(target=self._worker, args=(True,), daemon=True))
        for t in self.threads:
            t.start()

    # -- client side ----------------------------------------------------------
    def submit(self, req: Request) -> Request:
        req.arrival = time.perf_counter()
        with self.cv:
            self.queue.append(req)
            self.cv.notify_all()
        return req

    def close(self):
        with self.cv:
            self.running = False
            self.cv.notify_all()
        for t in self.threads:
            t.join()

    # -- workers ----------------------------------------------------------------
    def _worker(self, large: bool):
        stream = self.backend.make_stream()
        while True:
            with self.cv:
                while True:
                    picked, held = admit(self.queue, self.budget, self.in_use, self.large_n,
                                         large, self.max_batch)
                    if picked:
                        break
                    mine = any((r.n > self.large_n) == large for r in self.queue)
                    if not self.running and not mine:
                        return
                    self.cv.wait(timeout=0.05)
                for r in picked:
                    self.queue.remove(r)
                self.in_use += held
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                self.batches += 1
            t0 = time.perf_counter()
            for r in picked:
                r.started = t0
            try:
                self.backend.solve(picked, large, stream)
            except Exception as e:  # reported per request, the server keeps going
                for r in picked:
                    r.error = f"{type(e).__name__}: {e}"
            t1 = time.perf_counter()
            with self.cv:
                self.in_use -= held
                for r in picked:
                    r.done_at = t1
                    self.completed.append(r)
                    r.event.set()
                self.cv.notify_all()


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


def run_served(pool: List[Request], rate: float, count: int, seed: int = 0, wait_s: float = 600.0,
               **server_kw):
    """Replay `count` requests drawn from `pool` with Poisson arrivals at
    `rate` per second through a Server; returns (requests, summary)."""
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    picks = rng.integers(0, len(pool), size=count)
    times = poisson_arrivals(rate, count, seed)
    srv = Server(**server_kw)
    reqs = []
    t0 = time.perf_counter()
    for j, (p, at) in enumerate(zip(picks, times)):
        delay = t0 + at - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        src = pool[p]
        reqs.append(srv.submit(Request(src.row_ptr, src.col, src.labels, src.init, rid=int(p))))
    deadline = time.perf_counter() + wait_s
    for r in reqs:
        if not r.event.wait(max(0.0, deadline - time.perf_counter())):
            raise TimeoutError(f"request {r.rid} not served within {wait_s} s")
    srv.close()
    summ = latency_summary(reqs)
    summ.update(batches=srv.batches, peak_in_use_bytes=srv.peak_in_use)
    return reqs, summ


def run_one_at_a_time(pool: List[Request], rate: float, count: int, seed: int = 0,
                      max_rounds: int = 0):
    """The plain path on the same arrivals: one solve at a time, in arrival
    order, with mcc_consensus on one stream."""
    import torch
    import paper_2408_11331_amd as mcc
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    picks = rng.integers(0, len(pool), size=count)
    times = poisson_arrivals(rate, count, seed)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    reqs = []
    t0 = time.perf_counter()
    for p, at in zip(picks, times):
        now = time.perf_counter()
        if now < t0 + at:
            time.sleep(t0 + at - now)
        src = pool[p]
        r = Request(src.row_ptr, src.col, src.labels, src.init, rid=int(p))
        r.arrival = t0 + at
        out, st = mcc.consensus(T(r.row_ptr), T(r.col), T(r.labels),
                                None if r.init is None else T(r.init), max_rounds=max_rounds)
        r.out, r.stats = out.cpu().numpy(), st
        r.done_at = time.perf_counter()
        reqs.append(r)
    return reqs, latency_summary(reqs)
