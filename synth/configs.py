"""The benchmark workloads as seeded synthetic instances.

Each builder returns an ``Instance``: CSR graph, ``k`` input partitions laid
out partition-major (``labels[i, v]``), the initial consensus (input
partition 0) and a small manifest of realised statistics.

Seeds: the master seed of workload ``w`` is ``20240821 + w``; the graph uses
``PCG64(master)`` and input partition ``i`` uses ``PCG64([master, i + 1])``.

Workloads (sizes are the full ones; every builder also takes a smaller ``n``
for tests that the oracle must finish in seconds):

* ``sbm_small``  - planted partition, n=1000, 10 blocks, p_in=0.1, p_out=0.005,
  k=10 partitions = truth with 200 vertices given a random neighbour's truth label.
* ``lfr``        - LFR-style n=100000, degree exponent 2.5 (mean 20, max 200),
  community-size exponent 1.5 in [50, 1000], mu=0.4; k=32 partitions with
  10-50% reassignment, merges and BFS splits.
* ``gmm_knn``    - 2,000,000 points of a 50-component Gaussian mixture in 30-d
  (Zipf 1.2 sizes), symmetrised 15-NN graph; k=50 partitions with 5-40%
  reassignment, merges and feature-space splits.
* ``sbm_batch``  - many independent SBM instances of random size and k.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np

from . import graph as G
from . import perturb as P

MASTER = 20240821


def graph_rng(w: int):
    return np.random.Generator(np.random.PCG64(MASTER + w))


def part_rng(w: int, i: int):
    return np.random.Generator(np.random.PCG64([MASTER + w, i + 1]))


@dataclasses.dataclass
class Instance:
    name: str
    row_ptr: np.ndarray      # int64[n+1]
    col: np.ndarray          # int32[nnz]
    labels: np.ndarray       # int32[k, n], partition-major
    init: np.ndarray         # int32[n]
    truth: np.ndarray        # int32[n]
    meta: dict

    @property
    def n(self) -> int:
        return int(self.row_ptr.size - 1)

    @property
    def k(self) -> int:
        return int(self.labels.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.col.size)

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.row_ptr, self.col, self.labels, self.init):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def _finish(name, row_ptr, col, labels, truth, meta):
    labels = np.ascontiguousarray(np.stack(labels).astype(np.int32))
    meta = dict(meta)
    meta.update(n=int(row_ptr.size - 1), nnz=int(col.size), k=int(labels.shape[0]),
                mean_degree=float(col.size / max(1, row_ptr.size - 1)),
                labels_per_partition=[int(l.max()) + 1 for l in labels])
    return Instance(name, row_ptr, col, labels, labels[0].copy(), truth.astype(np.int32), meta)


def sbm_partitions(truth, row_ptr, col, k, count, w, first_part=0):
    out = []
    for i in range(k):
        rng = part_rng(w, first_part + i)
        out.append(P.reassign(truth, row_ptr, col, count, rng))
    return out


def sbm_small(n_blocks=10, block=100, p_in=0.1, p_out=0.005, k=10, reassigned=200, w=0):
    rng = graph_rng(w)
    row_ptr, col, truth = G.sbm([block] * n_blocks, p_in, p_out, rng)
    labels = sbm_partitions(truth, row_ptr, col, k, reassigned, w)
    return _finish("sbm_small", row_ptr, col, labels, truth,
                   dict(workload=w, blocks=n_blocks, p_in=p_in, p_out=p_out, reassigned=reassigned))


def perturbed_partitions(truth, row_ptr, col, k, w, rate=(0.10, 0.50), merge_frac=0.05,
                         points=None):
    """k partitions: merges of adjacent communities, splits of large ones,
    then reassignment of a random fraction to a random neighbour's label."""
    pairs = P.community_adjacency(truth, row_ptr, col)
    K = int(truth.max()) + 1
    out = []
    for i in range(k):
        rng = part_rng(w, i)
        r = rng.uniform(rate[0], rate[1])
        m = int(rng.integers(0, int(math.floor(merge_frac * K)) + 1))
        lab = P.merge(truth, pairs, m, rng)
        if points is None:
            lab = P.split_bfs(lab, row_ptr, col, rng)
        else:
            lab = P.split_voronoi(lab, points, rng)
        lab = P.reassign(lab, row_ptr, col, int(round(r * truth.size)), rng)
        out.append(P.relabel_dense(lab))
    return out


def lfr(n=100_000, k=32, w=1, mean_deg=20.0, max_deg=200, mu=0.4,
        min_comm=50, max_comm=1000):
    rng = graph_rng(w)
    row_ptr, col, truth, info = G.lfr_like(n, rng, mean_deg=mean_deg, max_deg=max_deg,
                                          mu=mu, min_comm=min_comm, max_comm=max_comm)
    labels = perturbed_partitions(truth, row_ptr, col, k, w)
    return _finish("lfr", row_ptr, col, labels, truth, dict(workload=w, **info))


def gmm_knn(n=2_000_000, k=50, w=2, dim=30, ncomp=50, zipf_a=1.2, sigma_m=0.8, nn=15,
            device="cpu", chunk=0):
    rng = graph_rng(w)
    pts, truth = G.gmm_points(n, dim, ncomp, zipf_a, sigma_m, rng)
    row_ptr, col = G.knn_graph(pts, nn, device=device, chunk=chunk)
    labels = perturbed_partitions(truth, row_ptr, col, k, w, rate=(0.05, 0.40), points=pts)
    src = np.repeat(np.arange(n), np.diff(row_ptr))
    mu = float(np.mean(truth[src] != truth[col])) if col.size else 0.0
    return _finish("gmm_knn", row_ptr, col, labels, truth,
                   dict(workload=w, dim=dim, components=ncomp, sigma_m=sigma_m, nn=nn,
                        mu_realised=mu, undirected_edges=int(col.size // 2)))


def sbm_batch_specs(count=4096, w=3, n_range=(200, 20_000), b_range=(4, 64),
                    d_range=(8, 32), mu_range=(0.1, 0.5), k_range=(8, 64)):
    """Per-instance parameters of the batched workload (no graphs built)."""
    rng = graph_rng(w)
    specs = []
    for j in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        B = int(rng.integers(b_range[0], b_range[1] + 1))
        B = min(B, n)
        d = float(rng.uniform(*d_range))
        mu = float(rng.uniform(*mu_range))
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        specs.append(dict(index=j, n=n, blocks=B, degree=d, mu=mu, k=k))
    return specs


def sbm_batch_instance(spec, w=3):
    """One instance of the batched workload from its spec (seeded per index)."""
    j = spec["index"]
    rng = np.random.Generator(np.random.PCG64([MASTER + w, 1_000_000 + j]))
    n, B = spec["n"], spec["blocks"]
    sizes = np.full(B, n // B, dtype=np.int64)
    sizes[: n - int(sizes.sum())] += 1
    bs = n / B
    p_in = min(1.0, (1 - spec["mu"]) * spec["degree"] / max(bs - 1, 1))
    p_out = spec["mu"] * spec["degree"] / max(n - bs, 1)
    row_ptr, col, truth = G.sbm(sizes, p_in, p_out, rng)
    labels = []
    for i in range(spec["k"]):
        prng = np.random.Generator(np.random.PCG64([MASTER + w, 1_000_000 + j, i + 1]))
        labels.append(P.reassign(truth, row_ptr, col, int(round(0.2 * n)), prng))
    return _finish("sbm_batch", row_ptr, col, labels, truth,
                   dict(workload=w, p_in=p_in, p_out=p_out, **spec))


def random_instance(n, k, avg_deg, n_labels, seed, init="p0", self_loops=0, dup_arcs=0):
    """Small unstructured instance for property tests: G(n, p) graph (plus
    optional self-loops and duplicate arcs), k independent random label
    vectors drawn from ``n_labels`` values (not necessarily contiguous)."""
    rng = np.random.Generator(np.random.PCG64([MASTER + 100, seed]))
    m = int(rng.binomial(n * (n - 1) // 2, min(1.0, avg_deg / max(n - 1, 1)))) if n > 1 else 0
    u = rng.integers(0, n, size=m)
    v = rng.integers(0, n, size=m)
    row_ptr, col = G.csr_from_edges(n, u, v)
    if self_loops or dup_arcs:
        src = list(np.repeat(np.arange(n), np.diff(row_ptr)))
        dst = list(col)
        for _ in range(self_loops):
            x = int(rng.integers(0, n))
            src.append(x)
            dst.append(x)
        for _ in range(dup_arcs):
            if len(src):
                t = int(rng.integers(0, len(src)))
                src.append(src[t])
                dst.append(dst[t])
        src = np.array(src, dtype=np.int64)
        dst = np.array(dst, dtype=np.int64)
        order = np.lexsort((dst, src))
        src, dst = src[order], dst[order]
        row_ptr = np.zeros(n + 1, np.int64)
        np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
        col = dst.astype(np.int32)
    vals = rng.choice(np.arange(0, 5 * n_labels + 7), size=n_labels, replace=False)
    labels = vals[rng.integers(0, n_labels, size=(k, n))].astype(np.int32)
    if init == "p0":
        ini = labels[0].copy()
        # init IDs must be vertex IDs range [0, n): use the dense form
        ini = P.relabel_dense(ini)
    elif init == "singleton":
        ini = np.arange(n, dtype=np.int32)
    else:
        ini = rng.integers(0, n, size=n).astype(np.int32)
    return Instance("random", row_ptr, col, np.ascontiguousarray(labels), ini.astype(np.int32),
                    labels[0].copy(), dict(n=n, k=k, seed=seed))


SERVED_LARGE = (200_000, 500_000, 1_000_000)


def served_pool_specs(small=16, large=SERVED_LARGE):
    """The request pool of the served workload: ``small`` LFR-style graphs
    with n log-uniform in [1000, 50000] and k uniform in [4, 16], and large
    ones (the given sizes, mean degree 16, k = 32).  Arrivals draw small
    requests four times as often as large ones in total (80/20)."""
    rng = np.random.Generator(np.random.PCG64(MASTER + 4))
    specs = []
    for j in range(small):
        n = int(np.exp(rng.uniform(np.log(1000), np.log(50_000))))
        specs.append(dict(index=j, n=n, k=int(rng.integers(4, 17)), large=False))
    for j, n in enumerate(large):
        specs.append(dict(index=small + j, n=int(n), k=32, large=True))
    return specs


def served_instance(spec):
    """One request of the served pool (seeded by its index)."""
    n = spec["n"]
    inst = lfr(n=n, k=spec["k"], w=4 + 1000 + spec["index"],
               mean_deg=16.0 if spec["large"] else 20.0, max_deg=200, min_comm=50,
               max_comm=1000)
    inst.name = "served"
    inst.meta.update(spec)
    return inst
