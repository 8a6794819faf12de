"""Seeded synthetic graphs: SBM, LFR-style and Gaussian-mixture kNN, as int32 CSR.

Every generator returns an undirected simple graph as CSR arrays
(``row_ptr`` int64[n+1], ``col`` int32[nnz], each row sorted) plus the
planted ground truth.  Nothing here computes any part of the consensus
method; these are the inputs both the oracle and the GPU library consume.
"""
from __future__ import annotations

import os
import subprocess

import numpy as np


# ----------------------------------------------------------------------------
# CSR helpers
# ----------------------------------------------------------------------------
def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray):
    """Symmetrise an edge list, drop self-loops and duplicates, return CSR.

    ``u``/``v`` are endpoint arrays of equal length (any integer dtype).
    Returns ``(row_ptr int64[n+1], col int32[nnz])`` with sorted rows.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    key = np.unique(src * n + dst)
    src = key // n
    dst = key - src * n
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, dst.astype(np.int32)


def expand_rows(row_ptr: np.ndarray, rows: np.ndarray):
    """Arc positions of the given rows: (source row per arc, arc index)."""
    starts = row_ptr[rows]
    lens = row_ptr[rows + 1] - starts
    total = int(lens.sum())
    if total == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    src = np.repeat(rows, lens)
    offs = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
    return src, offs + np.arange(total, dtype=np.int64)


def degrees(row_ptr: np.ndarray) -> np.ndarray:
    return np.diff(row_ptr)


# ----------------------------------------------------------------------------
# Stochastic block model
# ----------------------------------------------------------------------------
def _sample_pairs(rng, total: int, count: int) -> np.ndarray:
    """``count`` distinct integers drawn uniformly from ``[0, total)``."""
    if count <= 0:
        return np.zeros(0, np.int64)
    if count * 3 >= total:
        return np.sort(rng.choice(total, size=count, replace=False)).astype(np.int64)
    got = np.unique(rng.integers(0, total, size=int(count * 1.05) + 16, dtype=np.int64))
    while got.size < count:
        more = rng.integers(0, total, size=count - got.size + 16, dtype=np.int64)
        got = np.unique(np.concatenate([got, more]))
    if got.size > count:
        got = np.sort(rng.choice(got, size=count, replace=False))
    return got


def sbm(block_sizes, p_in: float, p_out: float, rng):
    """Planted-partition SBM with the given block sizes.

    Vertices are numbered block by block.  Each block pair's edge count is
    Binomial(pairs, p) and the edges are a uniform subset of that size, which
    is the same distribution as independent Bernoulli pairs.  Returns
    ``(row_ptr, col, truth)``.
    """
    sizes = np.asarray(block_sizes, dtype=np.int64)
    n = int(sizes.sum())
    first = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    us, vs = [], []
    B = sizes.size
    for a in range(B):
        sa = int(sizes[a])
        # within block a: upper triangle pairs
        tot = sa * (sa - 1) // 2
        m = int(rng.binomial(tot, min(p_in, 1.0))) if tot > 0 else 0
        t = _sample_pairs(rng, tot, m)
        if t.size:
            # invert t = i*(2*sa - i - 1)/2 + (j - i - 1)
            i = np.floor((2 * sa - 1 - np.sqrt((2 * sa - 1) ** 2 - 8.0 * t)) / 2).astype(np.int64)
            base = i * (2 * sa - i - 1) // 2
            # guard floating error
            fix = t < base
            i[fix] -= 1
            base = i * (2 * sa - i - 1) // 2
            over = t - base >= sa - i - 1
            i[over] += 1
            base = i * (2 * sa - i - 1) // 2
            j = t - base + i + 1
            us.append(first[a] + i)
            vs.append(first[a] + j)
        if p_out <= 0:
            continue
        # between block a and all later blocks at once
        if a + 1 < B:
            sb_tot = int(sizes[a + 1:].sum())
            tot = sa * sb_tot
            m = int(rng.binomial(tot, min(p_out, 1.0)))
            t = _sample_pairs(rng, tot, m)
            if t.size:
                us.append(first[a] + t // sb_tot)
                vs.append(first[a] + sa + t % sb_tot)
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    truth = np.repeat(np.arange(B, dtype=np.int32), sizes)
    row_ptr, col = csr_from_edges(n, u, v)
    return row_ptr, col, truth


# ----------------------------------------------------------------------------
# LFR-style benchmark graph (power-law degrees and community sizes, mixing mu)
# ----------------------------------------------------------------------------
def _powerlaw_mean(xmin, xmax, g):
    a, b = 1.0 - g, 2.0 - g
    return (a / b) * (xmax ** b - xmin ** b) / (xmax ** a - xmin ** a)


def _powerlaw_sample(rng, size, xmin, xmax, g):
    """Continuous power law p(x) ~ x^-g on [xmin, xmax] by inverse CDF."""
    u = rng.random(size)
    a = 1.0 - g
    return (xmin ** a + u * (xmax ** a - xmin ** a)) ** (1.0 / a)


def lfr_like(n: int, rng, gamma=2.5, mean_deg=20.0, max_deg=200, beta=1.5,
             min_comm=50, max_comm=1000, mu=0.4):
    """LFR-style graph built from the LFR recipe's description.

    Degrees follow a power law with exponent ``gamma`` on ``[d_min, max_deg]``
    with ``d_min`` solved so the mean is ``mean_deg``; community sizes follow
    a power law with exponent ``beta`` on ``[min_comm, max_comm]``.  Each
    vertex puts a fraction ``1-mu`` of its stubs inside its community; inside
    and outside stubs are wired by a configuration model, self-loops and
    multi-edges are dropped.  Returns ``(row_ptr, col, truth, info)``.
    """
    lo, hi = 1.0, float(mean_deg)
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if _powerlaw_mean(mid, max_deg, gamma) < mean_deg:
            lo = mid
        else:
            hi = mid
    d_min = 0.5 * (lo + hi)
    dr = _powerlaw_sample(rng, n, d_min, max_deg, gamma)
    deg = np.floor(dr + rng.random(n)).astype(np.int64)
    deg = np.clip(deg, 1, max_deg)

    sizes = []
    tot = 0
    while tot < n:
        s = int(np.floor(_powerlaw_sample(rng, 1, min_comm, max_comm + 1, beta)[0]))
        s = min(max(s, min_comm), max_comm)
        sizes.append(s)
        tot += s
    sizes = np.array(sizes, dtype=np.int64)
    excess = tot - n
    # trim the overshoot from the largest communities, never below min_comm
    order = np.argsort(-sizes, kind="stable")
    for c in order:
        if excess == 0:
            break
        cut = min(excess, int(sizes[c]) - min_comm)
        sizes[c] -= cut
        excess -= cut
    if excess > 0:
        sizes[order[0]] -= excess
    K = sizes.size

    d_in = np.rint((1.0 - mu) * deg).astype(np.int64)
    # cap internal degree by the largest community
    d_in = np.minimum(d_in, int(sizes.max()) - 1)
    comm = np.full(n, -1, dtype=np.int64)
    cap = sizes.copy()
    # constrained vertices (internal degree too big for the smallest
    # communities) are placed first, largest internal degree first
    constrained = np.nonzero(d_in >= min_comm - 1)[0]
    constrained = constrained[np.argsort(-d_in[constrained], kind="stable")]
    for v in constrained:
        ok = np.nonzero((sizes > d_in[v]) & (cap > 0))[0]
        if ok.size == 0:
            ok = np.nonzero(cap > 0)[0]
        c = ok[rng.integers(0, ok.size)]
        comm[v] = c
        cap[c] -= 1
    rest = np.nonzero(comm < 0)[0]
    slots = np.repeat(np.arange(K, dtype=np.int64), cap)
    rng.shuffle(slots)
    comm[rng.permutation(rest)] = slots[: rest.size]
    d_in = np.minimum(d_in, sizes[comm] - 1)
    d_out = deg - d_in

    # internal stubs: pair consecutive stubs after a random shuffle inside
    # each community
    st_v = np.repeat(np.arange(n, dtype=np.int64), d_in)
    st_c = comm[st_v]
    order = np.lexsort((rng.random(st_v.size), st_c))
    st_v, st_c = st_v[order], st_c[order]
    first_of_c = np.searchsorted(st_c, st_c, side="left")
    pos = np.arange(st_v.size) - first_of_c
    cnt = np.bincount(st_c, minlength=K)
    ok = (pos % 2 == 0) & (pos + 1 < cnt[st_c])
    a = np.nonzero(ok)[0]
    u_in, v_in = st_v[a], st_v[a + 1]
    # external stubs: one global configuration model
    ex_v = np.repeat(np.arange(n, dtype=np.int64), d_out)
    ex_v = ex_v[rng.permutation(ex_v.size)]
    m2 = ex_v.size // 2
    u_ex, v_ex = ex_v[0:2 * m2:2], ex_v[1:2 * m2:2]
    row_ptr, col = csr_from_edges(n, np.concatenate([u_in, u_ex]),
                                  np.concatenate([v_in, v_ex]))
    truth = comm.astype(np.int32)
    src = np.repeat(np.arange(n), np.diff(row_ptr))
    mu_real = float(np.mean(truth[src] != truth[col])) if col.size else 0.0
    info = dict(d_min=d_min, communities=int(K), mu_realised=mu_real,
                mean_degree=float(col.size / n))
    return row_ptr, col, truth, info


# ----------------------------------------------------------------------------
# Gaussian mixture + symmetrised kNN graph (single-cell-shaped)
# ----------------------------------------------------------------------------
def zipf_sizes(n: int, ncomp: int, a: float) -> np.ndarray:
    w = 1.0 / np.arange(1, ncomp + 1, dtype=np.float64) ** a
    w /= w.sum()
    sizes = np.floor(w * n).astype(np.int64)
    sizes[: n - int(sizes.sum())] += 1
    return sizes


def gmm_points(n: int, dim: int, ncomp: int, zipf_a: float, sigma_m: float, rng,
               scale: int = 32, clip: int = 300):
    """Points from a Gaussian mixture with unit covariance, in random order,
    on an integer grid.

    Component means are N(0, sigma_m^2 I); component sizes follow Zipf(a).
    Coordinates are rounded to multiples of 1/scale and stored as integers
    (x * scale, clipped to [-clip, clip]), so that every distance between
    points is an exact integer and the kNN graph is the same on any device.
    Returns ``(points int32[n, dim], truth int32[n])``.
    """
    sizes = zipf_sizes(n, ncomp, zipf_a)
    means = rng.normal(0.0, sigma_m, size=(ncomp, dim))
    truth = np.repeat(np.arange(ncomp, dtype=np.int32), sizes)
    perm = rng.permutation(n)
    truth = truth[perm]
    pts = rng.standard_normal(size=(n, dim), dtype=np.float32)
    pts += means[truth].astype(np.float32)
    q = np.clip(np.rint(pts * np.float32(scale)), -clip, clip).astype(np.int32)
    return q, truth


_KNN_C = os.path.join(os.path.dirname(os.path.abspath(__file__)), "knn.c")
_KNN_SO = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libknn.so")


def build_knn(force: bool = False) -> str:
    """Compile the exact CPU kNN search (knn.c) next to its source."""
    if force or not os.path.exists(_KNN_SO) or \
            os.path.getmtime(_KNN_SO) < os.path.getmtime(_KNN_C):
        tmp = _KNN_SO + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared",
                               _KNN_C, "-o", tmp, "-lm"])
        os.replace(tmp, _KNN_SO)
    return _KNN_SO


def _exact_range_ok(points: np.ndarray) -> bool:
    m = int(np.abs(points).max()) if points.size else 0
    return 4 * points.shape[1] * m * m < (1 << 24)


def knn_lists_cpu(points: np.ndarray, kk: int) -> np.ndarray:
    """Exact kNN lists (squared L2, ties to the lower index) by the
    compiled CPU search; int32[n, kk]."""
    import ctypes
    pts = np.ascontiguousarray(points, np.int32)
    n, dim = pts.shape
    out = np.empty((n, kk), np.int32)
    L = ctypes.CDLL(build_knn())
    L.knn_exact.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                            ctypes.c_void_p]
    L.knn_exact.restype = ctypes.c_int
    rc = L.knn_exact(pts.ctypes.data, n, dim, kk, out.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"knn_exact failed ({rc})")
    return out


def knn_lists_torch(points: np.ndarray, kk: int, device: str = "cpu", chunk: int = 0,
                    extra: int = 9) -> np.ndarray:
    """Exact kNN lists with torch (CPU or GPU); int32[n, kk].

    Distances of integer points are exact integers below 2^24, computed
    exactly in single precision (checked on one full row per block against
    integer arithmetic).  Each row keeps its ``kk + extra`` smallest
    distances, re-ranked by (distance, index); a row whose (kk + extra)-th
    distance still equals its kk-th (a tie that may reach past the kept
    entries) is recomputed over all points by (distance, index) keys."""
    import torch

    n, dim = points.shape
    Xl = torch.from_numpy(np.ascontiguousarray(points, np.int64)).to(device)
    X = Xl.float()
    sq = (X * X).sum(dim=1)
    if chunk <= 0:
        chunk = max(1, min(n, (1 << 28) // max(n, 1)))
    m = min(kk + extra, n - 1)
    ar = torch.arange(n, device=device, dtype=torch.int64)
    nbr = torch.empty((n, kk), dtype=torch.int64, device=device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        d = X[s:e] @ X.T
        d.mul_(-2.0).add_(sq[None, :]).add_(sq[s:e, None])
        # the block is exact: one row against integer arithmetic
        ref = ((Xl[s][None, :] - Xl) ** 2).sum(dim=1)
        if not torch.equal(d[0].long(), ref):
            raise RuntimeError("distance block is not exact on this device")
        rows = torch.arange(s, e, device=device)
        d[rows - s, rows] = float("inf")
        val, idx = torch.topk(d, m, dim=1, largest=False, sorted=True)
        key = (val.long() << 32) | idx
        key, _ = torch.sort(key, dim=1)
        nbr[s:e] = key[:, :kk] & 0xffffffff
        tied = torch.nonzero(val[:, m - 1] == val[:, kk - 1]).flatten()
        for r in tied.tolist():
            full = (d[r].long() << 32) | ar
            full[s + r] = torch.iinfo(torch.int64).max
            nbr[s + r] = torch.topk(full, kk, largest=False, sorted=True).values & 0xffffffff
        del d
    return nbr.to(torch.int32).cpu().numpy()


def knn_graph(points: np.ndarray, kk: int, device: str = "cpu", chunk: int = 0):
    """Exact symmetrised (union) kNN graph of integer points under the
    squared L2 distance, ties to the lower index.

    On the CPU the compiled search (knn.c) is used when gcc can build it,
    else torch; on a GPU, torch.  All give the same lists.  Returns
    ``(row_ptr, col)``."""
    if not _exact_range_ok(points):
        raise ValueError("point coordinates too large for exact distances")
    n = points.shape[0]
    if device == "cpu":
        try:
            nb = knn_lists_cpu(points, kk)
        except (OSError, subprocess.CalledProcessError):
            nb = knn_lists_torch(points, kk, device="cpu", chunk=chunk)
    else:
        nb = knn_lists_torch(points, kk, device=device, chunk=chunk)
    u = np.repeat(np.arange(n, dtype=np.int64), kk)
    return csr_from_edges(n, u, nb.reshape(-1))
