"""Seeded perturbations that turn a ground truth into k input partitions.

The input partitions of the paper come from repeated runs of community
detection algorithms (Results, "Input partitions"); those runs are not
reproducible here, so each partition is the truth with neighbour-label
reassignment plus resolution changes (merges of adjacent communities and
splits of large ones).  None of this is part of the consensus method.
"""
from __future__ import annotations

import numpy as np

from .graph import expand_rows


def relabel_dense(labels: np.ndarray) -> np.ndarray:
    """Map labels onto ``[0, L)`` (sorted-value order), int32."""
    _, inv = np.unique(labels, return_inverse=True)
    return inv.astype(np.int32)


def random_neighbour(row_ptr, col, verts, rng):
    """A uniformly random neighbour of each vertex in ``verts`` (-1 if isolated)."""
    deg = row_ptr[verts + 1] - row_ptr[verts]
    pick = np.floor(rng.random(verts.size) * np.maximum(deg, 1)).astype(np.int64)
    nb = col[np.minimum(row_ptr[verts] + pick, max(col.size - 1, 0))].astype(np.int64) if col.size else np.full(verts.size, -1)
    return np.where(deg > 0, nb, -1)


def reassign(base: np.ndarray, row_ptr, col, count: int, rng,
             source: np.ndarray | None = None) -> np.ndarray:
    """``count`` vertices, drawn without replacement, each take the label
    (in ``source``, default ``base``) of a uniformly random neighbour;
    isolated vertices keep theirs."""
    n = base.size
    src = base if source is None else source
    out = base.copy()
    count = min(int(count), n)
    if count <= 0:
        return out
    verts = rng.choice(n, size=count, replace=False).astype(np.int64)
    nb = random_neighbour(row_ptr, col, verts, rng)
    has = nb >= 0
    out[verts[has]] = src[nb[has]]
    return out


def community_adjacency(labels: np.ndarray, row_ptr, col) -> np.ndarray:
    """Sorted unique pairs (a, b), a < b, of communities joined by an edge."""
    K = int(labels.max()) + 1 if labels.size else 0
    src = np.repeat(np.arange(labels.size, dtype=np.int64), np.diff(row_ptr))
    a = labels[src].astype(np.int64)
    b = labels[col].astype(np.int64)
    m = a < b
    key = np.unique(a[m] * K + b[m])
    return np.stack([key // K, key % K], axis=1)


def merge(labels: np.ndarray, pairs: np.ndarray, count: int, rng) -> np.ndarray:
    """Merge ``count`` random communities each into a random adjacent one."""
    out = labels.copy()
    if count <= 0 or pairs.shape[0] == 0:
        return out
    K = int(labels.max()) + 1
    parent = np.arange(K)

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for _ in range(count):
        e = pairs[rng.integers(0, pairs.shape[0])]
        ra, rb = find(int(e[0])), find(int(e[1]))
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    root = np.array([find(x) for x in range(K)])
    return root[out].astype(labels.dtype)


def _split_plan(labels, rng, min_factor=2.0, prob=0.25, parts=(2, 3, 4)):
    sizes = np.bincount(labels)
    present = np.nonzero(sizes)[0]
    med = float(np.median(sizes[present]))
    big = present[sizes[present] >= min_factor * med]
    plan = []
    for c in big:
        if rng.random() < prob:
            plan.append((int(c), int(parts[rng.integers(0, len(parts))])))
    return plan


def split_bfs(labels: np.ndarray, row_ptr, col, rng, min_factor=2.0, prob=0.25,
              parts=(2, 3, 4)) -> np.ndarray:
    """Split each community of size >= ``min_factor`` x median, with
    probability ``prob``, into 2-4 parts grown by a multi-source BFS inside
    the community from random member seeds.  A vertex reached at the same
    depth from several seeds joins the lowest seed index; members no seed
    reaches stay with the first seed's part."""
    plan = _split_plan(labels, rng, min_factor, prob, parts)
    out = labels.astype(np.int64).copy()
    if not plan:
        return out.astype(np.int32)
    n = labels.size
    part = np.full(n, -1, dtype=np.int64)
    next_label = int(labels.max()) + 1
    seed_label = []
    frontier = []
    for c, p in plan:
        members = np.nonzero(labels == c)[0]
        seeds = rng.choice(members, size=min(p, members.size), replace=False)
        for j, s in enumerate(seeds):
            idx = len(seed_label)
            seed_label.append(c if j == 0 else next_label)
            if j:
                next_label += 1
            part[s] = idx
            frontier.append(s)
    frontier = np.array(frontier, dtype=np.int64)
    while frontier.size:
        src, arcs = expand_rows(row_ptr, frontier)
        dst = col[arcs].astype(np.int64)
        ok = (part[dst] < 0) & (labels[dst] == labels[src])
        d, p = dst[ok], part[src[ok]]
        if d.size == 0:
            break
        order = np.lexsort((p, d))
        d, p = d[order], p[order]
        first = np.ones(d.size, dtype=bool)
        first[1:] = d[1:] != d[:-1]
        d, p = d[first], p[first]
        part[d] = p
        frontier = d
    seed_label = np.array(seed_label, dtype=np.int64)
    hit = part >= 0
    out[hit] = seed_label[part[hit]]
    return out.astype(np.int32)


def split_voronoi(labels: np.ndarray, points: np.ndarray, rng, min_factor=2.0,
                  prob=0.25, parts=(2, 3, 4)) -> np.ndarray:
    """Resolution change for point data: split each chosen community by the
    nearest of 2-4 random member points (feature-space Voronoi cells).
    ``points`` are integers; distances are exact (int64) and ties go to the
    first seed."""
    plan = _split_plan(labels, rng, min_factor, prob, parts)
    out = labels.astype(np.int64).copy()
    next_label = int(labels.max()) + 1
    for c, p in plan:
        members = np.nonzero(labels == c)[0]
        seeds = rng.choice(members, size=min(p, members.size), replace=False)
        X = points[members].astype(np.int64)
        S = points[seeds].astype(np.int64)
        d = (X * X).sum(1)[:, None] - 2 * (X @ S.T) + (S * S).sum(1)[None, :]
        near = np.argmin(d, axis=1)
        newl = np.array([c] + list(range(next_label, next_label + len(seeds) - 1)))
        next_label += len(seeds) - 1
        out[members] = newl[near]
    return out.astype(np.int32)
