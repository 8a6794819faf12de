"""Brute-force definitions used to pin the oracle (test-only, numpy).

These are written from the definitions of the paper (pair indicators,
member sums), not from the oracle's closed forms, so that a slip in the
oracle (a dropped term, a wrong sign, a swapped operand) shows up as a
mismatch.
"""
from __future__ import annotations

import numpy as np


def co(a):
    """Co-clustering indicator matrix: co[u, v] = 1 iff a[u] == a[v]."""
    a = np.asarray(a)
    return a[:, None] == a[None, :]


def mirkin_pairs(a, b) -> int:
    """Ordered pairs (u, v), u != v, co-clustered in exactly one partition
    (Methods: Mirkin distance counts each disagreeing pair twice)."""
    d = co(a) != co(b)
    return int(d.sum())  # the diagonal always agrees


def objective_pairs(c, labels) -> int:
    return sum(mirkin_pairs(c, l) for l in labels)


def delta_matrix(labels):
    """delta_uv = number of input partitions that split u and v (Eq. rxyi
    summed over the partitions)."""
    labels = np.asarray(labels)
    k = labels.shape[0]
    agree = np.zeros((labels.shape[1], labels.shape[1]), dtype=np.int64)
    for l in labels:
        agree += co(l)
    return k - agree


def objective2_form(c, labels) -> int:
    """2 * [sum_{u<v} delta_uv + sum_{u<v} (k - 2 delta_uv) delta_uv(C)]: the
    reformulated objective (Eq. objective2) plus the constant the paper drops,
    doubled to ordered pairs."""
    labels = np.asarray(labels)
    k = labels.shape[0]
    D = delta_matrix(labels)
    split_c = ~co(c)
    iu = np.triu_indices(len(c), 1)
    return int(2 * (D[iu].sum() + ((k - 2 * D) * split_c)[iu].sum()))


def gain_member_sum(c, labels, v, x, literal=False) -> int:
    """Eq. objective3: sum over u of [sigma_u(x) - sigma_u(c)] (2 delta_uv - k),
    with the u = v term excluded unless ``literal``."""
    labels = np.asarray(labels)
    c = np.asarray(c)
    k = labels.shape[0]
    D = delta_matrix(labels)
    total = 0
    for u in range(len(c)):
        if u == v and not literal:
            continue
        sig_x = 1 if c[u] == x else 0
        sig_c = 1 if c[u] == c[v] else 0
        total += (sig_x - sig_c) * (2 * int(D[u, v]) - k)
    return total


def gain_by_objective(c, labels, v, x) -> int:
    """(O(after) - O(before)) / 2 with O by pair counting."""
    c = np.asarray(c).copy()
    before = objective_pairs(c, labels)
    c[v] = x
    after = objective_pairs(c, labels)
    assert (after - before) % 2 == 0
    return (after - before) // 2


def neighbour_clusters(row_ptr, col, c, v):
    s = set()
    for j in range(row_ptr[v], row_ptr[v + 1]):
        u = int(col[j])
        if u != v and c[u] != c[v]:
            s.add(int(c[u]))
    return sorted(s)


def best_move(row_ptr, col, c, labels, v, literal=False):
    """(best cluster or -1, its gain or 0, number of candidates), by member sums."""
    cands = neighbour_clusters(row_ptr, col, c, v)
    if not cands:
        return -1, 0, 0
    best = min(cands, key=lambda x: (gain_member_sum(c, labels, v, x, literal), x))
    return best, gain_member_sum(c, labels, v, best, literal), len(cands)


def set_partitions(n):
    """All set partitions of n items as restricted growth strings (B_n x n)."""
    rgs = np.zeros((1, 1), dtype=np.int8)
    mx = np.zeros(1, dtype=np.int8)
    for _ in range(1, n):
        rows, maxes = [], []
        for val in range(0, int(mx.max()) + 2):
            ok = val <= mx + 1
            r = rgs[ok]
            rows.append(np.concatenate([r, np.full((r.shape[0], 1), val, np.int8)], axis=1))
            maxes.append(np.maximum(mx[ok], val))
        rgs = np.concatenate(rows)
        mx = np.concatenate(maxes).astype(np.int8)
    return rgs


def objective_all(parts, labels):
    """O for every row of ``parts`` (B x n) by pair counting, vectorised."""
    labels = np.asarray(labels)
    k = labels.shape[0]
    n = labels.shape[1]
    A = k - delta_matrix(labels)           # agreements per pair
    off = ~np.eye(n, dtype=bool)
    coC = parts[:, :, None] == parts[:, None, :]
    # a pair co-clustered in C disagrees with the partitions that split it
    # (k - A); a pair split in C disagrees with those that join it (A)
    per_pair = np.where(coC, k - A[None], A[None]) * off[None]
    return per_pair.reshape(parts.shape[0], -1).sum(axis=1)
