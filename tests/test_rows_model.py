"""A host model of the hashed row table's sizing rule (CPU only).

The row table keeps one row of k counts per key (cluster x, label id l),
where the label ids of every partition have been relabelled injectively
(aligned to partition 0's labels).  The library sizes it from T0, the sum
over vertices of their distinct label ids, on two claims:

  * no clustering has more live rows (keys with a nonzero count) than T0:
    each live row (x, l) has a member of x holding id l, and a vertex holds
    at most its own distinct ids;
  * a batch of moves adds at most the sum of the movers' distinct ids as new
    keys to the rows already present (a mover v adds at most the keys
    (target, l) for its own ids l).

These tests check both claims on random instances and clusterings, and that
any injective relabelling leaves every count unchanged (so the alignment
cannot change a result).  They model the rule, not the kernels; the GPU
side is checked by the parity and golden tests in both hashed layouts.
"""
import numpy as np


def live_rows(C, A):
    """Distinct (cluster, id) keys over all vertices and partitions."""
    k, n = A.shape
    keys = (np.repeat(C[None, :].astype(np.int64), k, 0) << 32) | A.astype(np.int64)
    return np.unique(keys).size


def distinct_ids(A):
    S = np.sort(A.T, axis=1)
    return 1 + (S[:, 1:] != S[:, :-1]).sum(axis=1)


def counts(C, A):
    """The contingency counts as a dict (cluster, partition, id) -> count."""
    out = {}
    for i in range(A.shape[0]):
        for x, l in zip(C.tolist(), A[i].tolist()):
            out[(x, i, l)] = out.get((x, i, l), 0) + 1
    return out


def instance(rng, n, k, labels):
    base = rng.integers(0, labels, n)
    A = np.empty((k, n), np.int64)
    for i in range(k):
        lab = base.copy()
        flip = rng.random(n) < rng.uniform(0.0, 0.5)
        lab[flip] = rng.integers(0, labels + 3, int(flip.sum()))
        A[i] = lab
    return A


def test_live_rows_never_exceed_the_singletons_bound():
    rng = np.random.default_rng(11)
    for _ in range(60):
        n = int(rng.integers(1, 300))
        k = int(rng.integers(1, 12))
        A = instance(rng, n, k, int(rng.integers(1, 9)))
        T0 = int(distinct_ids(A).sum())
        assert live_rows(np.arange(n), A) == T0  # singletons reach it
        for K in (1, 2, 5, max(1, n // 3), n):
            C = rng.integers(0, K, n)
            assert live_rows(C, A) <= T0


def test_a_batch_adds_at_most_its_movers_distinct_ids():
    rng = np.random.default_rng(12)
    for _ in range(60):
        n = int(rng.integers(2, 300))
        k = int(rng.integers(1, 12))
        A = instance(rng, n, k, int(rng.integers(1, 9)))
        d = distinct_ids(A)
        C = rng.integers(0, int(rng.integers(1, n + 1)), n)
        before = (np.repeat(C[None, :].astype(np.int64), k, 0) << 32) | A
        movers = rng.random(n) < rng.uniform(0.0, 1.0)
        C2 = C.copy()
        C2[movers] = rng.integers(0, n, int(movers.sum()))
        after = (np.repeat(C2[None, :].astype(np.int64), k, 0) << 32) | A
        # keys present before the batch are never removed (a count that drops
        # to zero keeps its key until a rebuild), so the table then holds the
        # union of both key sets
        new = np.setdiff1d(np.unique(after), np.unique(before)).size
        assert new <= int(d[movers].sum())
        # the sizing: live rows plus the additions stay within 2 T0
        assert live_rows(C, A) + int(d[movers].sum()) <= 2 * int(d.sum())


def test_injective_relabelling_keeps_every_count():
    rng = np.random.default_rng(13)
    for _ in range(20):
        n = int(rng.integers(1, 120))
        k = int(rng.integers(1, 6))
        A = instance(rng, n, k, 6)
        C = rng.integers(0, max(1, n // 4), n)
        B = A.copy()
        maps = []
        for i in range(k):
            perm = rng.permutation(64) + 100 * i  # any injective map per partition
            B[i] = perm[A[i]]
            maps.append(perm)
        ca, cb = counts(C, A), counts(C, B)
        assert sorted(ca.values()) == sorted(cb.values())
        for (x, i, l), c in ca.items():
            assert cb[(x, i, int(maps[i][l]))] == c
