"""Pins of the oracle's partition-comparison metrics and grouping step
(Results, "Evaluation metrics"; Methods, "Grouping homogeneous
partitions") against library routines, closed forms and the metric axioms.

Readings (the paper names the measures and cites their definitions):
split-join distance = 2n - sum_A max_B |A n B| - sum_B max_A |A n B|;
variation of information = H(A) + H(B) - 2 I(A; B) in nats; Rand distance =
one minus the Rand index = Mirkin / (n (n - 1)) over ordered pairs."""
import math

import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.csgraph
import scipy.stats
import sklearn.metrics

import oracle

RNG = np.random.Generator(np.random.PCG64(2024))


def rand_partition(n, m, rng=RNG):
    return (rng.integers(0, m, size=n) * 7919 % 100_003).astype(np.int32)


# ------------------------------------------------------------ worked case ----
def test_hand_example():
    # a = {0,1}{2,3}{4}, b = {0,1,2}{3,4}; intersections 2,1,1,1:
    # rows of a take 2+1+1, rows of b take 2+1 -> split-join 1 + 2;
    # VI = (4 ln 2 + 3 ln 3 + 2 ln 2 - 2 * 2 ln 2) / 5; Mirkin 9 + 13 - 14
    r = oracle.compare([0, 0, 1, 1, 2], [0, 0, 0, 1, 1])
    assert (r["split_join_ab"], r["split_join_ba"], r["split_join"]) == (1, 2, 3)
    assert r["mirkin"] == 8 and r["rand"] == 8 / 20
    assert r["vi"] == pytest.approx((2 * math.log(2) + 3 * math.log(3)) / 5, rel=1e-14)
    assert (r["clusters_a"], r["clusters_b"]) == (3, 2)


# ------------------------------------------------------- library routines ----
@pytest.mark.parametrize("n,ma,mb", [(1, 1, 1), (2, 2, 1), (50, 3, 7), (1000, 40, 5),
                                     (5000, 700, 700)])
def test_rand_and_vi_against_sklearn_scipy(n, ma, mb):
    a, b = rand_partition(n, ma), rand_partition(n, mb)
    r = oracle.compare(a, b)
    if n > 1:
        assert r["rand"] == pytest.approx(1.0 - sklearn.metrics.rand_score(a, b), abs=1e-12)
    ha = scipy.stats.entropy(np.unique(a, return_counts=True)[1])
    hb = scipy.stats.entropy(np.unique(b, return_counts=True)[1])
    mi = sklearn.metrics.mutual_info_score(a, b)
    assert r["vi"] == pytest.approx(ha + hb - 2 * mi, rel=1e-10, abs=1e-12)
    assert r["mirkin"] == oracle.mirkin(a, b)


# ------------------------------------------------------------ closed forms ---
def test_closed_forms():
    n = 37
    one, single = np.zeros(n, np.int32), np.arange(n, dtype=np.int32)
    r = oracle.compare(one, single)
    # one cluster against singletons: every singleton lies in the one cluster
    # (nothing to join from that side), the one cluster keeps 1 element
    assert (r["split_join_ab"], r["split_join_ba"]) == (n - 1, 0)
    assert r["vi"] == pytest.approx(math.log(n), rel=1e-14)
    assert r["rand"] == 1.0
    # identical partitions (any labels)
    a = rand_partition(n, 5)
    r = oracle.compare(a, (a * 3 + 11).astype(np.int32))
    assert r["split_join"] == 0 and r["vi"] == 0.0 and r["mirkin"] == 0
    # b refines a: each cluster of b inside one cluster of a, so the b side
    # costs nothing and the a side loses all but its largest piece
    a = np.repeat(np.arange(4), [5, 7, 3, 9]).astype(np.int32)
    b = np.concatenate([[0, 0, 0, 1, 1], [2] * 4 + [3] * 3, [4, 5, 6], [7] * 9]).astype(np.int32)
    r = oracle.compare(a, b)
    assert r["split_join_ba"] == 0 and r["split_join_ab"] == 24 - (3 + 4 + 1 + 9)
    # independent halves: A = v mod 2, B = (v div 2) mod 2 on n = 4m share no
    # information: VI = H(A) + H(B) = 2 ln 2
    v = np.arange(400)
    r = oracle.compare((v % 2).astype(np.int32), ((v // 2) % 2).astype(np.int32))
    assert r["vi"] == pytest.approx(2 * math.log(2), rel=1e-14)


# ------------------------------------------------------------ metric axioms --
def test_metric_axioms():
    for _ in range(30):
        n = int(RNG.integers(1, 300))
        a, b, c = (rand_partition(n, int(RNG.integers(1, 20))) for _ in range(3))
        ab, ba, ac, bc = (oracle.compare(x, y) for x, y in ((a, b), (b, a), (a, c), (b, c)))
        assert ab["split_join"] == ba["split_join"]
        assert (ab["split_join_ab"], ab["split_join_ba"]) == (ba["split_join_ba"], ba["split_join_ab"])
        assert ab["vi"] == pytest.approx(ba["vi"], abs=1e-12)
        assert ac["split_join"] <= ab["split_join"] + bc["split_join"]
        assert ac["vi"] <= ab["vi"] + bc["vi"] + 1e-12
        assert ac["mirkin"] <= ab["mirkin"] + bc["mirkin"]
        assert min(ab["split_join_ab"], ab["split_join_ba"]) >= 0 and ab["vi"] >= -1e-12
        # relabelling invariance
        perm = RNG.permutation(100_003).astype(np.int32)
        r = oracle.compare(perm[a], b)
        assert r["split_join"] == ab["split_join"] and r["mirkin"] == ab["mirkin"]


# --------------------------------------------------------------- grouping ----
def test_split_join_matrix():
    labels = np.stack([rand_partition(300, m) for m in (2, 3, 3, 9, 30, 1)])
    d = oracle.split_join_matrix(labels)
    assert (d == d.T).all() and (np.diag(d) == 0).all()
    for i in range(6):
        for j in range(6):
            assert d[i, j] == oracle.compare(labels[i], labels[j])["split_join"]


@pytest.mark.parametrize("seed", range(6))
def test_group_against_scipy_components(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    k = int(rng.integers(1, 25))
    d = rng.integers(0, 100, size=(k, k))
    d = np.triu(d, 1)
    d = d + d.T
    lam = int(rng.integers(0, 100))
    g, ng = oracle.group(d, lam)
    adj = scipy.sparse.csr_matrix((d <= lam).astype(np.int8))
    nc, lab = scipy.sparse.csgraph.connected_components(adj, directed=False)
    assert ng == nc
    # same partition, numbered in order of the smallest member
    _, first = np.unique(lab, return_index=True)
    order = np.argsort(np.argsort(first))
    assert np.array_equal(g, order[lab])


def test_elbow_hand_case():
    # three tight pairs (distance 1), joined into one group at 2 and 3; every
    # other pair at 100: groups 3, 2, 1, 1 at t = 1, 2, 3, 100.  Scaled, the
    # points are (0, 1), (1/99, 1/2), (2/99, 0), (1, 0); the farthest below
    # the chord x + y = 1 is t = 3
    k = 6
    d = np.full((k, k), 100, np.int64)
    np.fill_diagonal(d, 0)
    for i, j, w in ((0, 1, 1), (2, 3, 1), (4, 5, 1), (1, 2, 2), (3, 4, 3)):
        d[i, j] = d[j, i] = w
    assert oracle.elbow_lambda(d) == 3
    g, ng = oracle.group(d, 3)
    assert ng == 1 and (g == 0).all()
    assert oracle.group(d, 2)[1] == 2 and oracle.group(d, 0)[1] == 6
    # degenerate cases
    assert oracle.elbow_lambda(np.zeros((1, 1), np.int64)) == 0
    two = np.array([[0, 5], [5, 0]])
    assert oracle.elbow_lambda(two) == 5
