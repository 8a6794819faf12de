"""Pins of the CPU oracle against definitions, closed forms, brute force and a
hand-worked trace.  CPU only."""
import json
import os

import numpy as np
import pytest

import bruteforce as bf
import oracle
import synth
from synth import graph as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="session", autouse=True)
def _built():
    oracle.build()


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def complete_graph(n):
    u, v = np.triu_indices(n, 1)
    return G.csr_from_edges(n, u, v)


def random_labels(r, k, n, nl):
    return r.integers(0, nl, size=(k, n)).astype(np.int32)


# ---------------------------------------------------------------- Mirkin ----
@pytest.mark.parametrize("seed", range(12))
def test_mirkin_matches_pair_count(seed):
    r = rng(seed)
    n = int(r.integers(1, 300))
    a = r.integers(0, int(r.integers(1, 40)), size=n)
    b = r.integers(0, int(r.integers(1, 40)), size=n)
    if seed % 3 == 0:  # large, sparse label values
        a = a * 1_000_003 % (2**31 - 1)
    assert oracle.mirkin(a, b) == bf.mirkin_pairs(a, b)


def test_mirkin_axioms():
    r = rng(99)
    for _ in range(20):
        n = int(r.integers(2, 120))
        a, b, c = (r.integers(0, int(r.integers(1, 12)), size=n) for _ in range(3))
        assert oracle.mirkin(a, a) == 0
        assert oracle.mirkin(a, b) == oracle.mirkin(b, a)
        assert oracle.mirkin(a, c) <= oracle.mirkin(a, b) + oracle.mirkin(b, c)
        perm = r.permutation(int(a.max()) + 1) * 7 + 3  # relabelling
        assert oracle.mirkin(perm[a], b) == oracle.mirkin(a, b)
    for n in (1, 2, 5, 1000):
        one = np.zeros(n, np.int32)
        single = np.arange(n, dtype=np.int32)
        assert oracle.mirkin(one, single) == n * (n - 1)


def test_mirkin_empty():
    assert oracle.mirkin(np.zeros(0, np.int32), np.zeros(0, np.int32)) == 0


# ------------------------------------------------------------- objective ----
@pytest.mark.parametrize("seed", range(8))
def test_objective_pair_count_and_objective2_identity(seed):
    r = rng(100 + seed)
    n = int(r.integers(2, 90))
    k = int(r.integers(1, 9))
    labels = random_labels(r, k, n, int(r.integers(1, 8)))
    c = r.integers(0, n, size=n).astype(np.int32)
    o = oracle.objective(c, labels)
    assert o == bf.objective_pairs(c, labels)
    assert o == bf.objective2_form(c, labels)


# ------------------------------------------------------------------ gain ----
@pytest.mark.parametrize("seed", range(10))
def test_gain_three_ways_every_move(seed):
    r = rng(200 + seed)
    n = int(r.integers(2, 28))
    k = int(r.integers(1, 7))
    labels = random_labels(r, k, n, int(r.integers(1, 5)))
    c = r.integers(0, max(1, n // 3), size=n).astype(np.int32)
    for v in range(n):
        for x in sorted(set(c.tolist()) - {int(c[v])}):
            closed = oracle.delta(c, labels, v, x)
            assert closed == bf.gain_member_sum(c, labels, v, x)
            assert closed == bf.gain_by_objective(c, labels, v, x)
            # the paper's printed sum keeps the u = v term, k more
            assert bf.gain_member_sum(c, labels, v, x, literal=True) == closed + k


@pytest.mark.parametrize("seed", range(6))
def test_score_matches_member_sum_argmin(seed):
    r = rng(300 + seed)
    inst = synth.random_instance(int(r.integers(3, 40)), int(r.integers(1, 6)),
                                 avg_deg=4.0, n_labels=4, seed=seed, self_loops=3,
                                 dup_arcs=5)
    c = r.integers(0, max(1, inst.n // 4), size=inst.n).astype(np.int32)
    for literal in (False, True):
        best, dbest, ncand = oracle.score(inst.row_ptr, inst.col, inst.labels, c,
                                          literal=literal)
        for v in range(inst.n):
            eb, ed, en = bf.best_move(inst.row_ptr, inst.col, c, inst.labels, v, literal)
            assert (best[v], dbest[v], ncand[v]) == (eb, ed, en), v


# ------------------------------------------------------------ exhaustive ----
@pytest.mark.parametrize("n,seed", [(7, 0), (8, 1), (9, 2), (10, 3)])
def test_exhaustive_median(n, seed):
    r = rng(400 + seed)
    k = int(r.integers(2, 6))
    labels = random_labels(r, k, n, 3)
    parts = bf.set_partitions(n)
    all_o = bf.objective_all(parts, labels)
    gmin = int(all_o.min())
    # the oracle's objective agrees with brute force on a sample of partitions
    idx = r.choice(parts.shape[0], size=min(400, parts.shape[0]), replace=False)
    for j in idx:
        assert oracle.objective(parts[j].astype(np.int32), labels) == int(all_o[j])
    rp, col = complete_graph(n)
    for init in (None, labels[0]):
        out, st, _ = oracle.consensus(rp, col, labels, init=init)
        assert st["converged"] == 1
        assert st["objective"] == bf.objective_pairs(out, labels) >= gmin
        # on a complete graph every existing cluster is a candidate: the
        # output is a local minimum under single-vertex moves between clusters
        for v in range(n):
            for x in set(out.tolist()) - {int(out[v])}:
                assert bf.gain_member_sum(out, labels, v, x) >= 0


# --------------------------------------------------------- special cases ----
def test_golden_s5_trace():
    g = json.load(open(os.path.join(GOLDEN, "s5_k6_trace.json")))
    rp, col = complete_graph(g["n"])
    out, st, tr = oracle.consensus(rp, col, np.array(g["labels"], np.int32),
                                   init=np.array(g["init"], np.int32), trace=True)
    e = g["expected"]
    assert out.tolist() == e["out"]
    for key in ("passes", "moves", "fallback_rounds", "converged", "objective_init",
                "objective", "candidate_evals"):
        assert st[key] == e[key], key
    assert tr.tolist() == e["trace"]


def _connected_blocks(r, n_blocks, size):
    # each block a path plus random chords, blocks joined by a few edges
    us, vs = [], []
    for b in range(n_blocks):
        base = b * size
        for j in range(size - 1):
            us.append(base + j)
            vs.append(base + j + 1)
        for _ in range(size):
            us.append(base + int(r.integers(0, size)))
            vs.append(base + int(r.integers(0, size)))
    for _ in range(n_blocks * 2):
        us.append(int(r.integers(0, n_blocks * size)))
        vs.append(int(r.integers(0, n_blocks * size)))
    return G.csr_from_edges(n_blocks * size, np.array(us), np.array(vs))


@pytest.mark.parametrize("k", [1, 4])
def test_s1_identical_partitions_from_singletons(k):
    r = rng(500 + k)
    nb, size = 5, 12
    rp, col = _connected_blocks(r, nb, size)
    p = np.repeat(np.arange(nb), size).astype(np.int32)
    labels = np.stack([p] * k)
    out, st, _ = oracle.consensus(rp, col, labels, init=None)
    assert st["converged"] == 1 and st["objective"] == 0
    assert oracle.mirkin(out, p) == 0


@pytest.mark.parametrize("k", [1, 3])
def test_s2_init_at_the_common_partition(k):
    r = rng(600 + k)
    rp, col = _connected_blocks(r, 4, 10)
    p = np.repeat(np.arange(4), 10).astype(np.int32)
    out, st, _ = oracle.consensus(rp, col, np.stack([p] * k), init=p)
    assert (st["passes"], st["moves"], st["objective"], st["converged"]) == (1, 0, 0, 1)
    assert (out == p).all()


def test_s3_no_edges():
    r = rng(700)
    n, k = 30, 4
    labels = random_labels(r, k, n, 5)
    rp = np.zeros(n + 1, np.int64)
    col = np.zeros(0, np.int32)
    init = r.integers(0, n, size=n).astype(np.int32)
    out, st, _ = oracle.consensus(rp, col, labels, init=init)
    assert (out == init).all() and st["passes"] == 1 and st["candidate_evals"] == 0


def test_empty_input():
    out, st, _ = oracle.consensus(np.zeros(1, np.int64), np.zeros(0, np.int32),
                                  np.zeros((3, 0), np.int32))
    assert out.size == 0 and st["passes"] == 1 and st["converged"] == 1


# ------------------------------------------------------------ invariants ----
@pytest.mark.parametrize("seed", range(6))
def test_invariants_on_random_instances(seed):
    r = rng(800 + seed)
    n = int(r.integers(20, 160))
    init_kind = ["p0", "singleton", "random"][seed % 3]
    inst = synth.random_instance(n, int(r.integers(1, 8)), avg_deg=5.0, n_labels=6,
                                 seed=seed, init=init_kind, self_loops=4, dup_arcs=4)
    out, st, tr = oracle.consensus(inst.row_ptr, inst.col, inst.labels, init=inst.init,
                                   trace=True)
    assert st["converged"] == 1
    assert st["objective"] == bf.objective_pairs(out, inst.labels)
    assert st["objective_init"] == bf.objective_pairs(inst.init, inst.labels)
    # output clusters are a subset of the initial ones
    assert set(out.tolist()) <= set(inst.init.tolist())
    # the objective strictly drops on every pass that moves anything
    prev = st["objective_init"]
    for acc, com, fb, o in tr[:-1]:
        assert acc > 0 and 0 < com <= acc
        assert o < prev
        prev = o
    assert tr[-1][0] == 0
    assert st["moves"] == int(tr[:, 1].sum())
    # I6: no neighbour-restricted improving move remains
    for v in range(n):
        for x in bf.neighbour_clusters(inst.row_ptr, inst.col, out, v):
            assert bf.gain_member_sum(out, inst.labels, v, x) >= 0
    # resuming from the output does nothing
    out2, st2, _ = oracle.consensus(inst.row_ptr, inst.col, inst.labels, init=out)
    assert (out2 == out).all() and st2["passes"] == 1 and st2["moves"] == 0


def test_candidate_evals_bounded_by_cut_arcs():
    inst = synth.sbm_small()
    best, dbest, ncand = oracle.score(inst.row_ptr, inst.col, inst.labels, inst.init)
    src = np.repeat(np.arange(inst.n), np.diff(inst.row_ptr))
    cut = np.bincount(src[inst.init[src] != inst.init[inst.col]], minlength=inst.n)
    assert (ncand <= cut).all()
    _, st, tr = oracle.consensus(inst.row_ptr, inst.col, inst.labels, inst.init, trace=True)
    assert st["candidate_evals"] >= int(ncand.sum())


def test_max_rounds_stops_early():
    inst = synth.sbm_small()
    out, st, tr = oracle.consensus(inst.row_ptr, inst.col, inst.labels, inst.init,
                                   max_rounds=1, trace=True)
    assert st["passes"] == 1 and st["converged"] == 0 and st["moves"] == tr[0][1] > 0


def test_quality_on_planted_partition():
    inst = synth.sbm_small()
    out, st, _ = oracle.consensus(inst.row_ptr, inst.col, inst.labels, inst.init)
    mean_input = np.mean([oracle.mirkin(l, inst.truth) for l in inst.labels])
    assert oracle.mirkin(out, inst.truth) < mean_input


def test_canonicalize():
    a = np.array([5, 5, 2, 4, 2, 0], np.int32)  # cluster ids lie in [0, n)
    out, cl = oracle.canonicalize(a)
    assert out.tolist() == [0, 0, 1, 2, 1, 3] and cl == 4


# ------------------------------------------------------------ error paths ----
def test_errors():
    inst = synth.random_instance(10, 2, 3.0, 3, seed=1)
    bad = inst.labels.copy()
    bad[1, 3] = -1
    with pytest.raises(oracle.OracleError) as e:
        oracle.consensus(inst.row_ptr, inst.col, bad, inst.init)
    assert e.value.code == oracle.EINVAL
    with pytest.raises(oracle.OracleError) as e:
        oracle.consensus(inst.row_ptr, inst.col, inst.labels, np.full(10, 10, np.int32))
    assert e.value.code == oracle.EINVAL
    rp = inst.row_ptr.copy()
    rp[5] = rp[6] + 1
    with pytest.raises(oracle.OracleError) as e:
        oracle.consensus(rp, inst.col, inst.labels, inst.init)
    assert e.value.code == oracle.EGRAPH
    col = inst.col.copy()
    if col.size:
        col[0] = 10
        with pytest.raises(oracle.OracleError) as e:
            oracle.consensus(inst.row_ptr, col, inst.labels, inst.init)
        assert e.value.code == oracle.EGRAPH
