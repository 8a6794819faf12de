"""Round-rule ablations of the oracle (Methods, "Parallel algorithm"): one
best move per pass, direction alternation and the unchecked batch, next to
the pinned rule.

Pins: hand-worked traces on the complete graph K6 (the same example as the
pinned rule's golden trace), brute force on tiny instances written from the
pair-counting objective (no contingency counts, no closed-form gain), and
the local-optimum property at convergence.

Readings (the paper names the alternatives without defining them):
one best move = score every vertex against the current partition, apply only
the smallest (gain, vertex) accepted move, repeat; direction alternation =
even passes allow moves only to larger cluster ids, odd passes only to
smaller ones, the batch applied unchecked, stop after one empty pass in each
direction; unchecked = the pinned rule without its validation check."""
import json
import os

import numpy as np
import pytest

import bruteforce as bf
import oracle
import synth
from synth import graph as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def k6():
    g = json.load(open(os.path.join(GOLDEN, "s5_k6_trace.json")))
    u, v = np.triu_indices(g["n"], 1)
    rp, col = G.csr_from_edges(g["n"], u, v)
    return rp, col, np.array(g["labels"], np.int32), np.array(g["init"], np.int32)


# ------------------------------------------------------- hand-worked K6 -----
# K6, init {0,1,2}{3,4,5}, k = 3 partitions that each put all six together;
# O = 54.  Every partition is one cluster, so S_y(v) = 3 |y| and the gain of
# v from c to y is 2 (3|c| - 3|y|) + 3 (|y| - |c| - 1) = 3 (|c| - |y| - 1).
def test_k6_one_best_move():
    # pass 0: all six gain 3(3-3-1) = -3; the smallest vertex, 0, moves to 1:
    #   O = 54 + 2(-3) = 48
    # pass 1: v1, v2 gain 3(2-4-1) = -9, cluster 1's members 3(4-2-1) = +3;
    #   v1 moves: O = 48 - 18 = 30
    # pass 2: v2 gains 3(1-5-1) = -15, the others 3(5-1-1) = +9; O = 0
    # pass 3: one cluster, no candidates
    rp, col, lab, ini = k6()
    out, st, tr = oracle.consensus_rule(rp, col, lab, ini, rule="one_best", trace=True)
    assert out.tolist() == [1] * 6
    assert (st["passes"], st["moves"], st["converged"], st["objective"]) == (4, 3, 1, 0)
    assert st["candidate_evals"] == 6 + 6 + 6 + 0
    assert tr.tolist() == [[6, 1, 0, 48], [2, 1, 0, 30], [1, 1, 0, 0], [0, 0, 0, 0]]


def test_k6_direction_alternation():
    # pass 0 (up): v0, v1, v2 may move 0 -> 1 (gain -3 each); 3, 4, 5 may not
    #   move down; applied together: one cluster, O = 0
    # passes 1 (down) and 2 (up): nothing to move -> converged
    rp, col, lab, ini = k6()
    out, st, tr = oracle.consensus_rule(rp, col, lab, ini, rule="alternate", trace=True)
    assert out.tolist() == [1] * 6
    assert (st["passes"], st["moves"], st["converged"], st["objective"]) == (3, 3, 1, 0)
    assert st["candidate_evals"] == 3
    assert tr.tolist() == [[3, 3, 0, 0], [0, 0, 0, 0], [0, 0, 0, 0]]


def test_k6_unchecked_batch_oscillates():
    # all six accept; the two clusters swap members every pass and O stays 54:
    # the reason for the pinned rule's validation check
    rp, col, lab, ini = k6()
    out, st, tr = oracle.consensus_rule(rp, col, lab, ini, rule="unchecked", max_rounds=9,
                                        trace=True)
    assert st["converged"] == 0 and st["passes"] == 9 and st["moves"] == 54
    assert st["objective"] == 54 and out.tolist() == [1, 1, 1, 0, 0, 0]
    assert all(r == [6, 6, 0, 54] for r in tr.tolist())


def test_pinned_rule_is_the_consensus():
    inst = synth.random_instance(90, 4, avg_deg=5.0, n_labels=6, seed=3, init="random")
    a = oracle.consensus_rule(inst.row_ptr, inst.col, inst.labels, inst.init, rule="pinned",
                              trace=True)
    b = oracle.consensus(inst.row_ptr, inst.col, inst.labels, inst.init, trace=True)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1] and np.array_equal(a[2], b[2])


def test_unknown_rule_rejected():
    rp, col, lab, ini = k6()
    L = oracle.lib()
    out = np.zeros(6, np.int32)
    rp = np.ascontiguousarray(rp, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    rc = L.mccref_consensus_rule(rp.ctypes.data, col.ctypes.data, 6, lab.ctypes.data, 3,
                                 ini.ctypes.data, out.ctypes.data, None, None, 9)
    assert rc == oracle.EINVAL


# ------------------------------------------------ brute force, tiny cases ---
def neighbour_clusters(rp, col, C, v):
    return sorted({int(C[u]) for u in col[rp[v]:rp[v + 1]] if u != v and C[u] != C[v]})


def best_moves_bf(rp, col, labels, C, O, direction=0):
    """Per vertex, the smallest (objective change, cluster) over its allowed
    neighbour clusters, by recomputing the objective from pair counts."""
    out = {}
    for v in range(len(C)):
        for x in neighbour_clusters(rp, col, C, v):
            if (direction > 0 and x < C[v]) or (direction < 0 and x > C[v]):
                continue
            C2 = C.copy()
            C2[v] = x
            d = bf.objective_pairs(C2, labels) - O
            if v not in out or (d, x) < out[v]:
                out[v] = (d, x)
    return out


def one_best_bf(rp, col, labels, C):
    C = np.array(C, np.int32)
    O = bf.objective_pairs(C, labels)
    trace = []
    while True:
        moves = best_moves_bf(rp, col, labels, C, O)
        acc = sorted((d, v, x) for v, (d, x) in moves.items() if d < 0)
        if not acc:
            trace.append(O)
            return C, trace
        d, v, x = acc[0]
        C[v] = x
        O += d
        trace.append(O)


def alternate_bf(rp, col, labels, C, cap=200):
    C = np.array(C, np.int32)
    O = bf.objective_pairs(C, labels)
    trace, empty = [], 0
    for p in range(cap):
        moves = best_moves_bf(rp, col, labels, C, O, direction=1 if p % 2 == 0 else -1)
        acc = {v: x for v, (d, x) in moves.items() if d < 0}
        for v, x in acc.items():
            C[v] = x
        O = bf.objective_pairs(C, labels)
        trace.append(O)
        empty = 0 if acc else empty + 1
        if empty == 2:
            return C, trace, True
    return C, trace, False


TINY = [(n, k, deg, seed) for seed, (n, k, deg) in enumerate(
    [(5, 1, 2.0), (6, 2, 3.0), (7, 3, 2.5), (8, 2, 4.0), (9, 3, 3.0), (10, 2, 2.0),
     (10, 3, 5.0), (8, 4, 7.0)])]


@pytest.mark.parametrize("n,k,deg,seed", TINY)
@pytest.mark.parametrize("init", ["singleton", "random"])
def test_one_best_matches_brute_force(n, k, deg, seed, init):
    inst = synth.random_instance(n, k, avg_deg=deg, n_labels=3, seed=500 + seed, init=init)
    ini = np.arange(n, dtype=np.int32) if init == "singleton" else inst.init
    C, trace = one_best_bf(inst.row_ptr, inst.col, inst.labels, ini)
    out, st, tr = oracle.consensus_rule(inst.row_ptr, inst.col, inst.labels, ini,
                                        rule="one_best", trace=True)
    assert out.tolist() == C.tolist()
    assert tr[:, 3].tolist() == trace
    assert st["passes"] == len(trace) and st["moves"] == len(trace) - 1


@pytest.mark.parametrize("n,k,deg,seed", TINY)
@pytest.mark.parametrize("init", ["singleton", "random"])
def test_alternate_matches_brute_force(n, k, deg, seed, init):
    inst = synth.random_instance(n, k, avg_deg=deg, n_labels=3, seed=600 + seed, init=init)
    ini = np.arange(n, dtype=np.int32) if init == "singleton" else inst.init
    C, trace, conv = alternate_bf(inst.row_ptr, inst.col, inst.labels, ini)
    out, st, tr = oracle.consensus_rule(inst.row_ptr, inst.col, inst.labels, ini,
                                        rule="alternate", max_rounds=200, trace=True)
    assert out.tolist() == C.tolist()
    assert tr[:, 3].tolist() == trace
    assert st["converged"] == int(conv)


# ----------------------------------------------- properties at any size ----
@pytest.mark.parametrize("rule", ["pinned", "one_best", "alternate"])
@pytest.mark.parametrize("seed", range(6))
def test_converged_rules_leave_no_improving_move(rule, seed):
    n = [40, 75, 120][seed % 3]
    inst = synth.random_instance(n, 3 + seed % 3, avg_deg=4.0 + seed, n_labels=5, seed=700 + seed,
                                 init=["p0", "singleton"][seed % 2])
    ini = None if seed % 2 else inst.init
    out, st, tr = oracle.consensus_rule(inst.row_ptr, inst.col, inst.labels, ini, rule=rule,
                                        max_rounds=5000, trace=True)
    assert st["objective"] == oracle.objective(out, inst.labels)
    if rule != "alternate":
        # every committed pass lowers the objective
        objs = [st["objective_init"]] + tr[:, 3].tolist()
        assert all(b < a for a, b in zip(objs[:-2], objs[1:-1]))
    assert st["converged"] == 1
    best, dbest, ncand = oracle.score(inst.row_ptr, inst.col, inst.labels, out)
    assert not np.any((ncand > 0) & (dbest < 0))


def test_ablation_study_script_runs():
    # the study script on one small instance: a row per rule and init, and
    # the summary table
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-m", "oracle.ablation", "--count", "1", "--n-max", "120"],
                       cwd=root, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    rows = [l for l in r.stdout.splitlines() if l.startswith("| 0 |")]
    assert len(rows) == 2 * 5
    assert "| P_0 | one_best |" in r.stdout and "| singletons | pinned |" in r.stdout
