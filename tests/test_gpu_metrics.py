"""Partition comparison and grouping on the GPU against the oracle.

Integers (Mirkin, split-join, cluster counts, distances, groups) are
compared exactly.  The variation of information is a double-precision sum
of x ln x terms in a different order and with a different logarithm than
the oracle's: both sides are within a few units in the last place per term,
so the tolerance is 1e-9 relative (plus 1e-12 absolute near zero)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mcc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2408_11331_amd as m
    m.lib()
    oracle.build(force=False)
    return m


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def same_comparison(g, o):
    for key in ("mirkin", "split_join_ab", "split_join_ba", "split_join", "clusters_a",
                "clusters_b"):
        assert g[key] == o[key], (key, g[key], o[key])
    assert g["rand"] == o["rand"]  # the same exact integer over the same double
    assert g["vi"] == pytest.approx(o["vi"], rel=1e-9, abs=1e-12)


CASES = [(1, 1, 1), (2, 1, 2), (5, 3, 2), (1000, 7, 40), (70_001, 300, 9),
         (200_000, 200_000, 50), (2_000_000, 2_000_000, 5000)]


@pytest.mark.parametrize("n,ma,mb", CASES)
def test_compare_against_oracle(mcc, n, ma, mb):
    # the last two have up to n clusters on one side: hashed tables
    announce(f"compare n={n} ma={ma} mb={mb}")
    r = np.random.Generator(np.random.PCG64(n + ma))
    a = (r.integers(0, ma, size=n) * 1_000_003 % (2 ** 31 - 1)).astype(np.int32)
    if ma == n:
        a = r.permutation(n).astype(np.int32)
    b = r.integers(0, mb, size=n).astype(np.int32)
    same_comparison(mcc.compare(dev(a), dev(b)), oracle.compare(a, b))
    same_comparison(mcc.compare(dev(b), dev(a)), oracle.compare(b, a))


def test_compare_deterministic_and_errors(mcc):
    announce("compare determinism/errors")
    r = np.random.Generator(np.random.PCG64(3))
    a, b = r.integers(0, 900, 300_000).astype(np.int32), r.integers(0, 77, 300_000).astype(np.int32)
    x, y = mcc.compare(dev(a), dev(b)), mcc.compare(dev(a), dev(b))
    assert x == y
    bad = b.copy()
    bad[5] = -2
    with pytest.raises(mcc.MccError) as e:
        mcc.compare(dev(a), dev(bad))
    assert e.value.code == mcc.MCC_EINVAL
    assert mcc.compare(dev(a[:0]), dev(b[:0]))["split_join"] == 0


@pytest.mark.parametrize("workload", ["sbm_small", "lfr", "random_wide"])
def test_split_join_matrix_against_oracle(mcc, workload):
    announce(f"split-join matrix {workload}")
    if workload == "sbm_small":
        labels = synth.sbm_small().labels
    elif workload == "lfr":
        labels = synth.lfr(n=30_000, k=12).labels
    else:  # label counts whose pair tables do not fit LDS, and one near-singleton partition
        r = np.random.Generator(np.random.PCG64(11))
        labels = np.stack([r.integers(0, m, 5000) for m in (2, 300, 500, 4999)]).astype(np.int32)
    d = mcc.split_join_matrix(dev(labels))
    assert np.array_equal(d, oracle.split_join_matrix(labels))


def test_group_partitions_and_grouped_consensus(mcc):
    # two families of partitions of one graph: five perturbed copies of the
    # planted partition and four of a vertex-shuffled one (split-join about
    # 240 within a family, 1700 across): the elbow threshold separates them,
    # and each group's consensus equals the oracle's consensus of that group
    announce("grouped consensus")
    a = synth.sbm_small(w=0)
    perm = np.random.Generator(np.random.PCG64(77)).permutation(a.n)
    labels = np.concatenate([a.labels[:5], a.labels[5:9][:, perm]]).astype(np.int32)
    g, ng, lam, d = mcc.group_partitions(dev(labels))
    od = oracle.split_join_matrix(labels)
    assert np.array_equal(d, od)
    assert lam == oracle.elbow_lambda(od)
    og, ong = oracle.group(od, lam)
    assert ng == ong and np.array_equal(g, og)
    assert ng >= 2 and len(set(g[:5])) == 1 and g[0] != g[5]
    gg, used, outs, stats = mcc.consensus_groups(dev(a.row_ptr), dev(a.col), dev(labels))
    assert np.array_equal(gg, g) and used == lam
    for j in range(ng):
        sub = labels[g == j]
        start, _ = oracle.canonicalize(sub[0])
        eo, est, _ = oracle.consensus(a.row_ptr, a.col, sub, start)
        assert np.array_equal(outs[j].cpu().numpy(), eo)
        assert stats[j]["objective"] == est["objective"]
