"""The seeded workload generators: deterministic, well-formed CSR, labels in
range, and symmetric graphs (the benchmark states symmetry to the library
with MCC_F_SYMMETRIC, which is exact only on symmetric graphs)."""
import numpy as np
import pytest

import synth


def csr_ok(row_ptr, col, n):
    assert row_ptr.dtype == np.int64 and col.dtype == np.int32
    assert row_ptr.shape == (n + 1,) and row_ptr[0] == 0 and row_ptr[-1] == col.size
    assert np.all(np.diff(row_ptr) >= 0)
    assert col.size == 0 or (col.min() >= 0 and col.max() < n)


def symmetric(row_ptr, col, n):
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    fwd = np.unique(src * n + col)
    rev = np.unique(col.astype(np.int64) * n + src)
    return np.array_equal(fwd, rev)


def small_instances():
    yield "sbm_small", synth.sbm_small()
    yield "lfr", synth.lfr(n=3000, k=6)
    yield "gmm_knn", synth.gmm_knn(n=4000, k=5)
    for sp in synth.sbm_batch_specs(count=3, n_range=(200, 900), k_range=(2, 6)):
        yield "sbm_batch", synth.sbm_batch_instance(sp)


@pytest.mark.parametrize("name,inst", list(small_instances()))
def test_generated_instances_well_formed_and_symmetric(name, inst):
    n, k = inst.labels.shape[1], inst.labels.shape[0]
    csr_ok(inst.row_ptr, inst.col, n)
    assert symmetric(inst.row_ptr, inst.col, n), name
    assert inst.labels.dtype == np.int32 and inst.labels.min() >= 0
    assert inst.init.shape == (n,) and inst.init.min() >= 0 and inst.init.max() < n
    assert k >= 1


def test_generators_are_deterministic():
    a = synth.lfr(n=2000, k=4)
    b = synth.lfr(n=2000, k=4)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
    assert np.array_equal(a.labels, b.labels) and np.array_equal(a.init, b.init)
    c = synth.gmm_knn(n=3000, k=3)
    d = synth.gmm_knn(n=3000, k=3)
    assert np.array_equal(c.col, d.col) and np.array_equal(c.labels, d.labels)


def test_knn_exact_on_every_path():
    """The kNN lists of integer points are exact (squared L2, ties to the
    lower index) on the compiled CPU search and on the torch path alike, so
    the 2M-point workload is the same instance on any machine.  Checked
    against brute force, including points placed to tie."""
    from synth import graph as G
    rng = np.random.Generator(np.random.PCG64(7))
    pts, _ = G.gmm_points(2500, 30, 20, 1.2, 0.8, rng)
    # exact duplicates and mirror images make equal distances
    pts[100:140] = pts[50]
    pts[200:230] = 2 * pts[7] - pts[300:330]
    a = G.knn_lists_cpu(pts, 15)
    b = G.knn_lists_torch(pts, 15, chunk=333)
    X = pts.astype(np.int64)
    for q in range(pts.shape[0]):
        d = ((X - X[q]) ** 2).sum(1)
        d[q] = np.iinfo(np.int64).max
        ref = np.lexsort((np.arange(d.size), d))[:15]
        assert np.array_equal(a[q], ref), q
    assert np.array_equal(a, b)
