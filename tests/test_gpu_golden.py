"""The workloads at the sizes they run at, against the oracle's stored results.

The oracle cannot finish the largest workloads within a test, so its results
were computed once on the CPU by ``tests/golden/make_goldens.py`` (which calls
only the generators and the oracle) and stored with the digest of each
instance.  Each test regenerates the instance on this machine, checks that the
digest matches (the generators are exact and device independent), solves it
through the C-ABI and compares every output bit for bit: the sha256 of the
cluster ids, every statistic and, where stored, the per-pass trace.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def load(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} has not been written by tests/golden/make_goldens.py")
    with open(path) as f:
        return json.load(f)


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, "<i4").tobytes()).hexdigest()


@pytest.fixture(scope="module")
def mcc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2408_11331_amd as m
    m.lib()
    return m


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check_solve(mcc, inst, rec, flags=0):
    import torch
    assert inst.digest() == rec["digest"], "regenerated instance differs from the stored one"
    init = dev(inst.init) if rec["init"] == "p0" else None
    out, st, tr = mcc.consensus(dev(inst.row_ptr), dev(inst.col), dev(inst.labels), init,
                                flags=flags, trace=True)
    torch.cuda.synchronize()
    assert sha(out.cpu().numpy()) == rec["out_sha256"], "cluster ids differ from the oracle's"
    for key, val in rec["stats"].items():
        assert st[key] == val, (key, st[key], val)
    if "trace" in rec:
        assert [list(r) for r in tr] == rec["trace"]
    return st


def solves(name):
    g = load(f"{name}.json")
    return {r["init"]: r for r in g["solves"]}


def test_sbm_small_full(mcc):
    announce("golden sbm_small n=1000 k=10, p0 and singleton")
    inst = synth.sbm_small()
    for init, rec in solves("sbm_small").items():
        check_solve(mcc, inst, rec)
        check_solve(mcc, inst, rec, flags=mcc.MCC_F_SYMMETRIC)


def test_lfr_full(mcc):
    announce("golden lfr n=100000 k=32, p0 and singleton")
    inst = synth.lfr()
    for init, rec in solves("lfr").items():
        check_solve(mcc, inst, rec)
        check_solve(mcc, inst, rec, flags=mcc.MCC_F_SYMMETRIC)


@pytest.fixture(scope="module")
def gmm(mcc):
    load("gmm_knn.json")
    announce("generating gmm_knn n=2000000 k=50 on the GPU")
    return synth.gmm_knn(device="cuda", chunk=4096)


def test_gmm_knn_full_p0(mcc, gmm):
    announce("golden gmm_knn n=2000000 k=50 p0: plain, symmetric (the benchmark's flags)")
    rec = solves("gmm_knn")["p0"]
    check_solve(mcc, gmm, rec)
    check_solve(mcc, gmm, rec, flags=mcc.MCC_F_SYMMETRIC)


def test_gmm_knn_full_singleton(mcc, gmm):
    announce("golden gmm_knn n=2000000 k=50 singleton start (hashed tables, both layouts)")
    rec = solves("gmm_knn")["singleton"]
    st = check_solve(mcc, gmm, rec, flags=mcc.MCC_F_SYMMETRIC)
    assert st["tables"] in (2, 3)
    other = mcc.MCC_F_HASH_KEYS if st["tables"] == 3 else mcc.MCC_F_HASH_ROWS
    st2 = check_solve(mcc, gmm, rec, flags=mcc.MCC_F_SYMMETRIC | other)
    assert st2["tables"] in (2, 3)


def _batch_one(spec):
    return synth.sbm_batch_instance(spec)


def test_sbm_batch_full(mcc):
    """Every one of the 4096 instances of the batched workload, solved in the
    persistent launch, against its stored oracle result."""
    import multiprocessing as mp

    import torch
    g = load("sbm_batch.json")
    cols = g["columns"]
    specs = synth.sbm_batch_specs()
    assert len(specs) == g["count"]
    announce(f"golden sbm_batch: generating {len(specs)} instances")
    with mp.get_context("fork").Pool(16) as pool:
        insts = pool.map(_batch_one, specs, chunksize=16)
    announce("golden sbm_batch: one persistent launch")
    pb = mcc.pack_batch(insts)
    info = mcc.consensus_batch_packed(pb)
    torch.cuda.synchronize()
    assert info["rc"] == 0
    outs = pb.out.cpu().numpy()
    bad = []
    for row, inst in zip(g["rows"], insts):
        rec = dict(zip(cols, row))
        j = rec["index"]
        assert inst.digest()[:16] == rec["digest16"], f"instance {j} regenerated differently"
        assert pb.status[j] == 0
        o = int(pb.v_off[j])
        got = sha(outs[o:o + inst.n])[:16]
        st = pb.stats[j].as_dict()
        if got != rec["out_sha16"] or any(st[key] != rec[key] for key in cols[3:]):
            bad.append(j)
    assert not bad, f"{len(bad)} instances differ from the oracle, first {bad[:10]}"
