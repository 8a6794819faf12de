"""The C-ABI library loads and exports every entry point include/mcc.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_2408_11331_amd as mcc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if f.endswith(".h"):
            txt = open(os.path.join(inc, f)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?\w[\w\s\*]*?\b(mcc_\w+)\s*\(", txt, re.M))
    return names


def test_header_matches_binding():
    assert declared() == set(mcc.EXPORTS)


def test_library_exports_every_symbol():
    if not os.path.exists(mcc.LIB_PATH):
        pytest.skip("libmcc.so not built")
    L = ctypes.CDLL(mcc.LIB_PATH)
    for name in declared():
        assert hasattr(L, name), name


def test_strerror_is_static_text():
    if not os.path.exists(mcc.LIB_PATH):
        pytest.skip("libmcc.so not built")
    L = mcc.lib()
    for code in (0, -1, -2, -3, -5, 7):
        assert isinstance(L.mcc_strerror(code), bytes)


# ------------------------------------------- tune table files (host only) ---
def _table():
    t = mcc.TuneTable()
    t.count, t.wg_per_cu = 2, 4
    for j, (nb, kc, lanes, cells) in enumerate([(9, 1, 8, 4096), (14, 3, 32, 1 << 20)]):
        e = t.entry[j]
        e.n_log2, e.k_class, e.lanes, e.instances, e.cells = nb, kc, lanes, 3 + j, cells
        for c in range(mcc.MCC_TUNE_LANES):
            e.ms[c] = 0.5 * (c + 1) + j
    return t


def test_tune_table_round_trip(tmp_path):
    if not os.path.exists(mcc.LIB_PATH):
        pytest.skip("libmcc.so not built")
    path = str(tmp_path / "tune.txt")
    mcc.tune_save(_table(), path)
    back = mcc.tune_load(path)
    assert back.as_dict() == _table().as_dict()


@pytest.mark.parametrize("text", [
    "",
    "mcc-tune 2\nwg_per_cu 2\nbuckets 0\n",                       # unknown version
    "mcc-tune 1\nwg_per_cu 9\nbuckets 0\n",                       # workgroups out of range
    "mcc-tune 1\nwg_per_cu 2\nbuckets 1\n9 1 12 1 10 1 1 1 1 1\n",  # lanes not offered
    "mcc-tune 1\nwg_per_cu 2\nbuckets 1\n9 7 8 1 10 1 1 1 1 1\n",   # k class out of range
    "mcc-tune 1\nwg_per_cu 2\nbuckets 2\n9 1 8 1 10 1 1 1 1 1\n",   # truncated
])
def test_tune_table_rejects_malformed(tmp_path, text):
    if not os.path.exists(mcc.LIB_PATH):
        pytest.skip("libmcc.so not built")
    path = tmp_path / "bad.txt"
    path.write_text(text)
    with pytest.raises(mcc.MccError) as e:
        mcc.tune_load(str(path))
    assert e.value.code == mcc.MCC_EINVAL
    with pytest.raises(mcc.MccError):
        mcc.tune_load(str(tmp_path / "missing.txt"))


# ------------------------------------------- grouping step (host only) ------
@pytest.mark.parametrize("seed", range(8))
def test_group_from_distances_matches_oracle(seed):
    if not os.path.exists(mcc.LIB_PATH):
        pytest.skip("libmcc.so not built")
    import numpy as np
    import oracle
    rng = np.random.Generator(np.random.PCG64(seed))
    k = int(rng.integers(1, 30))
    d = np.triu(rng.integers(0, [5, 50, 1000][seed % 3], size=(k, k)), 1)
    d = d + d.T
    for lam in (-1, 0, int(rng.integers(0, 60))):
        g, ng, used = mcc.group_from_distances(d, lam)
        want = oracle.elbow_lambda(d) if lam < 0 else lam
        assert used == want
        og, ong = oracle.group(d, want)
        assert ng == ong and np.array_equal(g, og)


def test_group_from_distances_rejects_bad_matrix():
    if not os.path.exists(mcc.LIB_PATH):
        pytest.skip("libmcc.so not built")
    import numpy as np
    with pytest.raises(mcc.MccError):
        mcc.group_from_distances(np.array([[0, 1], [2, 0]]), 3)
    with pytest.raises(mcc.MccError):
        mcc.group_from_distances(np.array([[0, -1], [-1, 0]]), 3)


def test_bench_refuses_several_gpus():
    # the bench measures one GPU; asking for more exits with a message and
    # status 2 before touching a device
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "4"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout


def test_bench_traffic_keyed_to_scorer_source():
    # the committed HBM counters apply while the scoring kernels' source is
    # the one they were taken on
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    sha = b.scorer_source_sha()
    assert len(sha) == 64
    assert b.traffic_from_profile("0" * 64) is None
    t = b.traffic_from_profile(sha)
    assert t is None or t > 0


def test_workspace_bound_properties():
    # host-only sizing: grows with the instance, counts the hashed table when
    # hashing is forced, and the row table when it is forced
    if not os.path.exists(mcc.LIB_PATH):
        pytest.skip("libmcc.so not built")
    wb = mcc.workspace_bound
    base = wb(100_000, 2_000_000, 16, 200, 500, 0)
    assert base > 0
    assert wb(200_000, 4_000_000, 16, 200, 500, 0) >= base
    assert wb(100_000, 2_000_000, 32, 200, 500, 0) >= base
    forced = wb(100_000, 2_000_000, 16, 200, 500, mcc.MCC_F_HASH_TABLES)
    assert forced >= base
    # the key table alone is 16 bytes a slot, 4 n k slots or more
    assert forced - base >= 16 * 4 * 100_000 * 16 // 2
    rows = wb(100_000, 2_000_000, 16, 200, 500, mcc.MCC_F_HASH_TABLES | mcc.MCC_F_HASH_ROWS)
    assert rows > forced
    # singletons choose hashing by themselves
    single = wb(100_000, 2_000_000, 16, 200, 0, 0)
    assert single >= 16 * 4 * 100_000 * 16
    with pytest.raises(Exception):
        wb(-1, 0, 1, 0, 0, 0)
