"""Batched persistent solver: each instance's output equals the
single-instance path (and the oracle) bit for bit."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
KEYS = ("passes", "converged", "fallback_rounds", "clusters", "moves", "candidate_evals",
        "objective_init", "objective")


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


def to_problem(inst, init="inst"):
    ini = inst.init if isinstance(init, str) else init
    return {"row_ptr": dev(inst.row_ptr), "col": dev(inst.col), "labels": dev(inst.labels),
            "init": None if ini is None else dev(ini)}


def instances():
    out = []
    specs = synth.sbm_batch_specs(count=24, n_range=(200, 3000), k_range=(2, 40))
    for sp in specs:
        out.append((synth.sbm_batch_instance(sp), "inst"))
    for seed in range(12):
        n = [1, 2, 50, 300, 700, 1500][seed % 6]
        init = ["p0", "singleton", "random"][seed % 3]
        inst = synth.random_instance(n, 1 + seed * 3, avg_deg=[2.0, 6.0, 30.0][seed % 3],
                                     n_labels=[2, 5, 40][seed % 3], seed=100 + seed, init=init,
                                     self_loops=seed % 4, dup_arcs=seed % 3)
        out.append((inst, None if init == "singleton" else "inst"))
    return out


@pytest.mark.parametrize("lanes", [0, 4, 8, 32, 64])
def test_batch_equals_single(mcc, lanes):
    import torch
    print(f"[gpu-case] batch lanes={lanes}", flush=True)
    items = instances()
    probs = [to_problem(i, init) for i, init in items]
    outs, stats, codes, info = mcc.consensus_batch(probs, lanes=lanes)
    torch.cuda.synchronize()
    assert all(c == 0 for c in codes)
    # singleton-initialised instances with large tables go to the
    # single-instance path; the rest stay in the persistent kernel
    assert info["solved_in_batch"] >= len(items) - 4
    for (inst, init), out, st, p in zip(items, outs, stats, probs):
        o2, st2 = mcc.consensus(p["row_ptr"], p["col"], p["labels"], p["init"])
        assert np.array_equal(out.cpu().numpy(), o2.cpu().numpy())
        for key in KEYS:
            assert st[key] == st2[key], key
    # and the oracle on every one
    for (inst, init), out, st in zip(items, outs, stats):
        eo, est, _ = oracle.consensus(inst.row_ptr, inst.col, inst.labels,
                                      None if init is None else inst.init)
        assert np.array_equal(out.cpu().numpy(), eo)
        for key in KEYS:
            assert st[key] == est[key], key


def test_batch_fallback_and_errors(mcc):
    import torch
    print("[gpu-case] batch fallback/errors", flush=True)
    small = synth.random_instance(100, 3, 5.0, 4, seed=7)
    huge = synth.random_instance(120, 3, 5.0, 4, seed=8)
    huge.labels[1] = huge.labels[1] * 1_000_003 + 5  # label values far above n: not batchable
    bad = synth.random_instance(90, 2, 5.0, 4, seed=9)
    bad.labels[0, 3] = -1
    many_k = synth.random_instance(40, 300, 4.0, 3, seed=10)  # k > 256
    items = [small, huge, bad, many_k]
    probs = [to_problem(i) for i in items]
    outs, stats, codes, info = mcc.consensus_batch(probs, max_rounds=50)
    torch.cuda.synchronize()
    assert codes == [0, 0, mcc.MCC_EINVAL, 0]
    assert info["solved_in_batch"] == 1 and info["rc"] == mcc.MCC_EINVAL
    for j in (0, 1, 3):
        inst = items[j]
        eo, est, _ = oracle.consensus(inst.row_ptr, inst.col, inst.labels, inst.init,
                                      max_rounds=50)
        assert np.array_equal(outs[j].cpu().numpy(), eo)
        for key in KEYS:
            assert stats[j][key] == est[key], (j, key)


def test_batch_max_rounds_and_literal(mcc):
    import torch
    print("[gpu-case] batch max_rounds/literal", flush=True)
    items = [synth.random_instance(400, 5, 6.0, 5, seed=20 + j, init="singleton") for j in range(5)]
    probs = [to_problem(i, None) for i in items]
    for mr in (1, 2):
        outs, stats, codes, _ = mcc.consensus_batch(probs, max_rounds=mr, flags=mcc.MCC_F_LITERAL)
        torch.cuda.synchronize()
        for inst, out, st in zip(items, outs, stats):
            eo, est, _ = oracle.consensus(inst.row_ptr, inst.col, inst.labels, None,
                                          max_rounds=mr, literal=True)
            assert np.array_equal(out.cpu().numpy(), eo)
            assert st["passes"] == est["passes"] and st["objective"] == est["objective"]


def test_autotune_then_tuned_batch(mcc, tmp_path):
    # the tuner's table (lanes per size bucket, table size, workgroups per
    # compute unit) changes where and how fast instances run, never results
    import torch
    print("[gpu-case] batch autotune", flush=True)
    items = instances()
    probs = [to_problem(i, init) for i, init in items]
    path = str(tmp_path / "tune.txt")
    table = mcc.batch_tune(probs, tune_cache_path=path)
    d = table.as_dict()
    assert 1 <= d["wg_per_cu"] <= 8 and d["buckets"]
    for b in d["buckets"]:
        assert b["lanes"] in mcc.TUNE_LANES
        if b["instances"]:
            ms = b["ms"]
            assert all(v >= 0 for v in ms.values()) and ms[b["lanes"]] == min(ms.values())
    back = mcc.tune_load(path).as_dict()
    assert back["wg_per_cu"] == d["wg_per_cu"]
    assert [(b["n_log2"], b["k_class"], b["lanes"], b["cells"]) for b in back["buckets"]] == \
        [(b["n_log2"], b["k_class"], b["lanes"], b["cells"]) for b in d["buckets"]]
    ref = [mcc.consensus(p["row_ptr"], p["col"], p["labels"], p["init"]) for p in probs]
    by_bucket = {(b["n_log2"], b["k_class"]): b["lanes"] for b in d["buckets"]}
    for kw in ({"tune": table}, {"tune_cache_path": path}):
        outs, stats, codes, info = mcc.consensus_batch(probs, **kw)
        torch.cuda.synchronize()
        assert all(c == 0 for c in codes)
        for (inst, _), out, st, (o2, st2) in zip(items, outs, stats, ref):
            assert np.array_equal(out.cpu().numpy(), o2.cpu().numpy())
            for key in KEYS:
                assert st[key] == st2[key], key
            n, k = inst.labels.shape[1], inst.labels.shape[0]
            if n > 0 and k <= 256 and st["lanes_used"]:
                kc = 0 if k <= 8 else 1 if k <= 16 else 2 if k <= 32 else 3 if k <= 64 else 4
                assert st["lanes_used"] == by_bucket[(max(n, 1).bit_length() - 1, kc)]


def test_packed_batch_equals_batch(mcc):
    # the same instances concatenated on the device with per-instance offsets
    import types
    import torch
    print("[gpu-case] packed batch", flush=True)
    items = instances()
    hosts = [types.SimpleNamespace(row_ptr=i.row_ptr, col=i.col, labels=i.labels,
                                   init=None if init is None else i.init) for i, init in items]
    pb = mcc.pack_batch(hosts)
    info = mcc.consensus_batch_packed(pb)
    torch.cuda.synchronize()
    assert info["rc"] == 0 and all(pb.status[j] == 0 for j in range(pb.count))
    probs = [to_problem(i, init) for i, init in items]
    outs, stats, codes, _ = mcc.consensus_batch(probs)
    torch.cuda.synchronize()
    for j in range(pb.count):
        assert np.array_equal(pb.output(j).cpu().numpy(), outs[j].cpu().numpy())
        got = pb.stats[j].as_dict()
        for key in KEYS:
            assert got[key] == stats[j][key], (j, key)


def test_batch_counts_widths(mcc):
    """Instances below 2^15 vertices keep int16 counts, larger ones int32:
    both against the oracle in one launch."""
    import torch
    print("[gpu-case] batch int16/int32 counts", flush=True)
    items = [synth.lfr(n=40000, k=6), synth.random_instance(700, 9, 8.0, 6, seed=31),
             synth.lfr(n=32767, k=5), synth.lfr(n=32768, k=5)]
    probs = [to_problem(i) for i in items]
    outs, stats, codes, info = mcc.consensus_batch(probs)
    torch.cuda.synchronize()
    assert all(c == 0 for c in codes) and info["solved_in_batch"] == len(items)
    for inst, out, st in zip(items, outs, stats):
        eo, est, _ = oracle.consensus(inst.row_ptr, inst.col, inst.labels, inst.init)
        assert np.array_equal(out.cpu().numpy(), eo)
        for key in KEYS:
            assert st[key] == est[key], key
