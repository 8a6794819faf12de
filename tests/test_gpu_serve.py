"""Serving: every result of a mixed, overlapping request stream equals the
request solved alone."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def pool():
    from paper_2408_11331_amd.serve import Request
    out = []
    for sp in synth.sbm_batch_specs(count=10, n_range=(200, 2500), k_range=(3, 20), w=7):
        i = synth.sbm_batch_instance(sp, w=7)
        out.append(Request(i.row_ptr, i.col, i.labels, i.init))
    for seed in range(3):  # above the large-request threshold used below
        i = synth.random_instance(4000 + 500 * seed, 6, 5.0, 6, seed=40 + seed)
        out.append(Request(i.row_ptr, i.col, i.labels, i.init))
    i = synth.random_instance(600, 4, 4.0, 5, seed=50, init="singleton")
    out.append(Request(i.row_ptr, i.col, i.labels, None))
    return out


def test_served_equals_alone():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2408_11331_amd as mcc
    from paper_2408_11331_amd.serve import run_served
    print("[gpu-case] serve mixed stream", flush=True)
    P = pool()
    reqs, summ = run_served(P, rate=400.0, count=60, seed=3, large_n=3000, max_batch=16,
                            budget_bytes=64 << 20)
    assert summ["solves"] == 60 and summ["batches"] >= 2
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    alone = {}
    for r in reqs:
        assert r.error is None, r.error
        if r.rid not in alone:
            s = P[r.rid]
            out, st = mcc.consensus(T(s.row_ptr), T(s.col), T(s.labels),
                                    None if s.init is None else T(s.init))
            alone[r.rid] = (out.cpu().numpy(), st)
        out, st = alone[r.rid]
        assert np.array_equal(r.out, out)
        for key in ("passes", "moves", "objective", "candidate_evals", "fallback_rounds"):
            assert r.stats[key] == st[key], key
