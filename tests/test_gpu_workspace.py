"""The host-side workspace bound covers what a solve takes, in every table
layout (the serving admission counts the bound of each call it starts)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def mcc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2408_11331_amd as m
    m.lib()
    return m


def solve_within_bound(mcc, inst, init, flags, want_tables):
    import torch
    D = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    clusters = 0 if init is None else int(np.unique(init).size)
    bound = mcc.workspace_bound(inst.n, int(inst.col.size), int(inst.labels.shape[0]),
                                int(inst.labels.max()), clusters, flags)
    mcc.release_workspace()  # fresh chunks: the call's own sizes
    torch.cuda.synchronize()
    out, st = mcc.consensus(D(inst.row_ptr), D(inst.col), D(inst.labels),
                            None if init is None else D(init), flags=flags)
    assert st["tables"] in want_tables, st["tables"]
    assert 0 < st["workspace_bytes"] <= bound, (st["workspace_bytes"], bound)
    return st


def test_bound_covers_every_layout(mcc):
    announce("workspace bound: dense, hashed keys, hashed rows")
    lfr = synth.lfr(n=20000, k=8)
    sym = mcc.MCC_F_SYMMETRIC
    # dense (first partition), interleaved or blocked
    solve_within_bound(mcc, lfr, lfr.init, sym, (0, 1))
    # singletons: hashed, the layout the library picks, then each one forced
    solve_within_bound(mcc, lfr, None, sym, (2, 3))
    solve_within_bound(mcc, lfr, None, sym | mcc.MCC_F_HASH_KEYS, (2,))
    solve_within_bound(mcc, lfr, None, sym | mcc.MCC_F_HASH_ROWS, (3,))
    # hashed tables forced where dense ones fit, both layouts, arc cache on
    small = synth.random_instance(3000, 20, 6.0, 40, seed=4, init="random")
    for extra in (mcc.MCC_F_HASH_KEYS, mcc.MCC_F_HASH_ROWS):
        solve_within_bound(mcc, small, small.init,
                           mcc.MCC_F_HASH_TABLES | mcc.MCC_F_ARC_CACHE | extra, (2, 3))
    mcc.release_workspace()
