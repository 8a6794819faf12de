"""mcc_consensus_noalloc: the entry point for callers that cannot allocate
device memory.  Through the C-ABI, its results equal mcc_consensus bit for
bit on two calls in a row (the second smaller, so stale contents of the
shared scratch array would show), it allocates no device memory, and it
rejects instances beyond its scratch array with MCC_ESCRATCH."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
KEYS = ("passes", "converged", "fallback_rounds", "clusters", "moves", "candidate_evals",
        "objective_init", "objective", "boundary", "tables")


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


def both(mcc, inst, init, flags=0):
    import torch
    args = (dev(inst.row_ptr), dev(inst.col), dev(inst.labels), None if init is None else dev(init))
    out_a = torch.empty(inst.n, dtype=torch.int32, device="cuda")
    out_b = torch.full((inst.n,), -7, dtype=torch.int32, device="cuda")
    _, sa, ta = mcc.consensus(*args, flags=flags, out=out_a, trace=True)
    _, sb, tb = mcc.consensus(*args, flags=flags, out=out_b, trace=True, noalloc=True)
    torch.cuda.synchronize()
    assert np.array_equal(out_a.cpu().numpy(), out_b.cpu().numpy())
    for key in KEYS:
        assert sa[key] == sb[key], (key, sa[key], sb[key])
    assert ta == tb


def test_noalloc_equals_consensus_twice(mcc):
    print("[gpu-case] noalloc: lfr n=20000 k=12 then sbm_small, twice", flush=True)
    big = synth.lfr(n=20000, k=12)
    small = synth.sbm_small()
    for _ in range(2):
        both(mcc, big, big.init)
        both(mcc, small, small.init)
    # the singleton start (hashed tables), the symmetric candidate cache and
    # the arc cache, each after a larger call
    both(mcc, big, None, flags=mcc.MCC_F_SYMMETRIC)
    both(mcc, small, None, flags=mcc.MCC_F_HASH_TABLES)
    both(mcc, small, small.init, flags=mcc.MCC_F_ARC_CACHE | mcc.MCC_F_SYMMETRIC)


def test_noalloc_allocates_nothing(mcc):
    """No device memory is taken by a no-allocation call, where
    mcc_consensus on a fresh stream takes workspace chunks of 16 MiB or more.
    The first launches of the library's kernels on a stream's hardware queue
    let the HIP runtime back that queue's private (register spill) memory,
    16 MiB here: runtime memory, not the call's, so the measured call is the
    stream's second."""
    import torch
    print("[gpu-case] noalloc: device memory unchanged", flush=True)
    inst = synth.lfr(n=20000, k=12)
    args = (dev(inst.row_ptr), dev(inst.col), dev(inst.labels), dev(inst.init))
    out = torch.empty(inst.n, dtype=torch.int32, device="cuda")
    mcc.consensus(*args, out=out, noalloc=True)  # loads the library's kernels
    torch.cuda.synchronize()
    mcc.release_workspace()
    s1 = torch.cuda.Stream()
    mcc.consensus(*args, out=out, stream=s1, noalloc=True)  # the queue's runtime set-up
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    mcc.consensus(*args, out=out, stream=s1, noalloc=True)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free0 - free1 < (4 << 20), (free0, free1)
    s2 = torch.cuda.Stream()
    mcc.consensus(*args, out=out, stream=s2)
    torch.cuda.synchronize()
    free2 = torch.cuda.mem_get_info()[0]
    assert free1 - free2 >= (16 << 20), (free1, free2)  # the cached path does allocate
    mcc.release_workspace()


def test_noalloc_rejects_beyond_scratch(mcc):
    import torch
    print("[gpu-case] noalloc: instances beyond the scratch array", flush=True)
    # label rows alone exceed the array: refused before any work
    n, k = 1_000_000, 64
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    col = torch.zeros(1, dtype=torch.int32, device="cuda")[:0]
    labels = torch.zeros((k, n), dtype=torch.int32, device="cuda")
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(mcc.MccError) as e:
        mcc.consensus(row_ptr, col, labels, None, out=out, noalloc=True)
    assert e.value.code == mcc.MCC_ESCRATCH
    del labels
    # label rows fit, the contingency tables do not: refused during set-up
    inst = synth.random_instance(200_000, 32, avg_deg=4.0, n_labels=1000, seed=5)
    out = torch.empty(inst.n, dtype=torch.int32, device="cuda")
    args = (dev(inst.row_ptr), dev(inst.col), dev(inst.labels), dev(inst.init))
    with pytest.raises(mcc.MccError) as e:
        mcc.consensus(*args, out=out, noalloc=True)
    assert e.value.code == mcc.MCC_ESCRATCH
    # the array is usable again right after
    small = synth.sbm_small()
    both(mcc, small, small.init)
