"""Python binding of libmcc (median consensus clustering on MI355X).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libmcc.so``; torch tensors provide device memory and streams.
The library must be built (``paper_2408_11331_amd.build.build()``); nothing
here falls back to another implementation when it is missing.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmcc.so")

MCC_OK, MCC_EINVAL, MCC_EGRAPH, MCC_ENOMEM, MCC_EDEVICE, MCC_ENOTSUP = 0, -1, -2, -3, -4, -5
MCC_ESCRATCH = -6
NOALLOC_SCRATCH_BYTES = 256 << 20
MCC_F_VALIDATE, MCC_F_TRACE, MCC_F_LITERAL, MCC_F_PROFILE = 0x1, 0x2, 0x4, 0x8
MCC_F_ARC_CACHE, MCC_F_HASH_TABLES, MCC_F_SYMMETRIC = 0x10, 0x20, 0x40
MCC_F_HASH_ROWS, MCC_F_HASH_KEYS = 0x80, 0x100

# every function include/mcc.h declares
EXPORTS = ("mcc_consensus", "mcc_consensus_noalloc", "mcc_objective", "mcc_mirkin", "mcc_canonicalize",
           "mcc_consensus_batch", "mcc_batch_tune", "mcc_tune_save", "mcc_tune_load",
           "mcc_compare", "mcc_split_join_matrix", "mcc_group_from_distances",
           "mcc_group_partitions", "mcc_release_workspace", "mcc_workspace_bound",
           "mcc_batch_workspace_bytes", "mcc_workspace_held", "mcc_strerror")
MCC_TUNE_LANES, MCC_TUNE_MAX_BUCKETS = 5, 160
TUNE_LANES = (4, 8, 16, 32, 64)


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [
        ("max_rounds", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("stream", ctypes.c_void_p), ("trace", ctypes.c_void_p),
        ("lanes", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("passes", ctypes.c_int32), ("converged", ctypes.c_int32),
        ("fallback_rounds", ctypes.c_int32), ("clusters", ctypes.c_int32),
        ("moves", ctypes.c_int64), ("candidate_evals", ctypes.c_int64),
        ("objective_init", ctypes.c_int64), ("objective", ctypes.c_int64),
        ("ms_total", ctypes.c_float), ("ms_passes", ctypes.c_float),
        ("boundary", ctypes.c_int64), ("ms_score", ctypes.c_float),
        ("lanes_used", ctypes.c_int32), ("tables", ctypes.c_int32),
        ("skipped_evals", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
    ]

    OUT = ("passes", "converged", "fallback_rounds", "clusters", "moves", "candidate_evals",
           "objective_init", "objective", "ms_total", "ms_passes", "boundary", "ms_score",
           "lanes_used", "tables", "skipped_evals", "workspace_bytes")

    def as_dict(self):
        return {f: getattr(self, f) for f in self.OUT}


class Problem(ctypes.Structure):
    _fields_ = [("g", Csr), ("labels", ctypes.c_void_p), ("k", ctypes.c_int32),
                ("init", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class Comparison(ctypes.Structure):
    _fields_ = [("mirkin", ctypes.c_int64), ("split_join_ab", ctypes.c_int64),
                ("split_join_ba", ctypes.c_int64), ("split_join", ctypes.c_int64),
                ("rand", ctypes.c_double), ("vi", ctypes.c_double),
                ("clusters_a", ctypes.c_int32), ("clusters_b", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TuneEntry(ctypes.Structure):
    _fields_ = [("n_log2", ctypes.c_int32), ("k_class", ctypes.c_int32),
                ("lanes", ctypes.c_int32), ("instances", ctypes.c_int32),
                ("cells", ctypes.c_int64), ("ms", ctypes.c_float * MCC_TUNE_LANES),
                ("pad", ctypes.c_int32)]


class TuneTable(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("entry", TuneEntry * MCC_TUNE_MAX_BUCKETS)]

    def as_dict(self):
        return {"wg_per_cu": self.wg_per_cu,
                "buckets": [{"n_log2": e.n_log2, "k_class": e.k_class, "lanes": e.lanes,
                             "instances": e.instances, "cells": e.cells,
                             "ms": dict(zip(TUNE_LANES, [round(x, 4) for x in e.ms]))}
                            for e in self.entry[:self.count]]}


class BatchOpts(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("max_rounds", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("lanes", ctypes.c_int32),
                ("wg_per_cu", ctypes.c_int32), ("status", ctypes.c_void_p),
                ("tune", ctypes.c_void_p), ("tune_cache_path", ctypes.c_char_p),
                ("solved_in_batch", ctypes.c_int32), ("ms_total", ctypes.c_float),
                ("workspace_bytes", ctypes.c_int64)]


class MccError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libmcc error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libmcc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2408_11331_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        p, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.mcc_consensus.argtypes = [ctypes.POINTER(Csr), p, i32, p, p, ctypes.POINTER(Stats)]
        L.mcc_consensus_noalloc.argtypes = [ctypes.POINTER(Csr), p, i32, p, p,
                                            ctypes.POINTER(Stats)]
        L.mcc_consensus_noalloc.restype = ctypes.c_int
        L.mcc_objective.argtypes = [p, p, i32, i64, p, p]
        L.mcc_mirkin.argtypes = [p, p, i64, p, p]
        L.mcc_canonicalize.argtypes = [p, p, i64, p, p]
        L.mcc_consensus_batch.argtypes = [ctypes.POINTER(Problem), i32, ctypes.POINTER(Stats),
                                          ctypes.POINTER(BatchOpts)]
        L.mcc_consensus_batch.restype = ctypes.c_int
        L.mcc_batch_tune.argtypes = [ctypes.POINTER(Problem), i32, ctypes.POINTER(BatchOpts),
                                     ctypes.POINTER(TuneTable)]
        L.mcc_batch_tune.restype = ctypes.c_int
        L.mcc_tune_save.argtypes = [ctypes.POINTER(TuneTable), ctypes.c_char_p]
        L.mcc_tune_save.restype = ctypes.c_int
        L.mcc_tune_load.argtypes = [ctypes.POINTER(TuneTable), ctypes.c_char_p]
        L.mcc_tune_load.restype = ctypes.c_int
        L.mcc_compare.argtypes = [p, p, i64, ctypes.POINTER(Comparison), p]
        L.mcc_split_join_matrix.argtypes = [p, i32, i64, p, p]
        L.mcc_group_from_distances.argtypes = [p, i32, i64, p, p, p]
        L.mcc_group_partitions.argtypes = [p, i32, i64, i64, p, p, p, p, p]
        L.mcc_release_workspace.argtypes = []
        L.mcc_workspace_bound.argtypes = [i64, i64, i32, i64, i64, ctypes.c_uint32, p]
        L.mcc_workspace_bound.restype = ctypes.c_int
        L.mcc_batch_workspace_bytes.argtypes = [ctypes.POINTER(Problem), i32,
                                                ctypes.POINTER(BatchOpts), p]
        L.mcc_batch_workspace_bytes.restype = ctypes.c_int
        L.mcc_workspace_held.argtypes = [p]
        L.mcc_workspace_held.restype = ctypes.c_int
        for f in ("mcc_compare", "mcc_split_join_matrix", "mcc_group_from_distances",
                  "mcc_group_partitions", "mcc_release_workspace"):
            getattr(L, f).restype = ctypes.c_int
        L.mcc_strerror.argtypes = [ctypes.c_int]
        L.mcc_strerror.restype = ctypes.c_char_p
        for f in ("mcc_consensus", "mcc_objective", "mcc_mirkin", "mcc_canonicalize"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise MccError(rc, lib().mcc_strerror(rc).decode())


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_i32(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int32:
        raise TypeError(f"{name} must be a CUDA int32 tensor")
    return t.contiguous()


def _label_ptrs(labels):
    """Labels as a (k, n) tensor or a sequence of n-vectors -> (objects to
    keep alive, ctypes array of row pointers)."""
    if hasattr(labels, "shape") and labels.dim() == 2:
        t = _dev_i32(labels, "labels")  # contiguous: row i starts i * n elements in
        k, n = t.shape
        base, step = t.data_ptr(), n * 4
        arr = (ctypes.c_void_p * max(1, k))(*[base + i * step for i in range(k)])
        return _Rows(t, k, n), arr
    rows = [_dev_i32(r, "labels") for r in labels]
    arr = (ctypes.c_void_p * max(1, len(rows)))(*[r.data_ptr() for r in rows])
    return rows, arr


class _Rows:
    """The rows of a (k, n) tensor without slicing it: len() and numel()."""

    def __init__(self, t, k, n):
        self.t, self.k, self.n = t, k, n

    def __len__(self):
        return self.k

    def __getitem__(self, i):
        return self.t[i]


def consensus(row_ptr, col, labels, init=None, *, max_rounds=0, flags=0, lanes=0,
              stream=None, out=None, trace=False, noalloc=False):
    """Greedy median consensus on the GPU.

    row_ptr: int64 CUDA tensor [n+1]; col: int32 CUDA tensor [nnz];
    labels: int32 CUDA tensor [k, n] (or k tensors [n]); init: int32 [n] in
    [0, n) or None (singletons).  ``noalloc`` calls mcc_consensus_noalloc
    (workspace in the library's static scratch array; pass ``out``).
    Returns ``(out, stats)`` (and the per-pass trace as a list of 4-tuples
    when ``trace``)."""
    import torch
    if row_ptr.dtype != torch.int64 or not row_ptr.is_cuda:
        raise TypeError("row_ptr must be a CUDA int64 tensor")
    row_ptr = row_ptr.contiguous()
    col = _dev_i32(col, "col")
    rows, arr = _label_ptrs(labels)
    n = row_ptr.numel() - 1
    if init is not None:
        init = _dev_i32(init, "init")
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int32, device=row_ptr.device)
    g = Csr(n, col.numel(), row_ptr.data_ptr(), col.data_ptr() if col.numel() else None)
    st = Stats()
    st.max_rounds = max_rounds
    st.flags = flags | (MCC_F_TRACE if trace else 0)
    st.stream = _stream_ptr(stream)
    st.lanes = lanes
    mr = max_rounds if max_rounds > 0 else 1000
    tbuf = (ctypes.c_int64 * (4 * mr))() if trace else None
    st.trace = ctypes.cast(tbuf, ctypes.c_void_p) if trace else None
    fn = lib().mcc_consensus_noalloc if noalloc else lib().mcc_consensus
    _check(fn(ctypes.byref(g), arr, len(rows),
                               init.data_ptr() if init is not None else None,
                               out.data_ptr() if n > 0 else None, ctypes.byref(st)))
    d = st.as_dict()
    if trace:
        tr = [tuple(tbuf[4 * j:4 * j + 4]) for j in range(d["passes"])]
        return out, d, tr
    return out, d


def objective(c, labels, stream=None) -> int:
    c = _dev_i32(c, "c")
    rows, arr = _label_ptrs(labels)
    res = ctypes.c_int64(0)
    _check(lib().mcc_objective(c.data_ptr() if c.numel() else None, arr, len(rows), c.numel(),
                               ctypes.byref(res), _stream_ptr(stream)))
    return res.value


def mirkin(a, b, stream=None) -> int:
    a, b = _dev_i32(a, "a"), _dev_i32(b, "b")
    if a.numel() != b.numel():
        raise ValueError("a and b differ in length")
    res = ctypes.c_int64(0)
    _check(lib().mcc_mirkin(a.data_ptr() if a.numel() else None,
                            b.data_ptr() if b.numel() else None, a.numel(),
                            ctypes.byref(res), _stream_ptr(stream)))
    return res.value


def canonicalize(x, out=None, stream=None):
    import torch
    x = _dev_i32(x, "x")
    if out is None:
        out = torch.empty_like(x)
    cl = ctypes.c_int32(0)
    _check(lib().mcc_canonicalize(x.data_ptr() if x.numel() else None,
                                  out.data_ptr() if x.numel() else None, x.numel(),
                                  ctypes.byref(cl), _stream_ptr(stream)))
    return out, cl.value


def _problems(problems, outs):
    """ctypes array of problems plus the tensors it points into."""
    count = len(problems)
    keep = []
    arr = (Problem * max(1, count))()
    for j, p in enumerate(problems):
        rp = p["row_ptr"].contiguous()
        col = _dev_i32(p["col"], "col")
        rows, larr = _label_ptrs(p["labels"])
        ini = p.get("init")
        ini = None if ini is None else _dev_i32(ini, "init")
        keep.extend([rp, col, rows, larr, ini])
        n = rp.numel() - 1
        arr[j].g = Csr(n, col.numel(), rp.data_ptr(), col.data_ptr() if col.numel() else None)
        arr[j].labels = ctypes.cast(larr, ctypes.c_void_p)
        arr[j].k = len(rows)
        arr[j].init = ini.data_ptr() if ini is not None else None
        arr[j].out = outs[j].data_ptr() if outs is not None and n > 0 else None
    return arr, keep


def _batch_opts(max_rounds, flags, lanes, wg_per_cu, stream, tune, tune_cache_path):
    o = BatchOpts()
    o.stream = _stream_ptr(stream)
    o.max_rounds = max_rounds
    o.flags = flags
    o.lanes = lanes
    o.wg_per_cu = wg_per_cu
    o.tune = ctypes.cast(ctypes.pointer(tune), ctypes.c_void_p) if tune is not None else None
    o.tune_cache_path = tune_cache_path.encode() if tune_cache_path else None
    return o


def consensus_batch(problems, *, max_rounds=0, flags=0, lanes=0, wg_per_cu=0, stream=None,
                    outs=None, tune=None, tune_cache_path=None):
    """Solve many independent instances in one persistent launch.

    problems: sequence of dicts with CUDA tensors ``row_ptr`` (int64),
    ``col`` (int32), ``labels`` (int32 [k, n]) and optional ``init``.
    ``lanes`` 0 takes each instance's lanes per vertex from ``tune`` (a
    TuneTable), else the table file ``tune_cache_path``, else the built-in
    rule.  Returns ``(outs, stats, status, info)``: output tensors,
    per-instance stats dicts, per-instance return codes and the batch call's
    info (instances finished in the persistent kernel, wall time)."""
    import torch
    count = len(problems)
    if outs is None:
        outs = [torch.empty(p["row_ptr"].numel() - 1, dtype=torch.int32,
                            device=p["row_ptr"].device) for p in problems]
    arr, keep = _problems(problems, outs)
    st = (Stats * max(1, count))()
    status = (ctypes.c_int32 * max(1, count))()
    o = _batch_opts(max_rounds, flags, lanes, wg_per_cu, stream, tune, tune_cache_path)
    o.status = ctypes.cast(status, ctypes.c_void_p)
    rc = lib().mcc_consensus_batch(arr, count, st, ctypes.byref(o))
    codes = [status[j] for j in range(count)]
    if rc not in (0, MCC_EINVAL):
        _check(rc)
    return outs, [st[j].as_dict() for j in range(count)], codes, \
        {"solved_in_batch": o.solved_in_batch, "ms_total": o.ms_total, "rc": rc,
         "workspace_bytes": o.workspace_bytes}


def batch_tune(problems, *, max_rounds=0, flags=0, wg_per_cu=0, stream=None,
               tune_cache_path=None):
    """Autotune the batched launch on a sample of a workload: lanes per
    vertex per size bucket, table size and resident workgroups per compute
    unit.  Returns a TuneTable (also written to ``tune_cache_path`` if
    given).  The problems' outputs are not written."""
    arr, keep = _problems(problems, None)
    o = _batch_opts(max_rounds, flags, 0, wg_per_cu, stream, None, tune_cache_path)
    table = TuneTable()
    _check(lib().mcc_batch_tune(arr, len(problems), ctypes.byref(o), ctypes.byref(table)))
    return table


def tune_save(table, path):
    _check(lib().mcc_tune_save(ctypes.byref(table), path.encode()))


def tune_load(path):
    table = TuneTable()
    _check(lib().mcc_tune_load(ctypes.byref(table), path.encode()))
    return table


# ---------------------------------------------------------------------------
# partition comparison and grouping
# ---------------------------------------------------------------------------
def compare(a, b, stream=None) -> dict:
    """Mirkin, split-join (both directions and their sum), Rand distance and
    variation of information of two partitions (CUDA int32 tensors)."""
    a, b = _dev_i32(a, "a"), _dev_i32(b, "b")
    if a.numel() != b.numel():
        raise ValueError("a and b differ in length")
    r = Comparison()
    _check(lib().mcc_compare(a.data_ptr() if a.numel() else None,
                             b.data_ptr() if b.numel() else None, a.numel(), ctypes.byref(r),
                             _stream_ptr(stream)))
    return r.as_dict()


def split_join_matrix(labels, stream=None):
    """k x k split-join distances of the partitions (a (k, n) CUDA int32
    tensor or a sequence of n-vectors), as a numpy int64 array."""
    import numpy as np
    rows, arr = _label_ptrs(labels)
    k, n = len(rows), rows[0].numel()
    d = np.zeros((k, k), np.int64)
    _check(lib().mcc_split_join_matrix(arr, k, n, d.ctypes.data, _stream_ptr(stream)))
    return d


def group_from_distances(dist, lam=-1):
    """Groups of homogeneous partitions from a split-join matrix (host);
    lam < 0 picks the threshold by the elbow rule.  Returns (group ids,
    number of groups, threshold used)."""
    import numpy as np
    d = np.ascontiguousarray(dist, np.int64)
    k = d.shape[0]
    g = np.zeros(k, np.int32)
    ng, used = ctypes.c_int32(0), ctypes.c_int64(0)
    _check(lib().mcc_group_from_distances(d.ctypes.data, k, int(lam), g.ctypes.data,
                                          ctypes.byref(ng), ctypes.byref(used)))
    return g, ng.value, used.value


def group_partitions(labels, lam=-1, stream=None):
    """split_join_matrix followed by group_from_distances, in one call.
    Returns (group ids, number of groups, threshold used, distances)."""
    import numpy as np
    rows, arr = _label_ptrs(labels)
    k, n = len(rows), rows[0].numel()
    d = np.zeros((k, k), np.int64)
    g = np.zeros(k, np.int32)
    ng, used = ctypes.c_int32(0), ctypes.c_int64(0)
    _check(lib().mcc_group_partitions(arr, k, n, int(lam), g.ctypes.data, ctypes.byref(ng),
                                      ctypes.byref(used), d.ctypes.data, _stream_ptr(stream)))
    return g, ng.value, used.value, d


def consensus_groups(row_ptr, col, labels, lam=-1, init="first", max_rounds=0, flags=0,
                     stream=None):
    """The paper's pipeline: group the homogeneous input partitions, then one
    consensus per group, all groups in one batched launch.  ``init``:
    "first" starts each group from its first partition, "singleton" from
    singletons.  Returns (group ids, threshold used, per-group outputs,
    per-group stats)."""
    import torch
    lab = labels if hasattr(labels, "shape") else torch.stack(list(labels))
    g, ng, used, _ = group_partitions(lab, lam, stream=stream)
    probs = []
    for j in range(ng):
        members = [i for i in range(len(g)) if g[i] == j]
        sub = lab[members].contiguous()
        # cluster ids must lie in [0, n): the first partition, relabelled
        start = canonicalize(sub[0].contiguous(), stream=stream)[0] if init == "first" else None
        probs.append({"row_ptr": row_ptr, "col": col, "labels": sub, "init": start})
    outs, stats, codes, _ = consensus_batch(probs, max_rounds=max_rounds, flags=flags,
                                            stream=stream)
    for c in codes:
        if c != 0:
            raise MccError(c, lib().mcc_strerror(c).decode())
    return g, used, outs, stats


def workspace_bound(n, nnz, k, max_label, clusters=0, flags=0) -> int:
    """Upper bound of the device workspace of one solve of that size (host)."""
    b = ctypes.c_int64(0)
    _check(lib().mcc_workspace_bound(int(n), int(nnz), int(k), int(max_label), int(clusters),
                                     int(flags), ctypes.byref(b)))
    return b.value


def batch_workspace_bytes(problems, *, lanes=0, wg_per_cu=0, tune=None, tune_cache_path=None) -> int:
    """Device workspace of one batched call over these problems (host)."""
    arr, keep = _problems(problems, None)
    o = BatchOpts()
    o.lanes, o.wg_per_cu = lanes, wg_per_cu
    o.tune = ctypes.cast(ctypes.pointer(tune), ctypes.c_void_p) if tune is not None else None
    o.tune_cache_path = tune_cache_path.encode() if tune_cache_path else None
    b = ctypes.c_int64(0)
    _check(lib().mcc_batch_workspace_bytes(arr, len(problems), ctypes.byref(o), ctypes.byref(b)))
    return b.value


def workspace_held() -> int:
    """Workspace the library keeps between calls on the current device,
    shared by every stream (host)."""
    b = ctypes.c_int64(0)
    _check(lib().mcc_workspace_held(ctypes.byref(b)))
    return b.value


def release_workspace():
    """Free the device workspace the library keeps between calls."""
    _check(lib().mcc_release_workspace())


# ---------------------------------------------------------------------------
# packed batches: many instances in a few concatenated device tensors
# ---------------------------------------------------------------------------
_PROBLEM_DTYPE = None


def _problem_dtype():
    """numpy record with the memory layout of mcc_problem (and of Problem)."""
    global _PROBLEM_DTYPE
    if _PROBLEM_DTYPE is None:
        import numpy as np
        _PROBLEM_DTYPE = np.dtype({
            "names": ["n", "nnz", "row_ptr", "col", "labels", "k", "init", "out"],
            "formats": ["<i8", "<i8", "<u8", "<u8", "<u8", "<i4", "<u8", "<u8"],
            "offsets": [Csr.n.offset, Csr.nnz.offset, Csr.row_ptr.offset, Csr.col.offset,
                        Problem.labels.offset, Problem.k.offset, Problem.init.offset,
                        Problem.out.offset],
            "itemsize": ctypes.sizeof(Problem)})
    return _PROBLEM_DTYPE


class PackedBatch:
    """Instances concatenated on the device: row offsets, arcs, labels
    (each instance's k x n block, row-major), initial clusters and outputs,
    with per-instance offsets; the mcc_problem records that point into them
    are built once, with array arithmetic.  Build with pack_batch."""

    def __init__(self, row_ptr, col, labels, init, out, n, nnz, k, rp_off, col_off, lab_off,
                 has_init):
        import numpy as np
        self.row_ptr, self.col, self.labels, self.init, self.out = row_ptr, col, labels, init, out
        self.n, self.nnz, self.k = n, nnz, k
        self.count = int(n.size)
        self.v_off = np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)
        # host array of all label row pointers: instance j, partition i
        kcum = np.concatenate([[0], np.cumsum(k)]).astype(np.int64)
        inst = np.repeat(np.arange(self.count), k)
        part = np.arange(int(kcum[-1])) - kcum[inst]
        self.label_rows = (labels.data_ptr() + 4 * (lab_off[inst] + part * n[inst])).astype(np.uint64)
        rec = np.zeros(self.count, dtype=_problem_dtype())
        rec["n"], rec["nnz"], rec["k"] = n, nnz, k
        rec["row_ptr"] = row_ptr.data_ptr() + 8 * rp_off
        rec["col"] = np.where(nnz > 0, col.data_ptr() + 4 * col_off, 0)
        rec["labels"] = self.label_rows.ctypes.data + 8 * kcum[:-1]
        rec["init"] = np.where(has_init, init.data_ptr() + 4 * self.v_off, 0)
        rec["out"] = np.where(n > 0, out.data_ptr() + 4 * self.v_off, 0)
        self.records = rec
        self.stats = (Stats * max(1, self.count))()
        self.status = (ctypes.c_int32 * max(1, self.count))()

    def output(self, j):
        """The output tensor of instance j (a view into the packed outputs)."""
        o = int(self.v_off[j])
        return self.out[o:o + int(self.n[j])]


def pack_batch(instances, device="cuda"):
    """Concatenate host instances (objects with numpy row_ptr int64 [n+1],
    col int32, labels int32 [k, n] and init int32 [n] or None) into one
    PackedBatch resident on the device."""
    import numpy as np
    import torch
    n = np.array([i.row_ptr.size - 1 for i in instances], np.int64)
    nnz = np.array([i.col.size for i in instances], np.int64)
    k = np.array([i.labels.shape[0] for i in instances], np.int64)
    rp_off = np.concatenate([[0], np.cumsum(n + 1)[:-1]]).astype(np.int64)
    col_off = np.concatenate([[0], np.cumsum(nnz)[:-1]]).astype(np.int64)
    lab_off = np.concatenate([[0], np.cumsum(n * k)[:-1]]).astype(np.int64)
    has_init = np.array([i.init is not None for i in instances])
    T = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dt)).to(device)
    row_ptr = T(np.concatenate([i.row_ptr for i in instances]), np.int64)
    col = T(np.concatenate([i.col for i in instances] + [np.zeros(1, np.int32)]), np.int32)
    labels = T(np.concatenate([i.labels.reshape(-1) for i in instances] + [np.zeros(1, np.int32)]),
               np.int32)
    init = T(np.concatenate([i.init if i.init is not None else np.zeros(i.row_ptr.size - 1, np.int32)
                             for i in instances] + [np.zeros(1, np.int32)]), np.int32)
    out = torch.empty(int(n.sum()) + 1, dtype=torch.int32, device=device)
    return PackedBatch(row_ptr, col, labels, init, out, n, nnz, k, rp_off, col_off, lab_off, has_init)


def consensus_batch_packed(pb, *, max_rounds=0, flags=0, lanes=0, wg_per_cu=0, stream=None,
                           tune=None, tune_cache_path=None):
    """mcc_consensus_batch over a PackedBatch: outputs land in pb.out (see
    pb.output(j)), per-instance stats in pb.stats, codes in pb.status.
    Returns the batch call's info (instances finished in the persistent
    kernel, wall time, return code)."""
    o = _batch_opts(max_rounds, flags, lanes, wg_per_cu, stream, tune, tune_cache_path)
    o.status = ctypes.cast(pb.status, ctypes.c_void_p)
    recs = ctypes.cast(pb.records.ctypes.data, ctypes.POINTER(Problem))
    rc = lib().mcc_consensus_batch(recs, pb.count, pb.stats, ctypes.byref(o))
    if rc not in (0, MCC_EINVAL):
        _check(rc)
    return {"solved_in_batch": o.solved_in_batch, "ms_total": o.ms_total, "rc": rc,
            "workspace_bytes": o.workspace_bytes}
