"""Python access to the plain CPU oracle (``mccref.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package smoke check
and by the benchmark's CPU-baseline leg.  The GPU library never imports or
links this module, and this module never touches the GPU library.

All arrays are host numpy arrays.  Labels are passed partition-major as an
int32 array of shape (k, n).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libmccref.so")
SRC = os.path.join(HERE, "mccref.c")

EINVAL, EGRAPH, ENOMEM = -1, -2, -3


class Stats(ctypes.Structure):
    _fields_ = [
        ("max_rounds", ctypes.c_int32),
        ("literal_self_term", ctypes.c_int32),
        ("passes", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("fallback_rounds", ctypes.c_int32),
        ("clusters", ctypes.c_int32),
        ("moves", ctypes.c_int64),
        ("candidate_evals", ctypes.c_int64),
        ("objective_init", ctypes.c_int64),
        ("objective", ctypes.c_int64),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_
                if f not in ("max_rounds", "literal_self_term")}


def build(force: bool = True) -> str:
    """Compile the oracle into a shared library next to its source."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC",
                               "-shared", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        p = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        L.mccref_mirkin.argtypes = [p, p, i64, p]
        L.mccref_objective.argtypes = [p, p, i32, i64, p]
        L.mccref_delta.argtypes = [p, p, i32, i64, i64, i32, p]
        L.mccref_score.argtypes = [p, p, i64, p, i32, p, i64, i64, i32, p, p, p]
        L.mccref_consensus.argtypes = [p, p, i64, p, i32, p, p, p, p]
        L.mccref_consensus_rule.argtypes = [p, p, i64, p, i32, p, p, p, p, i32]
        L.mccref_canonicalize.argtypes = [p, p, i64, p]
        L.mccref_compare.argtypes = [p, p, i64, p]
        L.mccref_split_join_matrix.argtypes = [p, i32, i64, p]
        L.mccref_group.argtypes = [p, i32, i64, p, p]
        L.mccref_elbow_lambda.argtypes = [p, i32, p]
        for f in ("mccref_mirkin", "mccref_objective", "mccref_delta", "mccref_score",
                  "mccref_consensus", "mccref_consensus_rule", "mccref_canonicalize",
                  "mccref_compare",
                  "mccref_split_join_matrix", "mccref_group", "mccref_elbow_lambda"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle returned {code}")
        self.code = code


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _check(rc):
    if rc != 0:
        raise OracleError(rc)


def mirkin(a, b) -> int:
    a, b = _i32(a), _i32(b)
    out = np.zeros(1, np.int64)
    _check(lib().mccref_mirkin(_ptr(a), _ptr(b), a.size, out.ctypes.data))
    return int(out[0])


def objective(c, labels) -> int:
    c, labels = _i32(c), _i32(labels)
    out = np.zeros(1, np.int64)
    _check(lib().mccref_objective(_ptr(c), _ptr(labels), labels.shape[0], c.size,
                                  out.ctypes.data))
    return int(out[0])


def delta(c, labels, v, target) -> int:
    c, labels = _i32(c), _i32(labels)
    out = np.zeros(1, np.int64)
    _check(lib().mccref_delta(_ptr(c), _ptr(labels), labels.shape[0], c.size, int(v),
                              int(target), out.ctypes.data))
    return int(out[0])


def score(row_ptr, col, labels, c, v_begin=0, v_end=None, literal=False):
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    col, labels, c = _i32(col), _i32(labels), _i32(c)
    n = row_ptr.size - 1
    v_end = n if v_end is None else v_end
    m = v_end - v_begin
    best = np.zeros(max(m, 1), np.int32)
    dbest = np.zeros(max(m, 1), np.int64)
    ncand = np.zeros(max(m, 1), np.int32)
    _check(lib().mccref_score(_ptr(row_ptr), _ptr(col), n, _ptr(labels), labels.shape[0],
                              _ptr(c), v_begin, v_end, int(literal), best.ctypes.data,
                              dbest.ctypes.data, ncand.ctypes.data))
    return best[:m], dbest[:m], ncand[:m]


def consensus(row_ptr, col, labels, init=None, max_rounds=0, literal=False, trace=False):
    """Run the oracle's consensus.  Returns ``(out, stats_dict, trace_or_None)``."""
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    col, labels = _i32(col), _i32(labels)
    n = row_ptr.size - 1
    ini = None if init is None else _i32(init)
    out = np.zeros(max(n, 1), np.int32)
    st = Stats()
    st.max_rounds = max_rounds
    st.literal_self_term = int(literal)
    mr = max_rounds if max_rounds > 0 else 1000
    tr = np.zeros((mr, 4), np.int64) if trace else None
    rc = lib().mccref_consensus(_ptr(row_ptr), _ptr(col), n, _ptr(labels), labels.shape[0],
                                _ptr(ini), out.ctypes.data, ctypes.byref(st),
                                tr.ctypes.data if tr is not None else None)
    _check(rc)
    d = st.as_dict()
    if tr is not None:
        tr = tr[: d["passes"]]
    return out[:n], d, tr


RULES = {"pinned": 0, "one_best": 1, "alternate": 2, "unchecked": 3}


def consensus_rule(row_ptr, col, labels, init=None, rule="pinned", max_rounds=0, literal=False,
                   trace=False):
    """The consensus under one of the round rules of ``RULES`` (Methods,
    "Parallel algorithm"): the pinned rule, one best move per pass, direction
    alternation, or the unchecked batch.  Returns ``(out, stats, trace)``."""
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    col, labels = _i32(col), _i32(labels)
    n = row_ptr.size - 1
    ini = None if init is None else _i32(init)
    out = np.zeros(max(n, 1), np.int32)
    st = Stats()
    st.max_rounds = max_rounds
    st.literal_self_term = int(literal)
    mr = max_rounds if max_rounds > 0 else 1000
    tr = np.zeros((mr, 4), np.int64) if trace else None
    rc = lib().mccref_consensus_rule(_ptr(row_ptr), _ptr(col), n, _ptr(labels), labels.shape[0],
                                     _ptr(ini), out.ctypes.data, ctypes.byref(st),
                                     tr.ctypes.data if tr is not None else None, RULES[rule])
    _check(rc)
    d = st.as_dict()
    if tr is not None:
        tr = tr[: d["passes"]]
    return out[:n], d, tr


def canonicalize(a):
    a = _i32(a)
    out = np.zeros(max(a.size, 1), np.int32)
    cl = np.zeros(1, np.int32)
    _check(lib().mccref_canonicalize(_ptr(a), out.ctypes.data, a.size, cl.ctypes.data))
    return out[: a.size], int(cl[0])


class _Comparison(ctypes.Structure):
    _fields_ = [("mirkin", ctypes.c_int64), ("split_join_ab", ctypes.c_int64),
                ("split_join_ba", ctypes.c_int64), ("split_join", ctypes.c_int64),
                ("rand", ctypes.c_double), ("vi", ctypes.c_double),
                ("clusters_a", ctypes.c_int32), ("clusters_b", ctypes.c_int32)]


def compare(a, b) -> dict:
    """Mirkin, split-join (both directions and their sum), Rand distance and
    variation of information between two partitions (Results, "Evaluation
    metrics")."""
    a, b = _i32(a), _i32(b)
    r = _Comparison()
    _check(lib().mccref_compare(_ptr(a), _ptr(b), a.size, ctypes.byref(r)))
    return {f: getattr(r, f) for f, _ in r._fields_}


def split_join_matrix(labels) -> np.ndarray:
    """k x k split-join distances between the input partitions."""
    labels = _i32(labels)
    k, n = labels.shape
    d = np.zeros((k, k), np.int64)
    _check(lib().mccref_split_join_matrix(_ptr(labels), k, n, d.ctypes.data))
    return d


def group(dist, lam):
    """Connected components of the partitions linked at distance <= lam."""
    dist = np.ascontiguousarray(dist, np.int64)
    k = dist.shape[0]
    g = np.zeros(k, np.int32)
    ng = ctypes.c_int32(0)
    _check(lib().mccref_group(dist.ctypes.data, k, int(lam), g.ctypes.data, ctypes.byref(ng)))
    return g, ng.value


def elbow_lambda(dist) -> int:
    dist = np.ascontiguousarray(dist, np.int64)
    lam = ctypes.c_int64(0)
    _check(lib().mccref_elbow_lambda(dist.ctypes.data, dist.shape[0], ctypes.byref(lam)))
    return lam.value
