#!/usr/bin/env python3
"""Write the stored expected results of the full-size workloads.

CPU only.  Every instance comes from the seeded generators (``synth``) and
every expected value from the oracle (``oracle``); nothing here loads or
calls the GPU library.  For each solve the record holds the instance's
digest (so that a test can check that it regenerated the same instance),
the oracle's statistics, its per-pass trace where kept, and the sha256 of
its output cluster ids (int32, little endian).

    python tests/golden/make_goldens.py [--only sbm_small,lfr,gmm_knn,sbm_batch,served]
                                        [--workers 4]

Files (next to this script): sbm_small.json, lfr.json, gmm_knn.json,
sbm_batch.json (every instance of the batched workload, one compact row
each) and served_pool.json (every request of the served pool).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

STAT_KEYS = ("passes", "converged", "fallback_rounds", "clusters", "moves", "candidate_evals",
             "objective_init", "objective")


def out_sha(out) -> str:
    return hashlib.sha256(np.ascontiguousarray(out, "<i4").tobytes()).hexdigest()


def solve_record(inst, init_kind: str, keep_trace: bool = True) -> dict:
    init = inst.init if init_kind == "p0" else None
    t0 = time.perf_counter()
    out, st, tr = oracle.consensus(inst.row_ptr, inst.col, inst.labels, init, trace=True)
    rec = {"workload": inst.name, "digest": inst.digest(), "n": inst.n, "k": inst.k,
           "nnz": inst.nnz, "init": init_kind,
           "stats": {key: int(st[key]) for key in STAT_KEYS},
           "out_sha256": out_sha(out), "oracle_seconds": round(time.perf_counter() - t0, 2)}
    if keep_trace:
        rec["trace"] = [[int(x) for x in row] for row in tr]
    return rec


def log(msg):
    print(f"[goldens] {msg}", flush=True)


def write(name, payload):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(payload, f, indent=1, sort_keys=True)
        f.write("\n")
    log(f"wrote {path}")


# ---- single instances -------------------------------------------------------
_INST = {}


def _solve_cached(args):
    key, init_kind = args
    return solve_record(_INST[key], init_kind)


def single(name, builder, inits, workers):
    t0 = time.perf_counter()
    _INST[name] = builder()
    inst = _INST[name]
    log(f"{name}: n={inst.n} nnz={inst.nnz} k={inst.k} built in "
        f"{time.perf_counter() - t0:.1f} s")
    jobs = [(name, i) for i in inits]
    if workers > 1 and len(jobs) > 1:
        with mp.get_context("fork").Pool(min(workers, len(jobs))) as pool:
            recs = pool.map(_solve_cached, jobs)
    else:
        recs = [_solve_cached(j) for j in jobs]
    for r in recs:
        log(f"{name}/{r['init']}: {r['stats']} in {r['oracle_seconds']} s")
    write(f"{name}.json", {"workload": name, "generator": "synth." + name, "meta": {
        key: v for key, v in inst.meta.items() if isinstance(v, (int, float, str))},
        "solves": recs})
    del _INST[name]


# ---- the batched workload -----------------------------------------------------
def _batch_row(spec):
    inst = synth.sbm_batch_instance(spec)
    out, st, _ = oracle.consensus(inst.row_ptr, inst.col, inst.labels, inst.init)
    return [spec["index"], inst.digest()[:16], out_sha(out)[:16]] + [int(st[k]) for k in STAT_KEYS]


def batch(workers):
    specs = synth.sbm_batch_specs()
    t0 = time.perf_counter()
    rows = []
    with mp.get_context("fork").Pool(workers) as pool:
        for j, r in enumerate(pool.imap_unordered(_batch_row, specs, chunksize=4)):
            rows.append(r)
            if (j + 1) % 256 == 0:
                log(f"sbm_batch: {j + 1}/{len(specs)} in {time.perf_counter() - t0:.0f} s")
    rows.sort()
    write("sbm_batch.json", {
        "workload": "sbm_batch", "generator": "synth.sbm_batch_specs + synth.sbm_batch_instance",
        "count": len(rows), "columns": ["index", "digest16", "out_sha16", *STAT_KEYS],
        "rows": rows})


# ---- the served pool -----------------------------------------------------------
def _served_rec(spec):
    inst = synth.served_instance(spec)
    rec = solve_record(inst, "p0", keep_trace=False)
    rec["spec"] = spec
    return rec


def served(workers):
    specs = synth.served_pool_specs()
    with mp.get_context("fork").Pool(workers) as pool:
        recs = pool.map(_served_rec, specs[::-1], chunksize=1)[::-1]
    for r in recs:
        log(f"served {r['spec']}: {r['stats']} in {r['oracle_seconds']} s")
    write("served_pool.json", {"workload": "served", "generator":
                               "synth.served_pool_specs + synth.served_instance", "requests": recs})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="sbm_small,lfr,gmm_knn,sbm_batch,served")
    ap.add_argument("--workers", type=int, default=4)
    args = ap.parse_args()
    oracle.build(force=False)
    only = args.only.split(",")
    if "sbm_small" in only:
        single("sbm_small", synth.sbm_small, ["p0", "singleton"], args.workers)
    if "lfr" in only:
        single("lfr", synth.lfr, ["p0", "singleton"], args.workers)
    if "gmm_knn" in only:
        single("gmm_knn", synth.gmm_knn, ["p0", "singleton"], args.workers)
    if "served" in only:
        served(args.workers)
    if "sbm_batch" in only:
        batch(args.workers)


if __name__ == "__main__":
    main()
