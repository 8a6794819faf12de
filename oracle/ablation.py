"""Round-rule ablation study on the oracle (Methods, "Parallel algorithm":
applying every vertex's best move together is claimed to reach the same
quality as one best move per iteration, in a few more iterations).

TEST INFRASTRUCTURE: runs only the CPU oracle on seeded synthetic SBM
instances (the batched workload's generator: planted blocks, degree 8-32,
mixing 0.1-0.5, k input partitions each reassigning 20% of the vertices to a
neighbour's block), from the first input partition and from singletons, and
prints one markdown row per instance and rule.

    python -m oracle.ablation [--count 12] [--n-max 400]
"""
from __future__ import annotations

import argparse
import time

import numpy as np

import oracle
import synth

RULES = ("pinned", "one_best", "alternate", "unchecked", "literal")


def run(inst, init, rule, max_rounds):
    t0 = time.perf_counter()
    if rule == "literal":  # the paper's printed gain (self pair kept), pinned rule
        out, st, _ = oracle.consensus_rule(inst.row_ptr, inst.col, inst.labels, init,
                                           rule="pinned", max_rounds=max_rounds, literal=True)
    else:
        out, st, _ = oracle.consensus_rule(inst.row_ptr, inst.col, inst.labels, init, rule=rule,
                                           max_rounds=max_rounds)
    return st, time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=12)
    ap.add_argument("--n-max", type=int, default=400)
    ap.add_argument("--max-rounds", type=int, default=5000)
    args = ap.parse_args()
    oracle.build(force=False)
    specs = synth.sbm_batch_specs(count=args.count, n_range=(100, args.n_max), b_range=(4, 16),
                                  k_range=(4, 16))
    print("| instance | n | k | init | rule | passes | moves | converged | objective | vs pinned |")
    print("|---|---|---|---|---|---|---|---|---|---|")
    summary = {}
    for sp in specs:
        inst = synth.sbm_batch_instance(sp)
        for init_name, init in (("P_0", inst.init), ("singletons", None)):
            ref = None
            for rule in RULES:
                st, _ = run(inst, init, rule, args.max_rounds)
                if rule == "pinned":
                    ref = st["objective"]
                rel = st["objective"] / ref if ref else float("nan")
                print(f"| {sp['index']} | {sp['n']} | {sp['k']} | {init_name} | {rule} | "
                      f"{st['passes']} | {st['moves']} | {st['converged']} | {st['objective']} | "
                      f"{rel:.4f} |", flush=True)
                s = summary.setdefault((init_name, rule), [])
                s.append((st["passes"], st["moves"], st["converged"], rel))
    print()
    print("| init | rule | mean passes | mean moves | converged | mean objective vs pinned |")
    print("|---|---|---|---|---|---|")
    for (init_name, rule), rows in summary.items():
        a = np.array(rows, dtype=np.float64)
        print(f"| {init_name} | {rule} | {a[:, 0].mean():.1f} | {a[:, 1].mean():.1f} | "
              f"{int(a[:, 2].sum())}/{len(rows)} | {a[:, 3].mean():.4f} |")


if __name__ == "__main__":
    main()
