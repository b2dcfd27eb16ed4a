"""Measured choice of block size k and method per (n, q) -- the automated
selection of k that the paper's Section 5 leaves as future work, extended to
the choice between the plain (Section 3.2) and contracted (Section 3.1)
methods.

    python -m paper_1706_06940_amd.autotune [--quick] [--out PATH]

For every (n, q) of a grid it times whole offline batches (median of the
library's kernel-attached stage events) for each candidate (method, k) and
keeps the fastest.  The result is a JSON table that `load_plan_table()`
installs into the library's planner (rmq_planner_set_table), which then
serves rmq_plan / path AUTO / batches from it.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NS = [10 ** 4, 10 ** 5, 10 ** 6, 10 ** 7, 10 ** 8]
QS = [10, 100, 10 ** 3, 10 ** 4, 10 ** 5, 10 ** 6, 10 ** 7]
FULL_KS = [256, 512, 1024, 2048, 4096, 8192, 16384, 65536]
CON_KS = [16, 64, 256, 512, 1024, 4096]
# two block levels (Section 3.3): (k, k1) pairs of the plain method
FULL2_KS = [(8192, 256), (16384, 512), (32768, 512), (65536, 1024), (262144, 1024)]


def time_call(rmq, A, L, R, path, k, reps, timer, k1=0):
    ts = []
    for _ in range(reps):
        rmq.query_batch(A, L, R, path=path, block_size=k, sub_block_size=k1, timer=timer)
        ts.append(timer.read()[1])
    return statistics.median(ts)


def tune(ns=NS, qs=QS, full_ks=FULL_KS, con_ks=CON_KS, full2_ks=FULL2_KS, reps=5,
         max_q_over_n=10, log=print):
    import torch

    import paper_1706_06940_amd as rmq
    import workloads as W

    d = torch.device("cuda:0")
    timer = rmq.Timer()
    entries = []
    for n in ns:
        A = torch.from_numpy(W.uniform_int31(n, W.BASE_SEED + 31)).to(d)
        for q in qs:
            if q > max_q_over_n * n:
                continue
            Lh, Rh = W.uniform_queries(n, q, W.BASE_SEED + 32)
            L, R = torch.from_numpy(Lh).to(d), torch.from_numpy(Rh).to(d)
            cands = [("full", k, 0) for k in full_ks if k <= max(256, n)]
            cands += [("contracted", k, 0) for k in con_ks if k <= max(16, 2 * q)]
            cands += [("full", k, k1) for k, k1 in full2_ks if 4 * k <= n]
            res = {}
            for path, k, k1 in cands:
                rmq.query_batch(A, L, R, path=path, block_size=k, sub_block_size=k1)  # warm-up
                res[(path, k, k1)] = time_call(rmq, A, L, R, path, k, reps, timer, k1)
            (bp, bk, bk1), bt = min(res.items(), key=lambda kv: kv[1])
            one = {c: t for c, t in res.items() if c[2] == 0}
            (op, ok, _), _ = min(one.items(), key=lambda kv: kv[1])
            e = {"n": n, "q": q, "block_size": bk, "path": bp, "ms": round(bt, 5),
                 "candidates": {f"{p}/{k}" + (f"/{k1}" if k1 else ""): round(t, 5)
                                for (p, k, k1), t in res.items()}}
            if bk1:
                # two levels won; batches (one level) take the best one-level
                # plan, which must use the same method for the table's path
                e["sub_block_size"] = bk1
                e["one_level_block_size"] = ok if op == "full" else min(
                    (t, k) for (p, k, k1), t in res.items() if p == "full" and k1 == 0)[1]
            entries.append(e)
            log(f"[tune] n={n:>10} q={q:>9}: {bp}/{bk}" + (f"/{bk1}" if bk1 else "") +
                f" {bt * 1e3:8.1f} us")
    return {"device": torch.cuda.get_device_name(d), "reps": reps,
            "created": time.strftime("%Y-%m-%d %H:%M:%S"), "entries": entries}


def main() -> int:
    import paper_1706_06940_amd as rmq

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=rmq.TUNE_TABLE)
    ap.add_argument("--quick", action="store_true", help="small grid (for tests)")
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    if args.quick:
        table = tune(ns=[10 ** 4, 10 ** 6], qs=[10, 10 ** 4], full_ks=[256, 1024, 4096],
                     con_ks=[16, 512], full2_ks=[(8192, 256)], reps=3)
    else:
        table = tune(reps=args.reps)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(f"[tune] wrote {len(table['entries'])} entries to {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
