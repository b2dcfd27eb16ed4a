#!/usr/bin/env python3
"""Throughput of batched offline RMQ on one MI355X.

Workload (the paper's scale, Section 4): A = 1e8 int32 values uniform in
[0, 2^31); query batches of q in {1e3, 1e4, 1e5, 1e6, 1e7} with both
endpoints uniform over [0, n) and swapped so l <= r.  A step answers every
batch of the sweep with both methods -- the block Sparse Table over A
(Section 3.2) and the contracted one (Section 3.1) -- through the C ABI,
each call doing the whole offline job (build + answers).  Inputs are resident
in HBM before timing starts.

value  = queries answered per second over the timed steps (all batches, both
         methods), timed with events on the stream the library runs on.
roofline = the full-array block-minima pass (the dominant kernel of the
         plain method): algorithmic bytes 4n + 8 ceil(n/k) over its average
         duration, measured with the library's per-stage events.
cpu_baseline = the CPU oracle (Sparse Table over 32-element blocks, build +
         answers for every batch of the sweep) on this host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("queries/s and HBM GB/s (% of peak) at n=1e8, q=1e3..1e7; "
          "p50/p99 latency served")
HBM_PEAK_GBS = 8000.0


def table_levels(nb: int) -> int:
    """Levels of the doubling block table over nb blocks (the library's
    rule: floor(log2(nb - 2)) + 1, one level for nb <= 3)."""
    return 1 if nb <= 3 else (nb - 2).bit_length()


def algorithmic_bytes(path: str, n: int, q: int, k: int, k1: int, lo: int, hi: int):
    """Bytes one whole job must move through HBM, by stage (Table 1's four
    stages), from the per-unit figures of the method:
      block minima: 4 B per element of A read + 8 B per block written;
      block table: 8 B per (block, level) written (+ 8 B per k1-block read
        and 8 B per block written when the blocks come from k1-blocks);
      queries: 12 B each (L, R read, out written), + 8 B of LR each on A_Q;
      endpoint sort: 2q 8-byte items read and written per pass of 8 key
        bits, ceil(log2 n / 8) passes, + remap 12 B per endpoint;
      contraction: 4 B per element between the outermost endpoints + 8 B per
        endpoint + 8 B per A_Q entry written;
      A_Q's table: 8 B per A_Q entry read, then as the block table above.
    lo, hi: smallest left and largest right endpoint of the batch."""
    def table(m, kk, kk1, per_elem):
        nb = -(-m // kk)
        b = 8 * nb * table_levels(nb)
        if kk1:
            nb1 = -(-m // kk1)
            return per_elem * m + 8 * nb1, b + 8 * nb1 + 8 * nb
        return per_elem * m + 8 * nb, b
    if path == "full":
        pass_b, st_b = table(n, k, k1, 4)
        return {"sort": 0, "contract_or_blockmin": pass_b, "sparse_table": st_b,
                "query": 12 * q}
    m = 2 * q - 1
    passes = -(-max(1, (n - 1).bit_length()) // 8)
    sort_b = passes * 2 * (2 * q) * 8 + 12 * (2 * q)
    contract_b = 4 * (hi - lo + 1) + 8 * (2 * q) + 8 * m
    pass_b, st_b = table(m, k, k1, 8)
    return {"sort": sort_b, "contract_or_blockmin": contract_b, "sparse_table": pass_b + st_b,
            "query": 20 * q}


def cpu_facts() -> dict:
    """The host's CPU model and core counts, for the oracle's baseline."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"cpu_model": model, "nproc": usable, "logical_cpus": os.cpu_count()}


def parse_qs(s: str):
    return [int(float(x)) for x in s.split(",") if x]


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=10 ** 8)
    ap.add_argument("--qs", default="1e3,1e4,1e5,1e6,1e7")
    ap.add_argument("--paths", default="full,contracted")
    ap.add_argument("--k-full", type=int, default=0, help="0 = planner's choice")
    ap.add_argument("--k-con", type=int, default=0, help="0 = the library's default per q")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--verify", action="store_true",
                    help="check every answer of the first step against the oracle")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="before timing, run one plain device copy of BYTES bytes (a known "
                         "HBM traffic figure to scale profiler byte counters by)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="repeat the CPU oracle sweep until this much time has passed")
    ap.add_argument("--no-batched", action="store_true", help="skip the many-arrays measurement")
    ap.add_argument("--no-served", action="store_true", help="skip the serving measurement")
    ap.add_argument("--served-requests", type=int, default=3000)
    ap.add_argument("--no-flushed", action="store_true",
                    help="skip the cache-flushed block-minima measurement")
    ap.add_argument("--flushed-reps", type=int, default=7)
    ap.add_argument("--no-lca", action="store_true",
                    help="skip the LCA front-end measurement (5e8-node tree)")
    ap.add_argument("--no-skewed", action="store_true",
                    help="skip the n = 1e9 skewed-query measurement")
    ap.add_argument("--no-lary", action="store_true",
                    help="skip the table-over-powers-of-l measurement")
    ap.add_argument("--no-resident", action="store_true",
                    help="skip the resident-index query-only measurement")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the small-instance measurement (n = 2^20, q = 1024)")
    ap.add_argument("--no-permutation", action="store_true",
                    help="skip the paper's permutation workload at n = 1e8")
    ap.add_argument("--blockmin-sweep", default="",
                    help="counter-profiling mode: after --copy-calibration, one block-minima "
                         "launch per listed block size on the n-element array, then exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}, world size {world}); "
              "the multi-GPU form of this method is a design note only", file=sys.stderr)
        return 2

    import torch

    import paper_1706_06940_amd as rmq
    import workloads as W

    d = torch.device("cuda:0")
    n = args.n
    qs = parse_qs(args.qs)
    paths = [p for p in args.paths.split(",") if p]
    seed = W.BASE_SEED + 1
    t0 = time.time()
    A_h = W.uniform_int31(n, seed)
    batches_h = [W.uniform_queries(n, q, seed, 100 + 2 * j) for j, q in enumerate(qs)]
    print(f"[bench] generated n={n} and {len(qs)} batches in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    A = torch.from_numpy(A_h).to(d)
    batches = [(torch.from_numpy(L).to(d), torch.from_numpy(R).to(d)) for L, R in batches_h]
    outs = [torch.empty(q, dtype=torch.int32, device=d) for q in qs]
    # block size per batch: the autotuner's table for the full method (its
    # entries all choose that method at this n), the contracted default else
    rmq.load_plan_table()

    def k_for(p, q):
        """(block size, sub-block size) of the batch; sub-block size > 0 is a
        two-level plan (Section 3.3) chosen by the autotuner."""
        if p == "full":
            if args.k_full:
                return args.k_full, 0
            k, path, k1 = rmq.plan_ex(n, q)
            return (k, k1) if path == "full" else (rmq.default_block(n, q, "full"), 0)
        if args.k_con:
            return args.k_con, 0
        # the library's default plan for the contracted method
        return rmq.default_block(n, q, "contracted"), rmq.default_sub_block(n, q, "contracted")

    plans = {p: {q: k_for(p, q) for q in qs} for p in ("full", "contracted")}
    k_used = {p: {q: plans[p][q][0] for q in qs} for p in plans}
    k1_used = {p: {q: plans[p][q][1] for q in qs} for p in plans}
    torch.cuda.synchronize()

    def step(timers=None):
        for p in paths:
            for j, q in enumerate(qs):
                L, R = batches[j]
                rmq.query_batch(A, L, R, path=p, block_size=k_used[p][q],
                                sub_block_size=k1_used[p][q], out=outs[j],
                                timer=timers[(p, j)] if timers else None)

    if args.copy_calibration:
        src = torch.empty(args.copy_calibration // 4, dtype=torch.int32, device=d).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.blockmin_sweep:
        ks = [int(x) for x in args.blockmin_sweep.split(",") if x]
        for k in ks:
            rmq.block_minima(A, k)
        torch.cuda.synchronize()
        print(json.dumps({"blockmin_sweep": ks, "n": n}), flush=True)
        return 0

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    if args.verify:
        import oracle

        orc = oracle.Oracle()
        for p in paths:
            for j, q in enumerate(qs):
                L, R = batches[j]
                got = rmq.query_batch(A, L, R, path=p, block_size=k_used[p][q],
                                      sub_block_size=k1_used[p][q]).cpu().numpy()
                exp = orc.rmq_sparse_table(A_h, batches_h[j][0], batches_h[j][1], 32)
                if not np.array_equal(got, exp):
                    print(f"[bench] MISMATCH path={p} q={q}", file=sys.stderr, flush=True)
                    return 1
        print("[bench] verified all batches against the oracle", file=sys.stderr, flush=True)

    # ---- timed region: plain launches, nothing attached ----
    stream = torch.cuda.current_stream(d)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for s in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    ms_per_step = total_ms / args.steps
    answered = sum(qs) * len(paths)
    value = answered / (ms_per_step / 1e3)

    # ---- the same steps again with the library's stage clock attached
    # (events recorded on the kernels themselves) for the per-stage figures
    # and the block-minima launch durations; not part of `value` ----
    timers = [{(p, j): rmq.Timer() for p in paths for j in range(len(qs))}
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    ev0.record(stream)
    for s in range(args.steps):
        step(timers[s])
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_per_step_clocked = ev0.elapsed_time(ev1) / args.steps

    # per-call and per-stage figures from the library's stage events
    breakdown = {}
    blockmin = []  # (block size, ms) of every full-method block-minima launch
    for p in paths:
        for j, q in enumerate(qs):
            per = [timers[s][(p, j)].read() for s in range(args.steps)]
            tot = statistics.median(t for _, t in per)
            stages = [statistics.median(st[i] for st, _ in per) for i in range(4)]
            L_h, R_h = batches_h[j]
            ab = algorithmic_bytes(p, n, q, k_used[p][q], k1_used[p][q], int(L_h.min()),
                                   int(R_h.max()))
            job_b = sum(ab.values())
            gbs = job_b / (tot / 1e3) / 1e9
            stage_gbs = {name: (round(ab[name] / (v / 1e3) / 1e9, 1) if v > 0 and ab[name] else None)
                         for name, v in zip(rmq.STAGE_NAMES, stages)}
            breakdown[f"{p}/q={q}"] = {
                "ms": round(tot, 4), "queries_per_s": round(q / (tot / 1e3), 1),
                "algorithmic_bytes": job_b, "GB_per_s": round(gbs, 1),
                "frac": round(gbs / HBM_PEAK_GBS, 4),
                "block_size": k_used[p][q], "sub_block_size": k1_used[p][q],
                "stage_ms": {name: round(v, 4) for name, v in zip(rmq.STAGE_NAMES, stages)},
                "stage_algorithmic_bytes": ab,
                "stage_GB_per_s": stage_gbs,
                "stage_frac": {name: (round(v / HBM_PEAK_GBS, 4) if v else None)
                               for name, v in stage_gbs.items()}}
            if p == "full":
                # the pass over A takes the k1-block minima under two levels
                kb = k1_used[p][q] or k_used[p][q]
                blockmin += [(kb, st[1]) for st, _ in per]
    roofline = None
    if blockmin:
        # algorithmic bytes of one launch: A once + one 8-byte key per block
        algo = [4 * n + 8 * (-(-n // k)) for k, _ in blockmin]
        avg_ms = sum(ms for _, ms in blockmin) / len(blockmin)
        avg_bytes = sum(algo) / len(algo)
        achieved = sum(algo) / (sum(ms for _, ms in blockmin) / 1e3) / 1e9
        prof = profiled_traffic(n)
        traffic = None
        if prof is not None and all(str(k) in prof for k, _ in blockmin):
            traffic = round(sum(prof[str(k)] for k, _ in blockmin) / len(blockmin))
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic,
                    "kernel": "k_blockmin_i32", "avg_ms": round(avg_ms, 5),
                    "algorithmic_bytes": round(avg_bytes),
                    "launches": len(blockmin),
                    "traffic_source": os.path.relpath(TRAFFIC_PROFILE, ROOT)}

    # the part's achievable read rate for this pass: the same loads over the
    # same A, keeping nothing (25 launches timed by events attached to them;
    # the bench's own helper library, not part of librmq)
    probe = read_probe_lib()
    if roofline is not None and probe is not None:
        sink = torch.zeros(1, dtype=torch.int32, device=d)
        s_ptr = int(torch.cuda.current_stream(d).cuda_stream)
        probe.bench_read_probe_ms(A.data_ptr(), n, sink.data_ptr(), 2, s_ptr)
        probe_ms = probe.bench_read_probe_ms(A.data_ptr(), n, sink.data_ptr(), 25, s_ptr)
        if probe_ms > 0:
            probe_gbs = 16 * (n // 4) / (probe_ms / 1e3) / 1e9  # 4 floor(n/4) int32 read
            roofline["read_ceiling"] = {
                "achieved": round(probe_gbs, 1), "frac": round(probe_gbs / HBM_PEAK_GBS, 4),
                "kernel_over_ceiling": round(roofline["achieved"] / probe_gbs, 4),
                "how": "bench_aux/read_probe.hip: the block-minima loads over the same A with "
                       "nothing kept, mean of 25 back-to-back launches"}

    # the same block-minima launches after a 1 GB write that evicts A from the
    # L2s and the MALL (the paper's cache flush before every repetition)
    if roofline is not None and not args.no_flushed:
        scratch = torch.empty(1 << 28, dtype=torch.int32, device=d)
        t_fl = rmq.Timer()
        ms_fl, bytes_fl = [], []
        for j, q in enumerate(qs):
            L, R = batches[j]
            for _ in range(args.flushed_reps):
                scratch.fill_(j)
                rmq.query_batch(A, L, R, path="full", block_size=k_used["full"][q],
                                sub_block_size=k1_used["full"][q], out=outs[j], timer=t_fl)
                ms_fl.append(t_fl.read()[0][1])
                kb = k1_used["full"][q] or k_used["full"][q]
                bytes_fl.append(4 * n + 8 * (-(-n // kb)))
        del scratch
        med = statistics.median(b / (m / 1e3) / 1e9 for b, m in zip(bytes_fl, ms_fl))
        roofline["flushed"] = {"achieved": round(med, 1), "frac": round(med / HBM_PEAK_GBS, 4),
                               "launches": len(ms_fl),
                               "how": "median over launches, each after writing 1 GiB of scratch"}

    # resident index: build once, then query-only batches (Section 3.2's
    # structure kept in HBM between batches)
    resident = None
    if not args.no_resident and "full" in paths:
        k_res, k1_res = k_used["full"][max(qs)], k1_used["full"][max(qs)]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        idx = rmq.Index(A, k_res, sub_block_size=k1_res)
        e1.record(stream)
        torch.cuda.synchronize()
        build_ms = e0.elapsed_time(e1)
        q_ms = {}
        for j, q in enumerate(qs):
            L, R = batches[j]
            reps = []
            for r in range(9):
                e0.record(stream)
                idx.query(L, R, out=outs[j])
                e1.record(stream)
                torch.cuda.synchronize()
                if r >= 2:
                    reps.append(e0.elapsed_time(e1))
            q_ms[str(q)] = round(statistics.median(reps), 4)
        resident = {"block_size": k_res, "sub_block_size": k1_res, "index_bytes": idx.bytes, "build_ms": round(build_ms, 4),
                    "query_ms": q_ms,
                    "queries_per_s": {q: round(int(q) / (ms / 1e3), 1) for q, ms in q_ms.items()}}
        del idx

    cpu = None
    if not args.no_cpu:
        import oracle

        orc = oracle.Oracle()
        reps, t = 0, time.perf_counter()
        while True:
            for j, q in enumerate(qs):
                orc.rmq_sparse_table(A_h, batches_h[j][0], batches_h[j][1], 32)
            reps += 1
            dt = time.perf_counter() - t
            if dt >= args.cpu_seconds or reps >= 200:
                break
        cpu = {"value": round(reps * sum(qs) / dt, 1), "unit": "queries/s",
               "cores": orc.num_threads(), "kind": "oracle",
               "omp_threads": orc.num_threads(), **cpu_facts(),
               "sample": (f"oracle Sparse Table over 32-element blocks, build + answers for "
                          f"each batch of the sweep q={qs} on the same n={n} array, "
                          f"{reps} sweeps in {dt:.1f}s on the host")}
        # one thread, one sweep
        threads = orc.num_threads()
        orc.set_threads(1)
        t = time.perf_counter()
        for j, q in enumerate(qs):
            orc.rmq_sparse_table(A_h, batches_h[j][0], batches_h[j][1], 32)
        dt1 = time.perf_counter() - t
        orc.set_threads(threads)
        cpu["value_1thread"] = round(sum(qs) / dt1, 1)
        cpu["sample_1thread"] = f"the same sweep once on 1 thread in {dt1:.1f}s"

    del A, batches, outs
    torch.cuda.empty_cache()
    small = None if args.no_small else bench_small(d)
    permutation = None if args.no_permutation else bench_permutation(d, qs)
    skewed = None if args.no_skewed else bench_skewed(d)
    lca = None if args.no_lca else bench_lca(d)
    lary = None if args.no_lary else bench_lary(d)
    batched = None if args.no_batched else bench_batched(d)
    served = None if args.no_served else bench_served(d, args.served_requests)

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "ms_per_step_with_stage_clock": round(ms_per_step_clocked, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": (f"batched RMQ, n={n} int32 uniform in [0,2^31), batches "
                                f"q={qs} uniform swapped queries, each answered by "
                                f"{' and '.join(paths)} method(s)"),
                   "n": n, "q": qs, "paths": paths,
                   "block_size": {p: k_used[p] for p in paths},
                   "sub_block_size": {p: k1_used[p] for p in paths},
                   "parallelism": "single GPU"},
        "value_cache_state": ("warm: A (400 MB) and the batches stay in HBM across steps with no "
                              "flush between them; part of the data may still sit in the 256 MB "
                              "MALL from the previous call. roofline.flushed is the block-minima "
                              "pass after a 1 GiB write before every launch"),
        "roofline": roofline, "cpu_baseline": cpu, "breakdown": breakdown,
        "resident": resident, "small": small, "permutation": permutation,
        "skewed": skewed, "lca": lca, "lary": lary,
        "batched": batched, "served": served,
    }
    print(json.dumps(line), flush=True)
    return 0


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_blockmin_i32_n1e8_traffic.md")


def read_probe_lib():
    """The benchmark's read-rate helper (bench_aux/libreadprobe.so), or None
    when it has not been built."""
    import ctypes

    path = os.path.join(ROOT, "bench_aux", "libreadprobe.so")
    if not os.path.exists(path):
        print("[bench] bench_aux/libreadprobe.so not built: no read ceiling", file=sys.stderr,
              flush=True)
        return None
    lib = ctypes.CDLL(path)
    v = ctypes.c_void_p
    lib.bench_read_probe_ms.argtypes = [v, ctypes.c_int64, v, ctypes.c_int32, v]
    lib.bench_read_probe_ms.restype = ctypes.c_float
    return lib


def profiled_traffic(n: int):
    """HBM bytes per launch of the block-minima kernel, by block size, from the
    committed counter profile (FETCH_SIZE / WRITE_SIZE, calibrated), when it
    was taken on this workload and on the kernel source as it is now; else
    None."""
    import hashlib

    if n != 10 ** 8 or not os.path.exists(TRAFFIC_PROFILE):
        return None
    text = open(TRAFFIC_PROFILE).read()
    block = text.split("```json", 1)[1].split("```", 1)[0]
    meta = json.loads(block)
    src = os.path.join(ROOT, meta["source"])
    cur = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if cur != meta["source_sha256"] or meta.get("n") != n:
        return None
    return {k: v["traffic_bytes"] for k, v in meta["per_block_size"].items()}


def time_runs(fn, stream, warmup=2, reps=5):
    import torch

    for _ in range(warmup):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    stream.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_small(d, warm_reps=20, flushed_reps=7):
    """The small instance: n = 2^20 uniform int32 (4 MiB, which stays in the
    L2s and the MALL between calls), q = 1024 uniform swapped queries; both
    methods over block sizes 256 .. 16384.  Warm: mean of back-to-back whole
    jobs.  Flushed: median of jobs each after writing 1 GiB of scratch.  Not a
    bandwidth point: A is cache-resident when warm."""
    import torch

    import paper_1706_06940_amd as rmq
    import workloads as W

    n, q = 1 << 20, 1024
    seed = W.BASE_SEED + 0
    A = torch.from_numpy(W.uniform_int31(n, seed)).to(d)
    L_h, R_h = W.uniform_queries(n, q, seed, 1)
    L, R = torch.from_numpy(L_h).to(d), torch.from_numpy(R_h).to(d)
    out = torch.empty(q, dtype=torch.int32, device=d)
    stream = torch.cuda.current_stream(d)
    scratch = torch.empty(1 << 28, dtype=torch.int32, device=d)
    t = rmq.Timer()
    res, ref = {}, None
    for path in ("full", "contracted"):
        for k in (256, 1024, 4096, 16384):
            run = lambda tm=None: rmq.query_batch(A, L, R, path=path, block_size=k, out=out,
                                                  timer=tm)
            run()
            torch.cuda.synchronize()
            if ref is None:
                ref = out.clone()
            same = bool(torch.equal(out, ref))
            warm = time_runs(run, stream, warmup=2, reps=warm_reps)
            fl = []
            for r in range(flushed_reps):
                scratch.fill_(r)
                run(t)
                fl.append(t.read()[1])
            flushed = statistics.median(fl)
            res[f"{path}/k={k}"] = {"warm_ms": round(warm, 4), "flushed_ms": round(flushed, 4),
                                    "warm_queries_per_s": round(q / (warm / 1e3), 1),
                                    "flushed_queries_per_s": round(q / (flushed / 1e3), 1),
                                    "same_answers_as_first": same}
    del A, scratch
    torch.cuda.empty_cache()
    return {"workload": "n=2^20 int32 uniform in [0,2^31), q=1024 uniform swapped queries",
            "results": res}


def bench_permutation(d, qs, reps=5):
    """The paper's own array workload: 1..n after n/2 random pair swaps (no
    ties), n = 1e8, with uniform swapped queries over the same q sweep; both
    methods with the planner's block sizes, and the comparison system
    ST-RMQ_CON (Section 2, Fig. 1's baseline); whole offline jobs (mean of
    `reps`)."""
    import torch

    import paper_1706_06940_amd as rmq
    import workloads as W

    n = 10 ** 8
    seed = W.BASE_SEED + 6
    t0 = time.time()
    A = torch.from_numpy(W.paper_permutation(n, seed)).to(d)
    print(f"[bench] permutation of {n} drawn in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    stream = torch.cuda.current_stream(d)
    res = {}
    for j, q in enumerate(qs):
        L_h, R_h = W.uniform_queries(n, q, seed, 10 + 2 * j)
        L, R = torch.from_numpy(L_h).to(d), torch.from_numpy(R_h).to(d)
        k, path_f, k1 = rmq.plan_ex(n, q)
        if path_f != "full":
            k, k1 = rmq.default_block(n, q, "full"), 0
        outs = {}
        for path in ("full", "contracted", "st_con"):
            if path == "st_con":  # the comparison system: no blocks
                kk, kk1 = 0, 0
            else:
                kk = k if path == "full" else rmq.default_block(n, q, "contracted")
                kk1 = k1 if path == "full" else rmq.default_sub_block(n, q, "contracted")
            out = torch.empty(q, dtype=torch.int32, device=d)
            run = lambda: rmq.query_batch(A, L, R, path=path, block_size=kk, sub_block_size=kk1,
                                          out=out)
            ms = time_runs(run, stream, warmup=2, reps=reps)
            outs[path] = out
            res[f"{path}/q={q}"] = {"ms": round(ms, 4), "queries_per_s": round(q / (ms / 1e3), 1),
                                    "block_size": kk, "sub_block_size": kk1}
        res[f"full/q={q}"]["same_answers_as_contracted"] = bool(
            torch.equal(outs["full"], outs["contracted"]))
        res[f"st_con/q={q}"]["same_answers_as_contracted"] = bool(
            torch.equal(outs["st_con"], outs["contracted"]))
        # the paper's Fig. 1 ratio (BbST_CON over ST-RMQ_CON), and the plain method's
        st_ms = res[f"st_con/q={q}"]["ms"]
        res[f"st_con/q={q}"]["contracted_speedup"] = round(st_ms / res[f"contracted/q={q}"]["ms"], 2)
        res[f"st_con/q={q}"]["full_speedup"] = round(st_ms / res[f"full/q={q}"]["ms"], 2)
    del A
    torch.cuda.empty_cache()
    return {"workload": "n=1e8: 1..n after n/2 uniform pair swaps (the paper's array), "
                        f"q={qs} uniform swapped queries; st_con: the comparison system "
                        "ST-RMQ_CON re-created on this GPU, with each method's speedup over it",
            "results": res}


def bench_skewed(d, reps=5):
    """n = 1e9 uniform int32 (4 GB, drawn in HBM by the generator's torch
    form), q = 1e7: half short ranges (length uniform in [1, 1024]), half
    uniform long ones.  The plain method with one, two and three block levels
    (Section 3.3), and the contracted method; whole offline jobs (mean of
    `reps` after a first run that also counts the entries read by partial-block
    scans)."""
    import torch

    import paper_1706_06940_amd as rmq
    import workloads as W

    n, q = 10 ** 9, 10 ** 7
    seed = W.BASE_SEED + 2
    A = W.uniform_int31_torch(n, seed, 0, device=d)
    L_h, R_h = W.skewed_queries(n, q, seed)
    L, R = torch.from_numpy(L_h).to(d), torch.from_numpy(R_h).to(d)
    out = torch.empty(q, dtype=torch.int32, device=d)
    stream = torch.cuda.current_stream(d)
    configs = [("full", 4096, 0, 0), ("full", 16384, 0, 0), ("full", 16384, 256, 0),
               ("full", 65536, 256, 0), ("full", 65536, 1024, 0), ("full", 65536, 1024, 64),
               ("full", 65536, 2048, 128), ("full", 262144, 4096, 128), ("contracted", 0, 0, 0)]
    res = {}
    ref = None
    for path, k, k1, k2 in configs:
        stats = torch.zeros(2, dtype=torch.int64, device=d)
        run = lambda st=None: rmq.query_batch(A, L, R, path=path, block_size=k,
                                              sub_block_size=k1, sub_block_size2=k2, out=out,
                                              stats=st)
        run(stats)
        torch.cuda.synchronize()
        got = out.clone()
        if ref is None:
            ref = got
        same = bool(torch.equal(got, ref))
        ms = time_runs(run, stream, warmup=0, reps=reps)
        name = f"{path}/k={k or 'default'}" + (f"/k1={k1}" if k1 else "") + \
            (f"/k2={k2}" if k2 else "")
        scans, reads = stats.tolist()
        res[name] = {"ms": round(ms, 4), "queries_per_s": round(q / (ms / 1e3), 1),
                     "partial_scans": scans, "entries_read_by_scans": reads,
                     "same_answers_as_first": same}
        print(f"[bench] skewed {name}: {ms:.3f} ms", file=sys.stderr, flush=True)
    del A
    torch.cuda.empty_cache()
    return {"workload": "n=1e9 int32 uniform in [0,2^31), q=1e7: 5e6 short ranges (length "
                        "uniform in [1,1024]) and 5e6 uniform long ranges, shuffled",
            "results": res}


def bench_lary(d, reps=5):
    """The block table over powers of l = 2^a instead of 2 (Section 3.1's
    generalisation) against the doubling table (a = 1) on the plain method:
    n = 1e8 uniform int32, q = 1e7 uniform queries, small blocks (where the
    table is large).  Whole offline jobs and resident-index queries (mean of
    `reps`), and the table's bytes."""
    import torch

    import paper_1706_06940_amd as rmq
    import workloads as W

    n, q = 10 ** 8, 10 ** 7
    seed = W.BASE_SEED + 5
    A = W.uniform_int31_torch(n, seed, 0, device=d)
    L, R = W.uniform_queries_torch(n, q, seed, 1, device=d)
    out = torch.empty(q, dtype=torch.int32, device=d)
    stream = torch.cuda.current_stream(d)
    res = {}
    for k in (32, 256):
        ref = None
        for a in (1, 2, 4, 5):
            ws = torch.empty(rmq.workspace_bytes(n, q, "full", k, arity_log2=a),
                             dtype=torch.uint8, device=d)
            job = lambda: rmq.query_batch(A, L, R, path="full", block_size=k, arity_log2=a,
                                          out=out, workspace=ws)
            job_ms = time_runs(job, stream, warmup=1, reps=reps)
            got = out.clone()
            ref = got if ref is None else ref
            idx = rmq.Index(A, k, arity_log2=a)
            q_ms = time_runs(lambda: idx.query(L, R, out=out), stream, warmup=1, reps=reps)
            res[f"k={k}/l={2 ** a}"] = {
                "levels": idx.levels, "table_bytes": idx.bytes, "job_ms": round(job_ms, 4),
                "index_query_ms": round(q_ms, 4),
                "same_answers_as_doubling": bool(torch.equal(got, ref))}
            del idx, ws
            print(f"[bench] lary k={k} l={2 ** a}: job {job_ms:.3f} ms, index query "
                  f"{q_ms:.3f} ms", file=sys.stderr, flush=True)
    del A, L, R, out
    torch.cuda.empty_cache()
    return {"workload": "n=1e8 int32 uniform in [0,2^31), q=1e7 uniform queries, plain method",
            "results": res}


def bench_lca(d, N=5 * 10 ** 8, q=10 ** 7, reps=5):
    """LCA through RMQ (Section 1) on a random recursive tree of N nodes
    (parent(i) uniform in [0, i)): the device build of the Euler tour (2N - 1
    steps) and its RMQ index, then batches of q uniform (u, v) pairs."""
    import torch

    import paper_1706_06940_amd as rmq
    import workloads as W

    seed = W.BASE_SEED + 2
    parent = torch.from_numpy(W.random_recursive_tree(N, seed)).to(d)
    rng = np.random.default_rng(seed)
    u = torch.from_numpy(rng.integers(0, N, q).astype(np.int32)).to(d)
    v = torch.from_numpy(rng.integers(0, N, q).astype(np.int32)).to(d)
    out = torch.empty(q, dtype=torch.int32, device=d)
    stream = torch.cuda.current_stream(d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = rmq.LCA(parent)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    ms = time_runs(lambda: h.query(u, v, out=out), stream, warmup=1, reps=reps)
    res = {"workload": f"random recursive tree, N={N} nodes (Euler tour of {2 * N - 1} steps), "
                       f"q={q} uniform node pairs",
           "build_ms": round(build_ms, 2), "query_ms": round(ms, 4),
           "queries_per_s": round(q / (ms / 1e3), 1), "device_bytes": h.bytes}
    h.free()
    del parent, u, v, out
    torch.cuda.empty_cache()
    print(f"[bench] lca build {build_ms:.1f} ms, query {ms:.3f} ms", file=sys.stderr, flush=True)
    return res


def bench_batched(d, count=256):
    """Many arrays of uneven length, each with its own query batch: one launch
    per phase for all of them (eager and replayed from a hipGraph) against one
    call per array.  n_j log-uniform in [1e4, 1e7], q_j log-uniform in
    [10, 1e5], values uniform in [0, 2^31), uniform queries."""
    import torch

    import paper_1706_06940_amd as rmq
    import workloads as W

    seed = W.BASE_SEED + 4
    rmq.load_plan_table()
    ns = W.loguniform_ints(count, 1e4, 1e7, seed, 1)
    qs = W.loguniform_ints(count, 10, 1e5, seed, 2)
    arrays = [W.uniform_int31_torch(int(n), seed, 100 + j, device=d) for j, n in enumerate(ns)]
    queries = [W.uniform_queries_torch(int(n), int(q), seed, 1000 + 2 * j, device=d)
               for j, (n, q) in enumerate(zip(ns, qs))]
    b = rmq.Batch(arrays, queries)
    plans = [b.plan(j) for j in range(count)]
    s = torch.cuda.Stream(device=d)
    res = {}
    outs = {}
    with torch.cuda.stream(s):
        for mode in ("per_item", "fused"):
            for graph in (False, True):
                ms = time_runs(lambda: b.run(mode, graph=graph, stream=s), s)
                res[mode + ("_graph" if graph else "")] = ms
            outs[mode] = [o.clone() for o in b.outs]
    s.synchronize()
    same = all(torch.equal(x, y) for x, y in zip(outs["per_item"], outs["fused"]))
    Q, N = int(qs.sum()), int(ns.sum())
    b.free()
    return {
        "workload": (f"{count} arrays, n log-uniform in [1e4,1e7] (total {N}), q log-uniform "
                     f"in [10,1e5] (total {Q}), int32 uniform values, uniform queries"),
        "plans": {"full": sum(p == "full" for _, p in plans),
                  "contracted": sum(p == "contracted" for _, p in plans),
                  "block_sizes": sorted({k for k, _ in plans})},
        "ms": {k: round(v, 4) for k, v in res.items()},
        "queries_per_s": {k: round(Q / (v / 1e3), 1) for k, v in res.items()},
        "input_GB_per_s": {k: round(4 * N / (v / 1e3) / 1e9, 1) for k, v in res.items()},
        "speedup_vs_per_item": {k: round(res["per_item"] / v, 3) for k, v in res.items()},
        "fused_equals_per_item": same,
    }


def bench_served(d, n_req):
    """64 resident arrays (n log-uniform in [1e6, 1e8]) and their block Sparse
    Tables; requests of q log-uniform in [1, 1e5] uniform queries on a
    uniformly chosen array.  Capacity with every request arriving at once,
    then Poisson arrivals at 0.5 / 0.8 / 0.95 of it; the same for the plain
    per-request server (one slot, one request per launch)."""
    import numpy as np

    import workloads as W
    from paper_1706_06940_amd import serving

    seed = W.BASE_SEED + 5
    ns = W.loguniform_ints(64, 1e6, 1e8, seed, 1)
    arrays = [W.uniform_int31_torch(int(n), seed, 200 + j, device=d) for j, n in enumerate(ns)]
    reqs = serving.make_requests(ns, n_req, 1, 1e5, seed)
    out = {"workload": (f"64 resident arrays, n log-uniform in [1e6,1e8] (total {int(ns.sum())}); "
                        f"{n_req} requests, q log-uniform in [1,1e5], uniform queries")}
    for name, cfg in (("coalesced", dict(num_streams=4, max_requests_per_batch=4096,
                                         budget_bytes=4 * 12 * (1 << 21) + (1 << 20))),
                      ("coalesced_copying", dict(num_streams=4, max_requests_per_batch=4096,
                                                 budget_bytes=4 * 12 * (1 << 21) + (1 << 20),
                                                 copy_queries=True)),
                      ("per_request", dict(num_streams=1, max_requests_per_batch=1,
                                           budget_bytes=12 * (1 << 21) + (1 << 20),
                                           copy_queries=True))):
        with serving.Server(max_tables=64, **cfg) as srv:
            for A in arrays:
                srv.add_array(A)
            serving.run_schedule(srv, reqs[:200], [serving.clock()] * 200)  # warm-up
            sat = serving.run_schedule(srv, reqs, [serving.clock()] * len(reqs))
            entry = {"capacity": sat.summary(),
                     "capacity_requests_per_s": round(len(reqs) / sat.makespan_s, 1)}
            if name == "coalesced":
                base_rate = len(reqs) / sat.makespan_s
            # untimed open-loop runs first: the first one or two open-loop
            # runs after the saturated one have each shown a single queueing
            # stall of about 10 ms (every later run is free of it)
            for w, frac in enumerate((0.5, 0.8)):
                serving.run_schedule(srv, reqs, serving.poisson_schedule(
                    len(reqs), frac * base_rate, seed + 7 + w, serving.clock() + 5e-3))
            for frac in (0.5, 0.8, 0.95):
                t0 = serving.clock() + 5e-3
                arr = serving.poisson_schedule(len(reqs), frac * base_rate, seed + int(100 * frac), t0)
                r = serving.run_schedule(srv, reqs, arr)
                entry[f"poisson_{frac}"] = dict(r.summary(), rate_requests_per_s=round(frac * base_rate, 1))
            st = srv.stats()
            entry["max_batches_in_flight"] = st["max_inflight"]
            entry["index_bytes"] = st["index_bytes"]
            out[name] = entry
    out["poisson_rates_are_fractions_of"] = "the coalesced server's capacity"
    return out


if __name__ == "__main__":
    sys.exit(main())
