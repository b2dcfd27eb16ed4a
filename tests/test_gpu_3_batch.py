"""Batches of many arrays (one launch per phase for all of them, and graph
replays), bit-exact against the oracle and against one call per array."""
import numpy as np
import pytest
import torch

import paper_1706_06940_amd as rmq
import workloads as W
from tests._gpu import dev, host, need_gpu, reference, say

pytestmark = pytest.mark.gpu


def make_batch(count, n_lo, n_hi, q_lo, q_hi, seed):
    ns = W.loguniform_ints(count, n_lo, n_hi, seed, 1)
    qs = W.loguniform_ints(count, q_lo, q_hi, seed, 2)
    arrays, queries = [], []
    for j, (n, q) in enumerate(zip(ns, qs)):
        n, q = int(n), int(q)
        A = W.uniform_int31(n, seed + 1000 + j) if j % 3 else \
            np.random.default_rng(j).integers(0, 5, n).astype(np.int32)
        L, R = W.uniform_queries(n, q, seed + 2000 + j)
        arrays.append(A)
        queries.append((L, R))
    return arrays, queries


def check_outs(orc, arrays, queries, outs, what):
    for j, (A, (L, R), o) in enumerate(zip(arrays, queries, outs)):
        got = host(o)
        exp = reference(orc, A, L, R)
        assert np.array_equal(got, exp), (what, j, A.shape[0], L.shape[0])


def to_dev(arrays, queries, d):
    return ([dev(A, d) for A in arrays], [(dev(L, d), dev(R, d)) for L, R in queries])


@pytest.mark.parametrize("mode", ["fused", "per_item"])
def test_batch_matches_oracle(orc, mode):
    d = need_gpu()
    say("batch", mode)
    arrays, queries = make_batch(48, 1e3, 2e5, 1, 5e3, 11)
    # edge cases: a one-element array, an empty query batch, a query per element
    arrays += [np.array([7], dtype=np.int32), W.uniform_int31(5000, 3), W.uniform_int31(300, 4)]
    queries += [(np.array([0], dtype=np.int32), np.array([0], dtype=np.int32)),
                (np.empty(0, dtype=np.int32), np.empty(0, dtype=np.int32)),
                (np.arange(300, dtype=np.int32), np.arange(300, dtype=np.int32))]
    At, Qt = to_dev(arrays, queries, d)
    b = rmq.Batch(At, Qt)
    b.run(mode)
    check_outs(orc, arrays, queries, b.outs, mode)
    b.free()


def test_batch_mixed_methods_and_block_sizes(orc):
    d = need_gpu()
    say("batch_mixed")
    arrays, queries = make_batch(24, 1e3, 1e5, 10, 3e3, 21)
    paths = ["contracted" if j % 4 == 0 else ("full" if j % 4 == 1 else "auto")
             for j in range(len(arrays))]
    ks = [0 if j % 2 else (16 << (j % 8)) for j in range(len(arrays))]
    At, Qt = to_dev(arrays, queries, d)
    b = rmq.Batch(At, Qt, block_sizes=ks, paths=paths)
    for j in range(len(arrays)):
        k, p = b.plan(j)
        assert (k & (k - 1)) == 0 and p in ("full", "contracted")
        if paths[j] != "auto":
            assert p == paths[j]
        if ks[j]:
            assert k == ks[j]
    for mode in ("fused", "per_item"):
        for o in b.outs:
            o.fill_(-7)
        b.run(mode)
        check_outs(orc, arrays, queries, b.outs, mode)
    b.free()


@pytest.mark.parametrize("mode", ["fused", "per_item"])
def test_batch_graph_replays(orc, mode):
    """Captured once, replayed with new query contents between replays and
    eager work and synchronisations in between; every replay is checked."""
    d = need_gpu()
    say("batch_graph", mode)
    arrays, queries = make_batch(32, 1e3, 1e5, 5, 2e3, 31)
    At, Qt = to_dev(arrays, queries, d)
    b = rmq.Batch(At, Qt)
    s = torch.cuda.Stream(device=d)
    for rep in range(4):
        # fresh queries written in place: the graph reads whatever L, R hold
        cur = []
        for j, (A, (L, R)) in enumerate(zip(arrays, queries)):
            Ln, Rn = W.uniform_queries(A.shape[0], L.shape[0], 500 + 37 * rep + j)
            Qt[j][0].copy_(torch.from_numpy(Ln))
            Qt[j][1].copy_(torch.from_numpy(Rn))
            cur.append((Ln, Rn))
        for o in b.outs:
            o.fill_(-1)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            b.run(mode, graph=True, stream=s)
        s.synchronize()
        check_outs(orc, arrays, cur, b.outs, f"{mode} replay {rep}")
        # eager single-array work in between
        eager = rmq.query_batch(At[0], Qt[0][0], Qt[0][1])
        assert np.array_equal(host(eager), reference(orc, arrays[0], *cur[0]))
    b.free()


def test_batch_equals_plain_calls(orc):
    d = need_gpu()
    say("batch_vs_plain")
    arrays, queries = make_batch(16, 1e4, 1e6, 100, 1e4, 41)
    At, Qt = to_dev(arrays, queries, d)
    b = rmq.Batch(At, Qt)
    b.run("fused")
    for j in range(len(arrays)):
        plain = rmq.query_batch(At[j], Qt[j][0], Qt[j][1])
        assert torch.equal(plain, b.outs[j])
    b.free()


@pytest.mark.parametrize("mode", ["fused", "per_item"])
def test_batch_two_level_items(orc, mode):
    """Items the planner gives two block levels (Section 3.3) run through the
    batched k1-block minima, the k-blocks from them and the two-level query
    launch, beside one-level items; every answer vs the oracle, eagerly and
    on graph replays."""
    d = need_gpu()
    say("batch_two_level", mode)
    arrays, queries = make_batch(40, 2e3, 3e5, 1, 4e3, 51)
    # every array near 1e5 elements takes k = 8192 over k1 = 256, near 1e4
    # one level with k = 256
    rmq.set_plan_table([(10 ** 5, 10 ** 3, 8192, "full", 256, 512),
                        (10 ** 4, 10 ** 3, 256, "full")])
    try:
        At, Qt = to_dev(arrays, queries, d)
        b = rmq.Batch(At, Qt)
        plans = [b.plan_ex(j) for j in range(len(arrays))]
        two = [j for j, (k, p, k1) in enumerate(plans) if k1 > 0]
        assert 0 < len(two) < len(arrays)
        for j in two:
            k, p, k1 = plans[j]
            assert p == "full" and k1 == 256 and k == 8192
        s = torch.cuda.Stream(device=d)
        for graph in (False, True, True):
            for o in b.outs:
                o.fill_(-3)
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                b.run(mode, graph=graph, stream=s)
            s.synchronize()
            check_outs(orc, arrays, queries, b.outs, f"{mode} graph={graph}")
        b.free()
    finally:
        rmq.set_plan_table([])
