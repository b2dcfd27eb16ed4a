"""Parity at the largest configurations, checked on every output:

* n = 1e9 int32 uniform values (4 GB), q = 1e7 queries, half short (length
  uniform in [1, 1024]) and half uniform long, both methods and the plain
  method with two block levels (Section 3.3);
* Euler-tour depth array of a random recursive tree with 5e8 nodes
  (999,999,999 steps, +-1), 1e7 LCA queries: the answer's tour node is the
  LCA found by climbing parent pointers, and equals the oracle's answer; the
  device LCA front-end builds the same tour as the oracle and gives the same
  LCAs;
* n = 1e8, q = 1e7 uniform (the benchmark's largest batch), both methods.

The oracle here is its Sparse Table over 32-element blocks (pinned against
brute force and the linear scan in the CPU tests).  Inputs are drawn on the
host; the device copies of the big arrays are drawn in HBM by the torch form
of the same generator, checked equal on a sample first.
"""
import time

import numpy as np
import pytest
import torch

import paper_1706_06940_amd as rmq
import workloads as W
from tests._gpu import dev, need_gpu, say

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def log(*a):
    print(f"[scale {time.strftime('%H:%M:%S')}]", *a, flush=True)


def compare_all(orc, A_h, L, R, got, what):
    exp = orc.rmq_sparse_table(A_h, L, R, 32)
    bad = np.nonzero(got != exp)[0]
    assert bad.size == 0, (what, bad.size, L[bad[:3]], R[bad[:3]], got[bad[:3]], exp[bad[:3]])


def test_c3_billion_skewed(orc):
    d = need_gpu()
    say("c3_billion_skewed")
    n, q, seed = 10 ** 9, 10 ** 7, W.BASE_SEED + 2
    log("drawing A on the host")
    A_h = W.uniform_int31(n, seed)
    log("drawing A in HBM")
    A = W.uniform_int31_torch(n, seed, 0, device=d)
    idx = W.uniform_index(n, 4096, seed, 99)
    assert np.array_equal(A[torch.from_numpy(idx).to(d)].cpu().numpy(), A_h[idx])
    L, R = W.skewed_queries(n, q, seed)
    Lt, Rt = dev(L, d), dev(R, d)
    exp = orc.rmq_sparse_table(A_h, L, R, 32)
    for path, k1 in (("full", 0), ("contracted", 0), ("full", 1024)):
        log("running", path, "two levels" if k1 else "")
        got = rmq.query_batch(A, Lt, Rt, path=path, sub_block_size=k1).cpu().numpy()
        log("checking", path)
        bad = np.nonzero(got != exp)[0]
        assert bad.size == 0, (path, k1, bad.size, L[bad[:3]], R[bad[:3]], got[bad[:3]], exp[bad[:3]])
    log("done")


# Host-heavy: the tree, its tour and the parent climbing take 1-2 minutes of
# CPU time at this size, more on a loaded host; the GPU parts take seconds.
@pytest.mark.timeout(600)
def test_c3_lca_half_billion_nodes(orc):
    d = need_gpu()
    say("c3_lca")
    N, q, seed = 5 * 10 ** 8, 10 ** 7, W.BASE_SEED + 2
    log("tree")
    parent = W.random_recursive_tree(N, seed)
    log("oracle tour")
    # the oracle's tour is both the RMQ input and the device tour's expected value
    exp = orc.euler_tour(parent)
    depth, node, first = exp
    assert depth.shape[0] == 2 * N - 1
    u, v, L, R = W.lca_queries(first, q, seed)
    log("rmq on the gpu")
    got = rmq.query_batch(dev(depth, d), dev(L, d), dev(R, d), path="full").cpu().numpy()
    log("oracle")
    compare_all(orc, depth, L, R, got, "lca")
    log("parent climbing")
    D = np.empty(N, dtype=np.int32)
    D[node] = depth
    a, b = u.astype(np.int64), v.astype(np.int64)
    for _ in range(10 ** 4):
        da, db = D[a], D[b]
        if np.array_equal(da, db):
            break
        m = da > db
        a[m] = parent[a[m]]
        m = db > da
        b[m] = parent[b[m]]
    for _ in range(10 ** 4):
        m = a != b
        if not m.any():
            break
        a[m] = parent[a[m]]
        b[m] = parent[b[m]]
    assert np.array_equal(node[got], a)
    log("device LCA front-end")
    h = rmq.LCA(dev(parent, d))
    got2 = h.query(dev(u, d), dev(v, d)).cpu().numpy()
    assert np.array_equal(got2, a)
    tour = [t.cpu().numpy() for t in h.tour()]
    h.free()
    assert all(np.array_equal(x, y) for x, y in zip(tour, exp))
    log("done")


def test_c2_largest_batch(orc):
    d = need_gpu()
    say("c2_largest_batch")
    n, q, seed = 10 ** 8, 10 ** 7, W.BASE_SEED + 1
    A_h = W.uniform_int31(n, seed)
    L, R = W.uniform_queries(n, q, seed, 77)
    At, Lt, Rt = dev(A_h, d), dev(L, d), dev(R, d)
    for path in ("full", "contracted"):
        log("running", path)
        got = rmq.query_batch(At, Lt, Rt, path=path).cpu().numpy()
        compare_all(orc, A_h, L, R, got, path)
    log("done")
