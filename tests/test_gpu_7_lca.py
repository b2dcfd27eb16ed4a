"""LCA through RMQ (Section 1), built on the device: the Euler tour equals
the oracle's (children in increasing id), and every LCA answer equals the
oracle's tour RMQ and parent climbing."""
import numpy as np
import pytest
import torch

import paper_1706_06940_amd as rmq
import workloads as W
from tests._gpu import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu


def climb_lca(parent, depth, u, v):
    """LCA by climbing parent pointers (node depths given), vectorised over
    the queries."""
    a, b = u.astype(np.int64).copy(), v.astype(np.int64).copy()
    while True:
        m = depth[a] > depth[b]
        if not m.any():
            break
        a[m] = parent[a[m]]
    while True:
        m = depth[b] > depth[a]
        if not m.any():
            break
        b[m] = parent[b[m]]
    while True:
        m = a != b
        if not m.any():
            break
        a[m] = parent[a[m]]
        b[m] = parent[b[m]]
    return a


def trees(rng):
    yield "single", np.array([-1], dtype=np.int32)
    yield "pair", np.array([-1, 0], dtype=np.int32)
    yield "golden", np.array([-1, 0, 1, 1, 2, 4, 5, 0, 5, 5], dtype=np.int32)
    for N in (3, 70, 4097, 20_000):
        yield f"recursive{N}", W.random_recursive_tree(N, N)
    yield "path", np.arange(-1, 4999, dtype=np.int32)
    yield "star", np.r_[-1, np.zeros(3000, dtype=np.int32)].astype(np.int32)
    yield "caterpillar", np.r_[-1, np.arange(0, 999), np.arange(0, 999)].astype(np.int32)
    perm = rng.permutation(6000)                          # relabelled: ids not in tree order
    base = W.random_recursive_tree(6000, 8)
    relab = np.empty(6000, dtype=np.int32)
    relab[perm] = np.where(base < 0, -1, perm[np.maximum(base, 0)])
    yield "relabelled", relab
    rev = np.arange(1, 3001, dtype=np.int32)               # a path with the root last
    rev[-1] = -1
    yield "path_root_last", rev


@pytest.mark.parametrize("k,k1", [(0, 0), (16, 0), (64, 16)])
def test_tour_and_answers(orc, k, k1):
    d = need_gpu()
    rng = np.random.default_rng(41)
    for name, parent in trees(rng):
        N = parent.shape[0]
        say("lca", name, N, k, k1)
        exp = orc.euler_tour(parent)
        assert exp is not None
        h = rmq.LCA(dev(parent, d), block_size=k, sub_block_size=k1)
        depth, node, first = (host(t) for t in h.tour())
        assert np.array_equal(depth, exp[0]) and np.array_equal(node, exp[1])
        assert np.array_equal(first, exp[2])
        q = 2000
        u = rng.integers(0, N, q).astype(np.int32)
        v = rng.integers(0, N, q).astype(np.int32)
        got = host(h.query(dev(u, d), dev(v, d)))
        L = np.minimum(exp[2][u], exp[2][v]).astype(np.int32)
        R = np.maximum(exp[2][u], exp[2][v]).astype(np.int32)
        assert np.array_equal(got, exp[1][orc.rmq_scan(exp[0], L, R)]), name
        node_depth = exp[0][exp[2]]  # depth at each node's first occurrence
        assert np.array_equal(got, climb_lca(parent, node_depth, u, v)), name
        h.free()


def test_large_random_recursive_tree(orc):
    d = need_gpu()
    say("lca_large")
    N, q = 3_000_000, 200_000
    parent = W.random_recursive_tree(N, 77)
    exp = orc.euler_tour(parent)
    h = rmq.LCA(dev(parent, d))
    depth, node, first = (host(t) for t in h.tour())
    assert np.array_equal(depth, exp[0]) and np.array_equal(node, exp[1])
    assert np.array_equal(first, exp[2])
    u, v, L, R = W.lca_queries(exp[2], q, 78)
    got = host(h.query(dev(u, d), dev(v, d)))
    assert np.array_equal(got, exp[1][orc.rmq_sparse_table(exp[0], L, R, 32)])


def test_invalid_trees_and_nodes(orc):
    d = need_gpu()
    say("lca_invalid")
    for bad in ([-1, -1, 0], [0], [-1, 5], [-1, 0, 3, 2], [1, 0, -1], [-1, 0, 0, 4, 3]):
        with pytest.raises(rmq.RMQError):
            rmq.LCA(dev(np.array(bad, dtype=np.int32), d))
    parent = W.random_recursive_tree(100, 5)
    h = rmq.LCA(dev(parent, d))
    u = np.array([0, -1, 5, 100, 7], dtype=np.int32)
    v = np.array([3, 2, 2**31 - 1, 0, 7], dtype=np.int32)
    bad = torch.zeros(1, dtype=torch.int64, device=d)
    got = host(h.query(dev(u, d), dev(v, d), bad_count=bad))
    assert got[1] == -1 and got[2] == -1 and got[3] == -1 and got[4] == 7
    assert int(host(bad)[0]) == 3
    exp = orc.euler_tour(parent)
    assert got[0] == exp[1][orc.rmq_scan(exp[0], np.array([min(exp[2][0], exp[2][3])], np.int32),
                                         np.array([max(exp[2][0], exp[2][3])], np.int32))[0]]
