"""The block table over powers of l instead of 2 (Section 3.1's
generalisation, l = 2^a for a in 2..5): level i holds the minima of l^i
consecutive blocks and a query reads at most l of them.  Every answer is
bit-exact against the oracle, on both methods, with two block levels, on the
resident index and under the LCA front-end; the stored levels equal the
doubling table's levels a, 2a, 3a, ... (same spans, same truncation at the
end of the table)."""
import numpy as np
import pytest
import torch

import paper_1706_06940_amd as rmq
import workloads as W
from tests._gpu import arrays, dev, host, need_gpu, query_sets, reference, say

pytestmark = pytest.mark.gpu


def natural_order(table, a):
    """Level i >= 1 of the table over powers of l = 2^a is stored by residue
    class mod s = l^i (block b at r * (nb // s) + min(r, nb % s) + b // s,
    r = b % s); return the levels in block order."""
    nb = table.shape[1]
    b = np.arange(nb, dtype=np.int64)
    out = table.copy()
    for i in range(1, table.shape[0]):
        s = 1 << (i * a)
        r = b % s
        addr = r * (nb // s) + np.minimum(r, nb % s) + b // s
        assert np.array_equal(np.sort(addr), b)  # a permutation of [0, nb)
        out[i] = table[i][addr]
    return out


@pytest.mark.parametrize("n,k,a", [(1, 16, 2), (100, 16, 2), (1025, 16, 3), (4099, 16, 5),
                                   (100_003, 16, 4), (100_003, 64, 2), (1_000_003, 32, 4),
                                   (1_000_003, 1024, 3), (3_000_017, 256, 5)])
def test_full_families(orc, n, k, a):
    d = need_gpu()
    q = 3000 if n > 64 else 200
    for aname, A in arrays(n, n + k + a):
        At = dev(A, d)
        for qname, L, R in query_sets(n, k, q, n * 3 + k + a):
            say("lary_full", n, k, a, aname, qname)
            exp = reference(orc, A, L, R)
            got = host(rmq.query_batch(At, dev(L, d), dev(R, d), path="full", block_size=k,
                                       arity_log2=a))
            bad = np.nonzero(got != exp)[0]
            assert bad.size == 0, (aname, qname, L[bad[:4]], R[bad[:4]], got[bad[:4]], exp[bad[:4]])


@pytest.mark.parametrize("n,q,k,a", [(10_007, 1, 16, 2), (10_007, 3000, 16, 4),
                                     (1_000_003, 100_000, 16, 5), (1_000_003, 100_000, 64, 3),
                                     (100_003, 50_000, 32, 2)])
def test_contracted(orc, n, q, k, a):
    d = need_gpu()
    A = W.uniform_int31(n, n + q)
    for qname, L, R in query_sets(n, k, q, q + a):
        say("lary_contracted", n, q, k, a, qname)
        exp = reference(orc, A, L, R)
        got = host(rmq.query_batch(dev(A, d), dev(L, d), dev(R, d), path="contracted",
                                   block_size=k, arity_log2=a))
        bad = np.nonzero(got != exp)[0]
        assert bad.size == 0, (qname, L[bad[:4]], R[bad[:4]], got[bad[:4]], exp[bad[:4]])


def test_all_ranges(orc):
    """Every range of arrays of up to 38 blocks of 16: every count of whole
    l^i-windows and every remainder."""
    d = need_gpu()
    for n in (1, 17, 70, 300, 600):
        for aname, A in list(arrays(n, n))[:4]:
            L, R = np.triu_indices(n)
            L, R = L.astype(np.int32), R.astype(np.int32)
            exp = orc.rmq_scan(A, L, R)
            At, Lt, Rt = dev(A, d), dev(L, d), dev(R, d)
            for a in (2, 3, 4, 5):
                say("lary_all_ranges", n, aname, a)
                got = host(rmq.query_batch(At, Lt, Rt, path="full", block_size=16, arity_log2=a))
                assert np.array_equal(got, exp), (n, aname, a)
                if n >= 300:
                    got = host(rmq.query_batch(At, Lt, Rt, path="full", block_size=64,
                                               sub_block_size=16, arity_log2=a))
                    assert np.array_equal(got, exp), (n, aname, a, "two levels")


@pytest.mark.parametrize("a", [2, 3, 4, 5])
def test_index_levels_are_doubling_levels(orc, a):
    d = need_gpu()
    n, k = 3_000_017, 32
    say("lary_index", a)
    A = W.uniform_int31(n, 71 + a)
    At = dev(A, d)
    idx = rmq.Index(At, k, arity_log2=a)
    nb = -(-n // k)
    assert idx.num_blocks == nb and idx.levels == rmq.table_levels(nb, a)
    assert idx.bytes == 8 * nb * idx.levels
    two = rmq.Index(At, k)
    t_l = natural_order(host(idx.table()), a)
    assert np.array_equal(t_l, host(two.table())[::a][:idx.levels])
    # against the oracle's block minima and its doubling table's levels a, 2a, ...
    blk = orc.block_argmin(A, k)
    ost = orc.block_sparse_table(A, blk, rmq.table_levels(nb))
    pos = (t_l & 0xFFFFFFFF).astype(np.int32)
    assert np.array_equal(pos[0], blk) and np.array_equal(pos, ost[::a][:idx.levels])
    for seed in (72, 73):
        L, R = W.skewed_queries(n, 50_000, seed)
        exp = reference(orc, A, L, R)
        assert np.array_equal(host(idx.query(dev(L, d), dev(R, d))), exp)
    idx2 = rmq.Index(At, 1024, sub_block_size=32, arity_log2=a)
    L, R = W.uniform_queries(n, 50_000, 74)
    assert np.array_equal(host(idx2.query(dev(L, d), dev(R, d))), reference(orc, A, L, R))


def test_lca_with_lary_table(orc):
    d = need_gpu()
    say("lary_lca")
    N = 200_003
    parent = W.random_recursive_tree(N, 75)
    depth, node, first = orc.euler_tour(parent)
    u = W.uniform_index(N, 20_000, 75, 1).astype(np.int32)
    v = W.uniform_index(N, 20_000, 75, 2).astype(np.int32)
    lo = np.minimum(first[u], first[v]).astype(np.int32)
    hi = np.maximum(first[u], first[v]).astype(np.int32)
    exp = node[orc.rmq_sparse_table(depth, lo, hi, 32)]
    for k, k1, a in ((32, 0, 4), (512, 32, 3)):
        h = rmq.LCA(dev(parent, d), block_size=k, sub_block_size=k1, arity_log2=a)
        got = host(h.query(dev(u, d), dev(v, d)))
        h.free()
        assert np.array_equal(got, exp), (k, k1, a)


def test_invalid_arity():
    d = need_gpu()
    say("lary_invalid")
    A = torch.zeros(1000, dtype=torch.int32, device=d)
    L = torch.zeros(4, dtype=torch.int32, device=d)
    for a in (-1, 6, 40):
        with pytest.raises(rmq.RMQError):
            rmq.query_batch(A, L, L, block_size=16, arity_log2=a)
        with pytest.raises(rmq.RMQError):
            rmq.Index(A, 256, arity_log2=a)
