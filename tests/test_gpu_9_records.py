"""Query records beside the doubling table (one block level): each block's
minimum paired with the window of 2^t blocks that starts just after it
(forward record) or ends just before it (backward record), for every level
t, so that a query reads each end block and the window beside it in one
16-byte load.  Answers with records, without them and from the oracle
agree bit for bit on every path that reads them, including the edge of the
record rule (8 MiB)."""
import numpy as np
import pytest
import torch

import paper_1706_06940_amd as rmq
import workloads as W
from tests._gpu import arrays, dev, host, need_gpu, query_sets, reference, say

pytestmark = pytest.mark.gpu


def both(At, Lt, Rt, **kw):
    a = host(rmq.query_batch(At, Lt, Rt, **kw))
    b = host(rmq.query_batch(At, Lt, Rt, records=False, **kw))
    return a, b


@pytest.mark.parametrize("n,k", [(1, 16), (33, 16), (48, 16), (64, 16), (1000, 16), (4099, 64),
                                 (262_144, 16), (279_616, 16), (279_617, 16),
                                 (1 << 20, 16), (4_194_400, 64), (1_000_003, 1 << 20)])
def test_full_families(orc, n, k):
    """nb from 1 to 65,538 blocks: records up to 17,476 blocks (15 levels,
    8 MiB), none above."""
    d = need_gpu()
    q = 3000 if n > 64 else 300
    for aname, A in list(arrays(n, n + k))[:5]:
        At = dev(A, d)
        for qname, L, R in query_sets(n, k, q, n + 3 * k):
            say("records_full", n, k, aname, qname)
            exp = reference(orc, A, L, R)
            a, b = both(At, dev(L, d), dev(R, d), path="full", block_size=k)
            assert np.array_equal(a, exp) and np.array_equal(b, exp), (n, k, aname, qname)


@pytest.mark.parametrize("n,q,k", [(10_007, 1, 16), (10_007, 5000, 16), (1_000_003, 300_000, 16),
                                   (1_000_003, 300_000, 256), (3_000_017, 1_000_000, 32)])
def test_contracted(orc, n, q, k):
    d = need_gpu()
    A = W.uniform_int31(n, q + k)
    for qname, L, R in query_sets(n, k, q, q + 7):
        say("records_contracted", n, q, k, qname)
        exp = reference(orc, A, L, R)
        a, b = both(dev(A, d), dev(L, d), dev(R, d), path="contracted", block_size=k)
        assert np.array_equal(a, exp) and np.array_equal(b, exp), (n, q, k, qname)


def test_all_ranges(orc):
    d = need_gpu()
    for n in (1, 2, 17, 100, 700):
        for aname, A in list(arrays(n, n + 1))[:4]:
            L, R = np.triu_indices(n)
            L, R = L.astype(np.int32), R.astype(np.int32)
            exp = orc.rmq_scan(A, L, R)
            At, Lt, Rt = dev(A, d), dev(L, d), dev(R, d)
            say("records_all_ranges", n, aname)
            for kw in (dict(path="full", block_size=16), dict(path="contracted", block_size=16),
                       dict(path="full", block_size=64, sub_block_size=16)):
                a, b = both(At, Lt, Rt, **kw)
                assert np.array_equal(a, exp) and np.array_equal(b, exp), (n, aname, kw)


def test_index_two_level_lca_and_serving_agree(orc):
    d = need_gpu()
    say("records_index")
    n = 3_000_017
    A = W.uniform_int31(n, 97)
    At = dev(A, d)
    L, R = W.skewed_queries(n, 100_000, 98)
    exp = reference(orc, A, L, R)
    Lt, Rt = dev(L, d), dev(R, d)
    for kw in (dict(block_size=1024), dict(block_size=4096, sub_block_size=256),
               dict(block_size=256)):
        on, off = rmq.Index(At, records=True, **kw), rmq.Index(At, records=False, **kw)
        if "sub_block_size" in kw:
            assert on.bytes == off.bytes  # no records under two block levels
        else:
            assert on.bytes > off.bytes  # records kept up to 17,476 blocks (here <= 11,719)
        assert np.array_equal(host(on.query(Lt, Rt)), exp), kw
        assert np.array_equal(host(off.query(Lt, Rt)), exp), kw
        assert torch.equal(on.table(), off.table())
    N = 100_003
    parent = W.random_recursive_tree(N, 99)
    depth, node, first = orc.euler_tour(parent)
    u = W.uniform_index(N, 20_000, 99, 1).astype(np.int32)
    v = W.uniform_index(N, 20_000, 99, 2).astype(np.int32)
    lo = np.minimum(first[u], first[v]).astype(np.int32)
    hi = np.maximum(first[u], first[v]).astype(np.int32)
    lca = node[orc.rmq_sparse_table(depth, lo, hi, 32)]
    for rec in (True, False):
        h = rmq.LCA(dev(parent, d), block_size=256, records=rec)
        got = host(h.query(dev(u, d), dev(v, d)))
        h.free()
        assert np.array_equal(got, lca), rec
