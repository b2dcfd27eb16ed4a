"""Whole batches through the C ABI, both methods, bit-exact against the oracle
(leftmost minimum; -1 for invalid queries)."""
import numpy as np
import pytest
import torch

import paper_1706_06940_amd as rmq
import workloads as W
from tests._gpu import arrays, dev, host, need_gpu, query_sets, reference, say

pytestmark = pytest.mark.gpu

PATHS = ["full", "contracted"]


def run(A_t, L, R, path, k, d, **kw):
    return host(rmq.query_batch(A_t, dev(L, d), dev(R, d), path=path, block_size=k, **kw))


@pytest.mark.parametrize("path,k", [("full", k) for k in (16, 64, 256, 1024, 4096, 16384, 65536)] +
                         [("contracted", k) for k in (16, 128, 512, 4096)] + [("auto", 0)])
def test_small_config(orc, path, k):
    """n = 2^20 uniform int31 values, 1024 uniform queries (the small configuration)."""
    d = need_gpu()
    say("small_config", path, k)
    n, q = 1 << 20, 1024
    seed = W.BASE_SEED + 0
    A = W.uniform_int31(n, seed)
    L, R = W.uniform_queries(n, q, seed)
    exp = orc.rmq_scan(A, L, R)
    got = run(dev(A, d), L, R, path, k, d)
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n,k", [(1, 16), (2, 16), (3, 16), (17, 16), (255, 64), (257, 256),
                                 (1023, 1024), (1025, 256), (4099, 16), (100_003, 1024),
                                 (1_000_003, 4096), (65_536, 65_536), (70_000, 131_072)])
def test_families(orc, path, n, k):
    d = need_gpu()
    q = 3000 if n > 64 else 200
    for aname, A in arrays(n, n + k):
        At = dev(A, d)
        for qname, L, R in query_sets(n, k, q, n * 13 + k):
            say(path, n, k, aname, qname)
            exp = reference(orc, A, L, R)
            got = run(At, L, R, path, k, d)
            bad = np.nonzero(got != exp)[0]
            assert bad.size == 0, (aname, qname, L[bad[:4]], R[bad[:4]], got[bad[:4]], exp[bad[:4]])


@pytest.mark.parametrize("path", PATHS)
def test_all_ranges_tiny(orc, path):
    d = need_gpu()
    for n in (1, 2, 5, 16, 17, 40, 64):
        for aname, A in arrays(n, n):
            L, R = np.triu_indices(n)
            L, R = L.astype(np.int32), R.astype(np.int32)
            say("all_ranges", path, n, aname)
            exp = orc.rmq_scan(A, L, R)
            for k in (16, 32):
                assert np.array_equal(run(dev(A, d), L, R, path, k, d), exp), (n, aname, k)


@pytest.mark.parametrize("path", PATHS)
def test_invalid_queries_and_bad_count(orc, path):
    d = need_gpu()
    say("invalid", path)
    n = 10_000
    A = W.uniform_int31(n, 77)
    L, R = W.uniform_queries(n, 500, 78)
    L[::7] = R[::7] + 1          # reversed
    L[3] = -5
    R[5] = n
    R[6] = n + 100
    L[8], R[8] = -1, -1
    L[9], R[9] = np.iinfo(np.int32).max, np.iinfo(np.int32).max
    bad = torch.zeros(1, dtype=torch.int64, device=d)
    got = run(dev(A, d), L, R, path, 256, d, bad_count=bad)
    exp = orc.rmq_scan(A, L, R)
    assert np.array_equal(got, exp)
    assert int(host(bad)[0]) == int((exp < 0).sum())


@pytest.mark.parametrize("path", PATHS)
def test_empty_batch(path):
    d = need_gpu()
    say("empty", path)
    A = dev(W.uniform_int31(1000, 1), d)
    e = torch.empty(0, dtype=torch.int32, device=d)
    out = rmq.query_batch(A, e, e, path=path)
    assert out.numel() == 0


@pytest.mark.parametrize("path", PATHS)
def test_lca_euler_tour(orc, path):
    """Section 1: LCA via RMQ over Euler-tour depths (massive ties, +-1 steps)."""
    d = need_gpu()
    from tests._pins import naive_lca, node_depths
    for N, seed in ((1, 1), (1000, 2), (200_000, 3)):
        say("lca", path, N)
        parent = W.random_recursive_tree(N, seed)
        depth, node, first = orc.euler_tour(parent)
        u, v, L, R = W.lca_queries(first, 4000, seed)
        got = run(dev(depth, d), L, R, path, 256, d)
        assert np.array_equal(got, orc.rmq_scan(depth, L, R))
        dn = node_depths(parent)
        for a, b, o in list(zip(u, v, got))[:500]:
            assert node[o] == naive_lca(parent, dn, int(a), int(b))


def test_paths_and_block_sizes_agree(orc):
    """Metamorphic: the answer depends on neither k nor the method."""
    d = need_gpu()
    say("metamorphic")
    n, q = 300_007, 20_000
    A = np.random.default_rng(5).integers(0, 1000, n).astype(np.int32)
    L, R = W.uniform_queries(n, q, 6)
    At = dev(A, d)
    base = run(At, L, R, "full", 1024, d)
    assert np.array_equal(base, reference(orc, A, L, R))
    for path, ks in (("full", (16, 256, 4096, 1 << 16, 1 << 20)), ("contracted", (16, 512, 8192))):
        for k in ks:
            assert np.array_equal(run(At, L, R, path, k, d), base), (path, k)
    perm = W.permutation(q, 7, 1)
    assert np.array_equal(run(At, L[perm], R[perm], "full", 1024, d), base[perm])


def test_resident_index(orc):
    d = need_gpu()
    say("index")
    n = 2_000_003
    A = W.uniform_int31(n, 91)
    At = dev(A, d)
    idx = rmq.Index(At, block_size=2048)
    nb = -(-n // 2048)
    # the table (Table 2's footprint), then the query records on a 256-byte boundary
    assert rmq.query_record_bytes(nb) > 0
    assert idx.bytes == -(-rmq.index_bytes(n, 2048) // 256) * 256 + rmq.query_record_bytes(nb)
    assert rmq.Index(At, block_size=2048, records=False).bytes == rmq.index_bytes(n, 2048)
    for seed in range(3):
        L, R = W.uniform_queries(n, 10_000, 100 + seed)
        got = host(idx.query(dev(L, d), dev(R, d)))
        assert np.array_equal(got, reference(orc, A, L, R))
    st = host(idx.table()).view(np.uint64)
    blk = orc.block_argmin(A, 2048)
    assert np.array_equal((st[0] & 0xFFFFFFFF).astype(np.int64), blk.astype(np.int64))
    idx.free()


def test_workspace_and_timer(orc):
    d = need_gpu()
    say("workspace_timer")
    n, q = 1 << 20, 50_000
    A = W.uniform_int31(n, 3)
    L, R = W.uniform_queries(n, q, 4)
    exp = reference(orc, A, L, R)
    for path, k in (("full", 1024), ("contracted", 512)):
        wsb = rmq.workspace_bytes(n, q, path, k)
        ws = torch.empty(wsb, dtype=torch.uint8, device=d)
        t = rmq.Timer()
        stats = torch.zeros(2, dtype=torch.int64, device=d)
        got = run(dev(A, d), L, R, path, k, d, workspace=ws, timer=t, stats=stats)
        assert np.array_equal(got, exp)
        stages, total = t.read()
        assert total > 0 and all(s >= 0 for s in stages)
        assert (stages[0] > 0) == (path == "contracted")
        s = host(stats)
        assert 0 <= s[0] <= 2 * q and s[1] <= s[0] * k
        with pytest.raises(rmq.RMQError):
            small = torch.empty(max(wsb // 2, 256), dtype=torch.uint8, device=d)
            rmq.query_batch(dev(A, d), dev(L, d), dev(R, d), path=path, block_size=k,
                            workspace=small)


# The contracted path's remap for long endpoint lists goes through LR windows
# built in LDS (2q >= 2^20, up to 6144 tiles of 8192 items); the window is
# the largest of 2^12 .. 2^15 tags that gives 256 windows, so it grows at
# 2q = 2^21, 2^22 and 2^23.  Shorter lists write LR with scattered stores.
# Both sides of the switch and of each window change, a ragged last window,
# the single-pass sort (n <= 256: the first pass is also the last), and both
# sides of the longest list the windows take.
@pytest.mark.parametrize("n,q", [(3_000_017, 524_287), (3_000_017, 524_288),
                                 (3_000_017, 1_048_575), (3_000_017, 1_048_576),
                                 (3_000_017, 2_097_151), (3_000_017, 2_097_152),
                                 (10_000_019, 2_100_007), (200, 2_200_001),
                                 (10_000_019, 4_194_303), (10_000_019, 4_194_304),
                                 (50_000_017, 12_000_007),
                                 # 6144 tiles of 8192 items exactly, and one item more
                                 (30_000_001, 25_165_824), (30_000_001, 25_165_825)])
def test_contracted_remap_windows(orc, n, q):
    d = need_gpu()
    say("remap_windows", n, q)
    A = W.uniform_int31(n, n + q)
    L, R = W.uniform_queries(n, q, n + q, 5)
    L[:3] = R[:3] = n // 2          # repeated single-point queries
    L[3], R[3] = n - 1, 0           # an invalid query: sorts as position 0
    L[4], R[4] = 0, n - 1
    exp = reference(orc, A, L, R)  # -1 for the invalid one
    got = host(rmq.query_batch(dev(A, d), dev(L, d), dev(R, d), path="contracted"))
    assert np.array_equal(got, exp), (n, q)
