"""Three block levels (Section 3.3 with h = 3, plain method): every answer
against the oracle over the value and query families and several (k, k1, k2),
ragged sizes, invalid queries, a batch large enough for the table in LDS,
the partial-scan counter, and sampled answers at n = 1e9 with skewed
queries against the two-level form."""
import numpy as np
import pytest
import torch

import paper_1706_06940_amd as rmq
import workloads as W
from tests._gpu import arrays, dev, host, need_gpu, query_sets, reference, say

pytestmark = pytest.mark.gpu

PLANS = [(256, 64, 16), (1024, 256, 32), (4096, 512, 64), (65536, 1024, 64), (16384, 4096, 2048)]


@pytest.mark.parametrize("k,k1,k2", PLANS)
@pytest.mark.parametrize("n", [1, 17, 1025, 70_001, 262_147])
def test_families(orc, n, k, k1, k2):
    d = need_gpu()
    for name, A in arrays(n, n + k2):
        At = dev(A, d)
        for qname, L, R in query_sets(n, k, 2000, n + k1):
            say("three_levels", n, k, k1, k2, name, qname)
            exp = reference(orc, A, L, R)
            got = host(rmq.query_batch(At, dev(L, d), dev(R, d), path="full", block_size=k,
                                       sub_block_size=k1, sub_block_size2=k2))
            wrong = np.nonzero(got != exp)[0]
            assert wrong.size == 0, (name, qname, wrong[:4], got[wrong[:4]], exp[wrong[:4]])


@pytest.mark.timeout(600)
@pytest.mark.parametrize("q", [100_001, 2_300_001])
def test_large_batches_and_counters(orc, q):
    """The second batch takes the table in LDS (2^21 queries or more)."""
    d = need_gpu()
    n, k, k1, k2 = 10_000_019, 65536, 1024, 64
    say("three_levels_large", n, q)
    A = W.uniform_int31(n, 5)
    L, R = W.uniform_queries(n, q, 6)
    sl, sr = W.short_queries(n, q // 4, 7, 1, 2048)
    L[: q // 4], R[: q // 4] = sl, sr
    L[1], R[1] = 7, 3  # invalid
    At, Lt, Rt = dev(A, d), dev(L, d), dev(R, d)
    bad = torch.zeros(1, dtype=torch.int64, device=d)
    stats3 = torch.zeros(2, dtype=torch.int64, device=d)
    stats2 = torch.zeros(2, dtype=torch.int64, device=d)
    got = host(rmq.query_batch(At, Lt, Rt, path="full", block_size=k, sub_block_size=k1,
                               sub_block_size2=k2, bad_count=bad, stats=stats3))
    two = host(rmq.query_batch(At, Lt, Rt, path="full", block_size=k, sub_block_size=k1,
                               stats=stats2))
    exp = reference(orc, A, L, R)
    assert np.array_equal(got, exp) and np.array_equal(two, exp)
    assert int(host(bad)[0]) == 1
    s3, s2 = host(stats3), host(stats2)
    # the same pieces are scanned; the third level reads fewer entries
    assert s3[0] >= s2[0] > 0 and s3[1] < s2[1]


@pytest.mark.timeout(900)
def test_n1e9_skewed_sampled(orc):
    d = need_gpu()
    n, q = 1_000_000_000, 2_000_000
    say("three_levels_n1e9", n, q)
    At = W.uniform_int31_torch(n, 11, 0, device=d)
    L, R = W.uniform_queries(n, q, 12)
    sl, sr = W.short_queries(n, q // 2, 13, 1, 1024)
    L[: q // 2], R[: q // 2] = sl, sr
    Lt, Rt = dev(L, d), dev(R, d)
    got = host(rmq.query_batch(At, Lt, Rt, path="full", block_size=65536, sub_block_size=1024,
                               sub_block_size2=64))
    two = host(rmq.query_batch(At, Lt, Rt, path="full", block_size=16384, sub_block_size=256))
    assert np.array_equal(got, two)
    idx = np.random.default_rng(14).choice(q // 2, 200, replace=False)  # short ranges
    A_h = At.cpu().numpy()
    assert np.array_equal(got[idx], orc.rmq_scan(A_h, L[idx], R[idx]))
    del At, A_h
    torch.cuda.empty_cache()
