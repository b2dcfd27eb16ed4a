"""The comparison system ST-RMQ_CON (Section 2) re-created on the GPU
(path "st_con"): every answer against the oracle over the value and query
families, with duplicate, point and invalid queries, ragged sizes, batches on
both sides of the sort's tile-size and remap-window switches, and against
the oracle one query at a time at n = 1e8; plus its failure report when the
endpoint sort gives up (forced from the host)."""
import numpy as np
import pytest
import torch

import paper_1706_06940_amd as rmq
import workloads as W
from tests._gpu import arrays, dev, host, need_gpu, query_sets, reference, say

pytestmark = pytest.mark.gpu


def run(A, L, R, d, bad=None):
    return host(rmq.query_batch(dev(A, d), dev(L, d), dev(R, d), path="st_con", bad_count=bad))


@pytest.mark.parametrize("n", [1, 2, 3, 1023, 1024, 1025, 70_001])
def test_families(orc, n):
    d = need_gpu()
    for name, A in arrays(n, n + 5):
        for qname, L, R in query_sets(n, 256, 3000, n + 7):
            say("st_con", n, name, qname, len(L))
            exp = reference(orc, A, L, R)
            got = run(A, L, R, d)
            wrong = np.nonzero(got != exp)[0]
            assert wrong.size == 0, (name, qname, wrong[:4], got[wrong[:4]], exp[wrong[:4]])


def test_every_range_of_tiny_arrays(orc):
    d = need_gpu()
    for n in (1, 5, 17, 40):
        A = W.uniform_int31(n, 100 + n) % 7  # many ties
        A = A.astype(np.int32)
        l, r = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        m = l <= r
        L, R = l[m].astype(np.int32), r[m].astype(np.int32)
        say("st_con_all_ranges", n, len(L))
        assert np.array_equal(run(A, L, R, d), reference(orc, A, L, R))


@pytest.mark.parametrize("n,q", [(100_003, 1), (100_003, 49_999), (100_003, 50_001),
                                 (1_000_003, 200_001), (3_000_017, 600_000)])
def test_batches_invalid_and_duplicates(orc, n, q):
    d = need_gpu()
    say("st_con_batch", n, q)
    A = W.uniform_int31(n, n + q)
    L, R = W.uniform_queries(n, q, n + q + 1)
    rng = np.random.default_rng(q)
    # repeated queries and shared endpoints, and five invalid ones
    if q > 10:
        rep = rng.choice(q, q // 10, replace=False)
        half = rep[: len(rep) // 2]
        L[half], R[half] = L[0], R[0]                    # the same query again
        rest = rep[len(rep) // 2:]
        R[rest] = np.maximum(R[rest], L[0])              # a shared left end
        L[rest] = L[0]
        bad_i = rng.choice(q, 5, replace=False)
        L[bad_i[0]], R[bad_i[0]] = 5, 4
        L[bad_i[1]], R[bad_i[1]] = -1, 3
        L[bad_i[2]], R[bad_i[2]] = 0, n
        L[bad_i[3]], R[bad_i[3]] = n - 1, n - 1
        L[bad_i[4]], R[bad_i[4]] = 0, n - 1
    bad = torch.zeros(1, dtype=torch.int64, device=d)
    exp = reference(orc, A, L, R)
    got = run(A, L, R, d, bad)
    wrong = np.nonzero(got != exp)[0]
    assert wrong.size == 0, (wrong[:4], L[wrong[:4]], R[wrong[:4]], got[wrong[:4]], exp[wrong[:4]])
    assert int(host(bad)[0]) == (3 if q > 10 else 0)


@pytest.mark.timeout(600)
def test_full_size_sampled(orc):
    """n = 1e8, q = 1e6 (the sort's window remap, a 4e6-entry A_Q and a
    22-level table): sampled answers against the oracle's scan, every answer
    against the contracted method's."""
    d = need_gpu()
    n, q = 100_000_000, 1_000_000
    say("st_con_full_size", n, q)
    A = W.uniform_int31(n, 1)
    L, R = W.uniform_queries(n, q, 2)
    At, Lt, Rt = dev(A, d), dev(L, d), dev(R, d)
    got = host(rmq.query_batch(At, Lt, Rt, path="st_con"))
    con = host(rmq.query_batch(At, Lt, Rt, path="contracted"))
    assert np.array_equal(got, con)
    idx = np.random.default_rng(3).choice(q, 64, replace=False)
    assert np.array_equal(got[idx], orc.rmq_scan(A, L[idx], R[idx]))


def test_sort_failure_reported(orc):
    d = need_gpu()
    n, q = 100_003, 20_000
    say("st_con_sort_abort", n, q)
    A = W.uniform_int31(n, 9)
    L, R = W.uniform_queries(n, q, 10)
    bad = torch.zeros(1, dtype=torch.int64, device=d)
    rmq.test_sort_abort(True)
    try:
        got = run(A, L, R, d, bad)
    finally:
        rmq.test_sort_abort(False)
    assert np.all(got == -1)
    assert int(host(bad)[0]) == q
    assert np.array_equal(run(A, L, R, d), reference(orc, A, L, R))


def test_options_refused():
    d = need_gpu()
    say("st_con_options")
    A = dev(W.uniform_int31(1000, 3), d)
    L, R = (dev(x, d) for x in W.uniform_queries(1000, 10, 4))
    for kw in (dict(block_size=256), dict(sub_block_size=64), dict(arity_log2=2)):
        with pytest.raises(rmq.RMQError):
            rmq.query_batch(A, L, R, path="st_con", **kw)
