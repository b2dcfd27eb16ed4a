"""The device sort's failure report, forced from the host.

The radix sort of the contracted method waits for earlier tiles with a
bounded wait and, should one run out, gives up on its order through a device
word.  rmq_test_sort_abort makes every later sort start with that word set,
so each wait ends at once and every kernel exits normally; the calls must
then report the failure as rmq.h documents it, never wrong answers.  Nothing
here spins a wait to its limit."""
import numpy as np
import pytest
import torch

import paper_1706_06940_amd as rmq
import workloads as W
from tests._gpu import dev, host, need_gpu, reference, say

pytestmark = pytest.mark.gpu


@pytest.fixture
def forced_abort():
    rmq.test_sort_abort(True)
    try:
        yield
    finally:
        rmq.test_sort_abort(False)


# list lengths 2q on both sides of the tile-size switches (1e5, 4e5 items)
# and of the remap-window path (2q >= 2^20), and a batch of 2^22 queries or
# more, whose default table over A_Q the query kernel keeps in LDS
@pytest.mark.parametrize("n,q", [(1000, 1), (100_003, 20_000), (1_000_003, 150_000),
                                 (3_000_017, 1_000_000), (10_000_019, 2_200_000),
                                 (10_000_019, 4_300_000)])
def test_contracted_batch_reports_every_query(orc, forced_abort, n, q):
    d = need_gpu()
    say("sort_abort_contracted", n, q)
    A = W.uniform_int31(n, n)
    L, R = W.uniform_queries(n, q, n + 1)
    At, Lt, Rt = dev(A, d), dev(L, d), dev(R, d)
    bad = torch.zeros(1, dtype=torch.int64, device=d)
    got = host(rmq.query_batch(At, Lt, Rt, path="contracted", bad_count=bad))
    assert np.all(got == -1)
    assert int(host(bad)[0]) == q
    # the plain method sorts nothing and is unaffected
    full = host(rmq.query_batch(At, Lt, Rt, path="full"))
    assert np.array_equal(full, reference(orc, A, L, R))


def test_stages_and_lca_report(forced_abort):
    d = need_gpu()
    say("sort_abort_stages")
    n, q = 50_000, 3000
    A = W.uniform_int31(n, 3)
    L, R = W.uniform_queries(n, q, 4)
    Lt, Rt = dev(L, d), dev(R, d)
    pos, tag = rmq.sort_endpoints(Lt, Rt, n)
    assert np.all(host(pos) == -1) and np.all(host(tag) == -1)
    # the stand-alone remap buckets the tags with one more sort sweep
    pos_ok = dev(np.sort(np.concatenate([L, R])).astype(np.int32), d)
    tag_in = dev(np.arange(2 * q, dtype=np.int32), d)
    Lc, Rc, _ = rmq.contract(dev(A, d), pos_ok, tag_in)
    assert np.all(host(Lc) == -1) and np.all(host(Rc) == -1)
    parent = W.random_recursive_tree(10_000, 5)
    with pytest.raises(rmq.RMQError) as e:
        rmq.LCA(dev(parent, d))
    assert e.value.status == 3


def test_sorting_recovers_after_the_forced_report(orc):
    d = need_gpu()
    say("sort_abort_recovers")
    n, q = 200_003, 50_000
    A = W.uniform_int31(n, 8)
    L, R = W.uniform_queries(n, q, 9)
    At, Lt, Rt = dev(A, d), dev(L, d), dev(R, d)
    rmq.test_sort_abort(True)
    try:
        assert np.all(host(rmq.query_batch(At, Lt, Rt, path="contracted")) == -1)
    finally:
        rmq.test_sort_abort(False)
    bad = torch.zeros(1, dtype=torch.int64, device=d)
    got = host(rmq.query_batch(At, Lt, Rt, path="contracted", bad_count=bad))
    assert np.array_equal(got, reference(orc, A, L, R))
    assert int(host(bad)[0]) == 0
