"""Serving: resident arrays, coalesced batches over several streams.  Every
answer is checked against the oracle, and a request's answer is the same
when it is served alone and when it is served inside a mix."""
import numpy as np
import pytest
import torch

import paper_1706_06940_amd as rmq
import workloads as W
from paper_1706_06940_amd import serving
from tests._gpu import dev, need_gpu, reference, say

pytestmark = pytest.mark.gpu


def arrays_for(count, seed, lo=2e3, hi=3e5):
    ns = W.loguniform_ints(count, lo, hi, seed, 1)
    return [W.uniform_int31(int(n), seed + j) if j % 2 else
            np.random.default_rng(j).integers(0, 9, int(n)).astype(np.int32)
            for j, n in enumerate(ns)]


def check(orc, arrays, reqs):
    for tab, L, R, out in reqs:
        assert np.array_equal(out, reference(orc, arrays[tab], L, R)), (tab, L.shape[0])


@pytest.mark.parametrize("copy", [False, True])
def test_burst_is_coalesced_and_exact(orc, copy):
    d = need_gpu()
    say("serve_burst", copy)
    arrays = arrays_for(8, 3)
    with serving.Server(num_streams=3, max_tables=16, copy_queries=copy) as srv:
        for A in arrays:
            srv.add_array(dev(A, d))
        reqs = serving.make_requests([a.shape[0] for a in arrays], 300, 1, 5e3, 5)
        t0 = serving.clock()
        res = serving.run_schedule(srv, reqs, [t0] * len(reqs))  # all arrive at once
        check(orc, arrays, reqs)
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["batches"] < len(reqs)
        assert res.mean_batch_requests > 1
        assert np.all(res.latencies_s > 0)


@pytest.mark.parametrize("copy", [False, True])
def test_alone_equals_in_mix(orc, copy):
    d = need_gpu()
    say("serve_alone_vs_mix", copy)
    arrays = arrays_for(6, 11)
    with serving.Server(num_streams=4, max_tables=8, copy_queries=copy) as srv:
        for A in arrays:
            srv.add_array(dev(A, d))
        ns = [a.shape[0] for a in arrays]
        probe = serving.make_requests(ns, 5, 100, 4e3, 13)
        alone = []
        for tab, L, R, out in probe:
            srv.wait(srv.submit(tab, L, R, out))
            alone.append(out.copy())
        # the same requests again, interleaved with 400 others arriving as a
        # Poisson stream fast enough that batches form and overlap
        mix = serving.make_requests(ns, 400, 1, 2e4, 17)
        again = [(t, L, R, np.full(L.shape[0], -3, dtype=np.int32)) for t, L, R, _ in probe]
        reqs = mix[:100] + [again[0]] + mix[100:200] + again[1:3] + mix[200:] + again[3:]
        t0 = serving.clock() + 1e-3
        arr = serving.poisson_schedule(len(reqs), 2e5, 19, t0)
        serving.run_schedule(srv, reqs, arr)
        for a, (tab, L, R, out) in zip(alone, again):
            assert np.array_equal(a, out)
            assert np.array_equal(out, reference(orc, arrays[tab], L, R))
        check(orc, arrays, mix)


def test_plain_per_request_server_agrees(orc):
    d = need_gpu()
    say("serve_plain")
    arrays = arrays_for(4, 23)
    ns = [a.shape[0] for a in arrays]
    reqs = serving.make_requests(ns, 60, 1, 3e3, 29)
    with serving.Server(num_streams=1, max_requests_per_batch=1, max_tables=4,
                        copy_queries=True) as srv:
        for A in arrays:
            srv.add_array(dev(A, d))
        serving.run_schedule(srv, reqs, [serving.clock()] * len(reqs))
        st = srv.stats()
        assert st["batches"] == len(reqs) and st["max_inflight"] == 1
    check(orc, arrays, reqs)


@pytest.mark.parametrize("copy", [False, True])
def test_admission_and_invalid_queries(orc, copy):
    d = need_gpu()
    say("serve_admission", copy)
    arrays = arrays_for(2, 31, 1e4, 2e4)
    # a small budget: each slot holds only a few thousand queries
    with serving.Server(num_streams=2, max_tables=2, max_requests_per_batch=64,
                        budget_bytes=2 * (3 * 4 * 3000 + 8192), copy_queries=copy) as srv:
        for A in arrays:
            srv.add_array(dev(A, d))
        cap = srv.stats()["slot_capacity"]
        assert 1000 < cap < 4000
        too_big = np.zeros(cap + 1, dtype=np.int32)
        with pytest.raises(rmq.RMQError):
            srv.submit(0, too_big, too_big, too_big.copy())
        reqs = serving.make_requests([a.shape[0] for a in arrays], 40, 500, cap, 37)
        tab, L, R, out = reqs[0]
        L[:3] = [5, -1, 7]
        R[:3] = [4, 3, arrays[tab].shape[0]]  # reversed, negative, past the end
        serving.run_schedule(srv, reqs, [serving.clock()] * len(reqs))
        assert np.all(out[:3] == -1)
        check(orc, arrays, reqs)
        st = srv.stats()
        assert st["queries"] == sum(r[1].shape[0] for r in reqs)


@pytest.mark.parametrize("copy", [False, True])
def test_two_level_tables_serve_exactly(orc, copy):
    """Every resident table with two block levels (Section 3.3): coalesced
    batches answered by the two-level query launch, vs the oracle."""
    d = need_gpu()
    say("serve_two_level", copy)
    arrays = arrays_for(6, 43, 2e4, 4e5)
    with serving.Server(num_streams=3, max_tables=8, copy_queries=copy,
                        sub_block_size=256) as srv:
        for A in arrays:
            srv.add_array(dev(A, d))
        reqs = serving.make_requests([a.shape[0] for a in arrays], 200, 1, 6e3, 47)
        t0 = serving.clock() + 1e-3
        serving.run_schedule(srv, reqs, serving.poisson_schedule(len(reqs), 1e5, 53, t0))
        check(orc, arrays, reqs)
        # the tables hold the k1-block minima beside the block table
        st = srv.stats()
        assert st["index_bytes"] == sum(rmq.build_bytes(a.shape[0], 0, 256) for a in arrays)
