"""The batched and served forms at the shapes they are benchmarked on, every
answer checked element by element against the oracle (its Sparse Table over
32-element blocks), and the server's admission by device-memory footprint.

* batch: 256 arrays, n log-uniform in [1e4, 1e7], q log-uniform in [10, 1e5],
  values uniform in [0, 2^31), uniform queries -- the benchmark's batch, with
  the autotuner's plans; run fused, per item, and replayed from a hipGraph.
* served: the first 8 of the benchmark's 64 resident arrays (n from 1.06e6
  to 7.95e7; the five above ~4.5e6 elements carry no query records, the
  three below do), requests of q log-uniform in [1, 1e5] arriving as a
  Poisson stream.
"""
import numpy as np
import pytest
import torch

import paper_1706_06940_amd as rmq
import workloads as W
from paper_1706_06940_amd import serving
from tests._gpu import dev, host, need_gpu, reference, say

pytestmark = pytest.mark.gpu


def oracle_answers(orc, A_host, L_host, R_host):
    return orc.rmq_sparse_table(A_host, L_host, R_host, 32)


@pytest.mark.timeout(600)
def test_batch_256_arrays_at_benchmark_shape(orc):
    d = need_gpu()
    seed = W.BASE_SEED + 4
    ns = W.loguniform_ints(256, 1e4, 1e7, seed, 1)
    qs = W.loguniform_ints(256, 10, 1e5, seed, 2)
    say("batch256 total n", int(ns.sum()), "total q", int(qs.sum()))
    arrays = [W.uniform_int31_torch(int(n), seed, 100 + j, device=d) for j, n in enumerate(ns)]
    queries = [W.uniform_queries_torch(int(n), int(q), seed, 1000 + 2 * j, device=d)
               for j, (n, q) in enumerate(zip(ns, qs))]
    torch.cuda.synchronize()
    exp = [oracle_answers(orc, A.cpu().numpy(), L.cpu().numpy(), R.cpu().numpy())
           for A, (L, R) in zip(arrays, queries)]
    rmq.load_plan_table()
    try:
        b = rmq.Batch(arrays, queries)
        plans = {b.plan(j)[1] for j in range(256)}
        assert plans <= {"full", "contracted"}

        def check(what):
            for j, (o, e) in enumerate(zip(b.outs, exp)):
                got = host(o)
                assert np.array_equal(got, e), (what, j, int(ns[j]), int(qs[j]))

        s = torch.cuda.Stream(device=d)
        for mode in ("fused", "per_item"):
            say("batch256", mode)
            for o in b.outs:
                o.fill_(-7)
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                b.run(mode, stream=s)
            s.synchronize()
            check(mode)
            for rep in range(3):
                say("batch256", mode, "graph replay", rep)
                for o in b.outs:
                    o.fill_(-7)
                torch.cuda.synchronize()
                with torch.cuda.stream(s):
                    b.run(mode, graph=True, stream=s)
                s.synchronize()
                check(f"{mode} graph replay {rep}")
                # eager single-array work between the replays
                j = rep * 50
                eager = rmq.query_batch(arrays[j], *queries[j])
                assert np.array_equal(host(eager), exp[j])
        b.free()
    finally:
        rmq.set_plan_table([])


@pytest.mark.timeout(600)
@pytest.mark.parametrize("copy", [False, True])
def test_served_mix_at_benchmark_shape(orc, copy):
    d = need_gpu()
    seed = W.BASE_SEED + 5
    ns = W.loguniform_ints(64, 1e6, 1e8, seed, 1)[:8]
    say("serve8", copy, "n", [int(n) for n in ns])
    arrays = [W.uniform_int31_torch(int(n), seed, 200 + j, device=d) for j, n in enumerate(ns)]
    hosts = [A.cpu().numpy() for A in arrays]
    reqs = serving.make_requests(ns, 600, 1, 1e5, seed)
    with serving.Server(num_streams=4, max_tables=8, max_requests_per_batch=4096,
                        budget_bytes=4 * 12 * (1 << 21) + (1 << 20), copy_queries=copy) as srv:
        for A in arrays:
            srv.add_array(A)
        st = srv.stats()
        records = [rmq.query_record_bytes(-(-int(n) // k)) > 0
                   for n, k in ((n, _default_k(int(n))) for n in ns)]
        assert any(records) and not all(records)  # both query forms are served
        # first all at once (batches fill up), then a Poisson stream
        serving.run_schedule(srv, reqs[:200], [serving.clock()] * 200)
        t0 = serving.clock() + 1e-3
        res = serving.run_schedule(srv, reqs[200:], serving.poisson_schedule(400, 5e4, seed, t0))
        assert res.mean_batch_requests >= 1
        st = srv.stats()
        assert st["completed"] == 600
    # one oracle call per array over all of its requests' queries
    for tab in range(len(arrays)):
        mine = [r for r in reqs if r[0] == tab]
        if not mine:
            continue
        L = np.concatenate([r[1] for r in mine])
        R = np.concatenate([r[2] for r in mine])
        got = np.concatenate([r[3] for r in mine])
        exp = oracle_answers(orc, hosts[tab], L, R)
        assert np.array_equal(got, exp), (tab, L.shape[0])


def _default_k(n):
    """Block size the server's tables take for n elements (rmq_build's
    default: the power of two near sqrt(n) / 4, at least 256)."""
    k = 256
    while k < (1 << 20) and 2 * k <= (n ** 0.5) / 4:
        k *= 2
    return k


def test_server_refuses_a_table_beyond_its_hbm_budget(orc):
    d = need_gpu()
    say("serve hbm budget")
    n1, n2 = 2_000_003, 3_000_017
    A1 = W.uniform_int31(n1, 8101)
    A2 = W.uniform_int31(n2, 8102)
    b1, b2 = rmq.build_bytes(n1), rmq.build_bytes(n2)
    assert b1 > 0 and b2 > 0
    # a budget below what the server itself holds is refused at creation
    with pytest.raises(rmq.RMQError) as ei:
        serving.Server(num_streams=2, max_tables=4, copy_queries=True,
                       budget_bytes=1 << 20, hbm_budget_bytes=1 << 16)
    assert ei.value.status == 2
    with serving.Server(num_streams=2, max_tables=4, copy_queries=True,
                        budget_bytes=1 << 20, hbm_budget_bytes=(1 << 20) + b1 + b2 // 2) as srv:
        fixed = srv.stats()["hbm_bytes"]
        assert 0 < fixed <= (1 << 20) + 4096
        t1 = srv.add_array(dev(A1, d))
        st = srv.stats()
        assert st["index_bytes"] == b1 and st["hbm_bytes"] == fixed + b1
        with pytest.raises(rmq.RMQError) as ei:
            srv.add_array(dev(A2, d))
        assert ei.value.status == 2
        st = srv.stats()
        assert st["index_bytes"] == b1 and st["hbm_bytes"] == fixed + b1
        # the resident table still serves, and a smaller array still fits
        L, R = W.uniform_queries(n1, 3000, 8103)
        out = np.full(3000, -5, dtype=np.int32)
        srv.wait(srv.submit(t1, L, R, out))
        assert np.array_equal(out, reference(orc, A1, L, R))
        A3 = W.uniform_int31(5000, 8104)
        t3 = srv.add_array(dev(A3, d))
        L3, R3 = W.uniform_queries(5000, 100, 8105)
        out3 = np.full(100, -5, dtype=np.int32)
        srv.wait(srv.submit(t3, L3, R3, out3))
        assert np.array_equal(out3, reference(orc, A3, L3, R3))
