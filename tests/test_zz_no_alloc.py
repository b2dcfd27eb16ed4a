"""rmq_query_batch_noalloc (scratch in the library's fixed device array)
against rmq_query_batch_ex (scratch from the pool) and the oracle, on two
calls in a row, the second smaller, so that it runs over what the first left
in the array."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1706_06940_amd as rmq
import workloads as W
from tests._gpu import dev, host, need_gpu, reference, say

pytestmark = pytest.mark.gpu

SHAPES = [(3_000_017, 200_001), (70_001, 5_003)]  # second call smaller


@pytest.mark.parametrize("path,k,k1", [("full", 0, 0), ("full", 4096, 256), ("contracted", 0, 0),
                                       ("contracted", 256, 32), ("auto", 0, 0)])
def test_noalloc_equals_pool_scratch(orc, path, k, k1):
    d = need_gpu()
    for call, (n, q) in enumerate(SHAPES):
        say("noalloc", path, k, k1, "call", call, "n", n, "q", q)
        seed = 7100 + 10 * call
        A = W.uniform_int31(n, seed) if call == 0 else \
            np.random.default_rng(seed).integers(-3, 3, n).astype(np.int32)
        L, R = W.uniform_queries(n, q, seed + 1)
        L[:2], R[:2] = [4, -1], [3, 2]  # two invalid queries
        At, Lt, Rt = dev(A, d), dev(L, d), dev(R, d)
        bad_a = torch.zeros(1, dtype=torch.int64, device=d)
        bad_b = torch.zeros(1, dtype=torch.int64, device=d)
        out = torch.full((q,), -5, dtype=torch.int32, device=d)
        rmq.query_batch_noalloc(At, Lt, Rt, out, path=path, block_size=k, sub_block_size=k1,
                                bad_count=bad_a)
        ref = rmq.query_batch(At, Lt, Rt, path=path, block_size=k, sub_block_size=k1,
                              bad_count=bad_b)
        got = host(out)
        assert np.array_equal(got, host(ref)), (path, call)
        assert np.array_equal(got, reference(orc, A, L, R)), (path, call)
        assert int(bad_a.item()) == int(bad_b.item()) == 2


def test_noalloc_allocates_nothing_after_setup(orc):
    d = need_gpu()
    say("noalloc repeat")
    n, q = 1_000_003, 50_000
    A = W.uniform_int31(n, 7301)
    L, R = W.uniform_queries(n, q, 7302)
    At, Lt, Rt = dev(A, d), dev(L, d), dev(R, d)
    exp = reference(orc, A, L, R)
    outs = [torch.empty(q, dtype=torch.int32, device=d) for _ in range(3)]
    for path in ("full", "contracted"):
        rmq.query_batch_noalloc(At, Lt, Rt, outs[0], path=path)  # first call: set-up
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info(d)[0]
        for o in outs[1:]:
            rmq.query_batch_noalloc(At, Lt, Rt, o, path=path)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info(d)[0] == free0, path
        for o in outs:
            assert np.array_equal(host(o), exp), path


def test_noalloc_refuses_beyond_its_array():
    d = need_gpu()
    say("noalloc limit")
    n, q = 1 << 20, 3_000_000  # the contracted method needs ~170 MiB here
    assert rmq.workspace_bytes(n, q, "contracted") > rmq.NOALLOC_SCRATCH_BYTES
    A = torch.zeros(n, dtype=torch.int32, device=d)
    L = torch.zeros(q, dtype=torch.int32, device=d)
    out = torch.full((q,), -9, dtype=torch.int32, device=d)
    with pytest.raises(rmq.RMQError) as ei:
        rmq.query_batch_noalloc(A, L, L, out, path="contracted")
    assert ei.value.status == 6
    torch.cuda.synchronize()
    assert bool((out == -9).all())  # nothing was enqueued
    # a caller workspace is not taken
    o = rmq._options(0, "full")
    o.workspace, o.workspace_bytes = A.data_ptr(), 4 * n
    st = rmq.lib().rmq_query_batch_noalloc(A.data_ptr(), n, L.data_ptr(), L.data_ptr(), 16,
                                           out.data_ptr(), None, ctypes.byref(o))
    assert st == 1
