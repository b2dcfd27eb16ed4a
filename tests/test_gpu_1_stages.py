"""Each step of the two methods on its own, bit-exact against the oracle.

Section 3.2 / 3.1 step 3: block minima and the block Sparse Table.
Section 3.1 steps 1-2: endpoint sort, remap and contraction."""
import numpy as np
import pytest
import torch

import paper_1706_06940_amd as rmq
import workloads as W
from tests._gpu import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu


def check_keys(keys: np.ndarray, A: np.ndarray, pos_expected: np.ndarray, what: str):
    pos = (keys & 0xFFFFFFFF).astype(np.int64)
    assert np.array_equal(pos, pos_expected.astype(np.int64)), what
    hi = ((keys.astype(np.uint64) >> np.uint64(32)) ^ np.uint64(0x80000000)).astype(np.uint32)
    assert np.array_equal(hi.view(np.int32), A[pos_expected]), what + " values"


@pytest.mark.parametrize("n", [1, 3, 255, 256, 1000, 4097, 65536, (1 << 20) + 3])
@pytest.mark.parametrize("k", [16, 64, 256, 512, 1024, 2048, 4096, 16384, 65536])
def test_block_minima(orc, n, k):
    d = need_gpu()
    say("block_minima", n, k)
    for name, A in (("uniform", W.uniform_int31(n, n + k)),
                    ("ties", np.random.default_rng(k).integers(0, 3, n).astype(np.int32)),
                    ("max", np.full(n, np.iinfo(np.int32).max, dtype=np.int32))):
        keys = host(rmq.block_minima(dev(A, d), k)).view(np.uint64)
        check_keys(keys, A, orc.block_argmin(A, k), f"{name} n={n} k={k}")


def test_block_minima_unaligned(orc):
    d = need_gpu()
    say("block_minima_unaligned")
    A = W.uniform_int31(100_003, 4)
    At = dev(np.concatenate([[0], A]).astype(np.int32), d)[1:]  # 4-byte offset
    for k in (16, 256, 4096):
        keys = host(rmq.block_minima(At, k)).view(np.uint64)
        check_keys(keys, A, orc.block_argmin(A, k), f"unaligned k={k}")


@pytest.mark.parametrize("m", [1, 2, 127, 128, 1000, 100_001])
@pytest.mark.parametrize("k", [16, 128, 512, 4096])
def test_block_minima_keys(orc, m, k):
    d = need_gpu()
    say("block_minima_keys", m, k)
    rng = np.random.default_rng(m * 7 + k)
    S = rng.integers(0, 2 ** 63, m, dtype=np.int64)
    keys = host(rmq.block_minima_keys(dev(S, d), k)).view(np.uint64)
    Su = S.view(np.uint64)
    exp = np.array([Su[j:j + k].min() for j in range(0, m, k)], dtype=np.uint64)
    assert np.array_equal(keys, exp)


@pytest.mark.parametrize("nb", [1, 2, 3, 4, 5, 17, 1000, 1024, 1025, 4099, 97657])
def test_sparse_table(orc, nb):
    d = need_gpu()
    say("sparse_table", nb)
    k = 16
    n = nb * k - (k // 2 if nb > 1 else 0)
    A = np.random.default_rng(nb).integers(0, 50, n).astype(np.int32)
    blk = orc.block_argmin(A, k)
    levels = rmq.table_levels(nb)
    keys = rmq.block_minima(dev(A, d), k)
    st = host(rmq.sparse_table(keys, levels)).view(np.uint64)
    exp = orc.block_sparse_table(A, blk, levels)
    for j in range(levels):
        check_keys(st[j], A, exp[j], f"level {j} nb={nb}")


def test_sparse_table_all_levels_small(orc):
    """Every level a table of nb blocks can hold (windows cut at the end)."""
    d = need_gpu()
    say("sparse_table_all_levels")
    for nb in (2, 7, 64, 300, 3000):
        A = np.random.default_rng(nb + 1).integers(-5, 5, nb * 16).astype(np.int32)
        levels = int(np.floor(np.log2(nb))) + 1
        st = host(rmq.sparse_table(rmq.block_minima(dev(A, d), 16), levels)).view(np.uint64)
        exp = orc.block_sparse_table(A, orc.block_argmin(A, 16), levels)
        for j in range(levels):
            check_keys(st[j], A, exp[j], f"nb={nb} level {j}")


@pytest.mark.parametrize("n,q", [(1, 1), (10, 7), (1000, 1), (5000, 300), (1 << 20, 1024),
                                 (1_000_003, 40_000), (100_000, 1 << 17),
                                 # either side of the tile-size changes at 2q = 1e5 and 4e5
                                 (1_000_003, 49_999), (1_000_003, 50_000),
                                 (3_000_017, 199_999), (3_000_017, 200_000),
                                 (3_000_017, 250_001)])
def test_sort_endpoints(orc, n, q):
    d = need_gpu()
    say("sort_endpoints", n, q)
    L, R = W.uniform_queries(n, q, n + q)
    if q > 4:
        L[:3] = R[:3] = n // 2  # repeated and single-point endpoints
    pos, tag = rmq.sort_endpoints(dev(L, d), dev(R, d), n)
    ep, et = orc.sort_endpoints(L, R)
    assert np.array_equal(host(pos), ep) and np.array_equal(host(tag), et)


def test_sort_endpoints_invalid_queries_sort_as_zero(orc):
    d = need_gpu()
    say("sort_invalid")
    n = 1000
    L = np.array([5, 7, -1, 900, 3], dtype=np.int32)
    R = np.array([9, 2, 4, 1000, 3], dtype=np.int32)
    pos, tag = rmq.sort_endpoints(dev(L, d), dev(R, d), n)
    ok = (L >= 0) & (L <= R) & (R < n)
    Lx, Rx = np.where(ok, L, 0).astype(np.int32), np.where(ok, R, 0).astype(np.int32)
    ep, et = orc.sort_endpoints(Lx, Rx)
    assert np.array_equal(host(pos), ep) and np.array_equal(host(tag), et)


# the last rows leave most waves of the contraction without endpoints, the
# first of them with a last wave shorter than the others and the second with
# a partial last tile
@pytest.mark.parametrize("n,q", [(1, 1), (10, 7), (1000, 3), (5000, 300), (1 << 20, 1024),
                                 (1_000_003, 40_000), (3000, 20_000), (1021 * 1024, 5),
                                 (3_000_017, 6), (1 << 22, 2)])
def test_contract(orc, n, q):
    d = need_gpu()
    say("contract", n, q)
    for name, A in (("uniform", W.uniform_int31(n, q)),
                    ("ties", np.random.default_rng(q).integers(0, 4, n).astype(np.int32))):
        L, R = W.uniform_queries(n, q, n * 3 + q)
        if q > 10:
            L[:4] = R[:4] = n // 3
            L[4:8] = 0
            R[8:10] = n - 1
        ep, et = orc.sort_endpoints(L, R)
        Lc, Rc, aq = rmq.contract(dev(A, d), dev(ep, d), dev(et, d))
        eLc, eRc = orc.remap(et)
        assert np.array_equal(host(Lc), eLc) and np.array_equal(host(Rc), eRc), name
        exp = orc.contract(A, ep)
        check_keys(host(aq).view(np.uint64), A, exp, f"A_Q {name} n={n} q={q}")


def test_device_generator_matches_host():
    """The torch form of the seeded generator gives the same values on the GPU."""
    d = need_gpu()
    say("device_generator")
    got = W.uniform_int31_torch(1_000_003, 5, 3, device=d).cpu().numpy()
    assert np.array_equal(got, W.uniform_int31(1_000_003, 5, 3))
    Lt, Rt = W.uniform_queries_torch(10 ** 8, 20_000, 6, 8, device=d)
    Ln, Rn = W.uniform_queries(10 ** 8, 20_000, 6, 8)
    assert np.array_equal(Lt.cpu().numpy(), Ln) and np.array_equal(Rt.cpu().numpy(), Rn)

