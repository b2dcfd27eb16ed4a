"""Large plain-method batches over a small doubling table, where the query
kernel copies the whole table into each CU's LDS (tables of at most 144 KiB,
batches of at least 2^21 queries): every answer against the oracle, on both
sides of both switches, with one and two block levels, ragged last waves,
invalid queries mixed in, and through the resident index."""
import numpy as np
import pytest
import torch

import paper_1706_06940_amd as rmq
import workloads as W
from tests._gpu import dev, host, need_gpu, reference, say

pytestmark = pytest.mark.gpu

QMIN = 1 << 21          # the smallest batch that takes the LDS table
TABLE_WORDS = 144 * 1024 // 8


def words(nb):
    """Words of a doubling table of nb blocks (levels = floor(log2(nb - 2)) + 1)."""
    levels = 1 if nb <= 3 else int(nb - 2).bit_length()
    return nb * levels


def queries(n, q, seed):
    L, R = W.uniform_queries(n, q, seed)
    rng = np.random.default_rng(seed)
    # a tenth short ranges, and a few invalid ones (answer -1)
    m = q // 10
    sl, sr = W.short_queries(n, m, seed, 3, max(1, min(n, 4096)))
    L[:m], R[:m] = sl, sr
    bad = rng.choice(q, 5, replace=False)
    L[bad[0]], R[bad[0]] = 5, 4          # reversed
    L[bad[1]], R[bad[1]] = -1, 3         # negative
    L[bad[2]], R[bad[2]] = 0, n          # past the end
    L[bad[3]], R[bad[3]] = n - 1, n - 1  # last element
    L[bad[4]], R[bad[4]] = 0, n - 1      # whole array
    return L, R


@pytest.mark.timeout(600)
@pytest.mark.parametrize("n,k,k1,q", [
    # one level: table of 1465 blocks (129 KiB), batches on both sides of 2^19
    (3_000_017, 2048, 0, QMIN - 1), (3_000_017, 2048, 0, QMIN), (3_000_017, 2048, 0, 2_400_001),
    # one level, 2930 blocks (281 KiB): too big, the gathering kernel answers
    (3_000_017, 1024, 0, 2_400_001),
    # two levels, 1221 blocks of 16384 over 256-element sub-blocks
    (20_000_003, 16384, 256, QMIN + 37), (20_000_003, 16384, 256, 2_500_001),
    # tables at the size limit: 1536 blocks fit (16896 words), 2048 do not
    (1536 * 4096, 4096, 0, QMIN + 1), (2048 * 4096, 4096, 0, QMIN + 1),
    # a table of one level (2 blocks)
    (2 * 65536 - 5, 65536, 1024, QMIN + 63),
])
def test_lds_table_queries(orc, n, k, k1, q):
    d = need_gpu()
    nb = -(-n // k)
    say("lds_queries", n, k, k1, q, "table words", words(nb), "lds" if
        (q >= QMIN and words(nb) <= TABLE_WORDS) else "gather")
    A = W.uniform_int31(n, n + k + q)
    L, R = queries(n, q, n + q)
    exp = reference(orc, A, L, R)
    At = dev(A, d)
    bad = torch.zeros(1, dtype=torch.int64, device=d)
    got = host(rmq.query_batch(At, dev(L, d), dev(R, d), path="full", block_size=k,
                               sub_block_size=k1, bad_count=bad))
    wrong = np.nonzero(got != exp)[0]
    assert wrong.size == 0, (wrong[:4], L[wrong[:4]], R[wrong[:4]], got[wrong[:4]], exp[wrong[:4]])
    assert int(bad.item()) == 3


@pytest.mark.timeout(600)
def test_lds_table_resident_index(orc):
    d = need_gpu()
    n, k, k1, q = 10_000_019, 65536, 1024, 2_300_001
    say("lds_index", n, k, k1, q)
    A = W.uniform_int31(n, 77)
    At = dev(A, d)
    ix = rmq.Index(At, block_size=k, sub_block_size=k1)
    assert words(ix.num_blocks) <= TABLE_WORDS
    for rep in range(2):
        L, R = queries(n, q - rep * 1000, 91 + rep)
        exp = reference(orc, A, L, R)
        got = host(ix.query(dev(L, d), dev(R, d)))
        assert np.array_equal(got, exp), rep
