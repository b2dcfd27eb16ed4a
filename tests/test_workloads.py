"""Seeded input generators (CPU only)."""
import numpy as np

import workloads as W


def test_counter_based_draws_are_piecewise_consistent():
    full = W.hashes(123, 4, 0, 1000)
    assert np.array_equal(full[500:], W.hashes(123, 4, 500, 500))
    assert all(int(full[i]) == W.hash_one(123, 4, i) for i in (0, 1, 77, 999))
    assert not np.array_equal(full, W.hashes(123, 5, 0, 1000))


def test_value_and_query_ranges():
    A = W.uniform_int31(100_000, 7)
    assert A.dtype == np.int32 and A.min() >= 0
    L, R = W.uniform_queries(1000, 50_000, 7)
    assert np.all((0 <= L) & (L <= R) & (R < 1000))
    Ls, Rs = W.short_queries(5000, 10_000, 7, 3, 1024)
    ln = Rs - Ls + 1
    assert ln.min() >= 1 and ln.max() <= 1024 and Rs.max() < 5000
    Lk, Rk = W.skewed_queries(10_000, 1001, 7)
    assert np.all((0 <= Lk) & (Lk <= Rk) & (Rk < 10_000))
    s = W.loguniform_ints(10_000, 10, 1e5, 7, 2)
    assert s.min() >= 10 and s.max() <= 100_000
    # roughly log-uniform: median near sqrt(10 * 1e5) = 1000
    assert 600 < np.median(s) < 1600


def test_random_recursive_tree():
    parent = W.random_recursive_tree(5000, 3)
    assert parent[0] == -1 and np.all(parent[1:] >= 0)
    assert np.all(parent[1:] < np.arange(1, 5000))
    assert not hasattr(W, "euler_tour")  # the tour is the oracle's, never the generator's


def test_paper_permutation_is_a_permutation():
    a = W.paper_permutation(10_001, 5)
    assert np.array_equal(np.sort(a), np.arange(1, 10_002))
    assert np.mean(a != np.arange(1, 10_002)) > 0.5


def test_torch_form_is_bit_identical():
    assert np.array_equal(W.hashes_torch(77, 3, 5, 10_000).numpy().view(np.uint64),
                          W.hashes(77, 3, 5, 10_000))
    assert np.array_equal(W.uniform_int31_torch(300_001, 9, 2, chunk=1 << 16).numpy(),
                          W.uniform_int31(300_001, 9, 2))
    for n in (1, 7, 10 ** 8, 2 ** 31 - 1):
        Lt, Rt = W.uniform_queries_torch(n, 5000, 11, 4)
        Ln, Rn = W.uniform_queries(n, 5000, 11, 4)
        assert np.array_equal(Lt.numpy(), Ln) and np.array_equal(Rt.numpy(), Rn)
