"""Pins for the CPU oracle: checks against what the paper and mathematics fix,
never against the oracle's own code.  Each check raises AssertionError on a
mismatch.  `run_all` is also used to show that planted mistakes in the oracle
are caught (tests/test_oracle_mutants.py).

Sources of truth used here:
  * brute force over every range of tiny arrays, via Python's min with the
    lexicographic (value, position) key -- the definition of RMQ with the
    leftmost tie-break (Section 1);
  * numpy.argmin, which returns the first occurrence of the minimum;
  * invariants of the answer (inside the range, minimal, leftmost);
  * the Euler-tour reduction of LCA to RMQ (Section 1): the minimum-depth step
    between first visits is the lowest common ancestor, checked against LCA
    found by climbing parent pointers;
  * examples worked by hand (tests/golden/handworked.json);
  * structural facts of the contraction (Section 3.1 steps 1-2): 2q-1
    entries, segments that tile each query exactly, numpy.lexsort order.
"""
from __future__ import annotations

import json
import os

import numpy as np

import workloads as W

INT_MIN = np.iinfo(np.int32).min
INT_MAX = np.iinfo(np.int32).max

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "handworked.json")


def tiny_arrays():
    """Named small arrays covering ties, monotone runs and extreme values."""
    out = []
    rng = np.random.default_rng(1706)
    for n in (1, 2, 3, 7, 16, 33, 64):
        out.append((f"rand5_n{n}", rng.integers(0, 5, n).astype(np.int32)))
    out.append(("equal", np.full(40, 7, dtype=np.int32)))
    out.append(("increasing", np.arange(50, dtype=np.int32)))
    out.append(("decreasing", np.arange(50, 0, -1).astype(np.int32)))
    walk = np.cumsum(rng.choice([-1, 1], 64)).astype(np.int32)
    out.append(("pm1_walk", walk))
    ext = rng.choice(np.array([INT_MIN, INT_MAX, 0, -1, 1], dtype=np.int64), 48).astype(np.int32)
    out.append(("extremes", ext))
    out.append(("negative", (-rng.integers(0, 1 << 31, 64)).astype(np.int32)))
    out.append(("wide", rng.integers(INT_MIN, INT_MAX, 64, endpoint=True).astype(np.int32)))
    return out


def all_ranges(n: int):
    L, R = np.triu_indices(n)
    return L.astype(np.int32), R.astype(np.int32)


def brute(A, l, r):
    return min(range(l, r + 1), key=lambda t: (int(A[t]), t))


def check_scan_bruteforce(orc):
    for name, A in tiny_arrays():
        L, R = all_ranges(A.shape[0])
        got = orc.rmq_scan(A, L, R)
        for l, r, g in zip(L, R, got):
            exp = brute(A, int(l), int(r))
            assert g == exp, (name, l, r, g, exp)
            assert g == l + int(np.argmin(A[l:r + 1])), (name, l, r)


def check_sparse_table_bruteforce(orc):
    for name, A in tiny_arrays():
        L, R = all_ranges(A.shape[0])
        exp = np.array([brute(A, int(l), int(r)) for l, r in zip(L, R)], dtype=np.int32)
        for b in (1, 2, 3, 5, 8, 32):
            got = orc.rmq_sparse_table(A, L, R, b)
            bad = np.nonzero(got != exp)[0]
            assert bad.size == 0, (name, b, L[bad[:3]], R[bad[:3]], got[bad[:3]], exp[bad[:3]])


def check_invariants(orc, n=100_000, q=3000, seed=5):
    rng = np.random.default_rng(seed)
    for vals in (16, 1 << 31):
        A = (rng.integers(0, vals, n) - vals // 2).astype(np.int32)
        L, R = W.uniform_queries(n, q, seed)
        sL, sR = W.short_queries(n, q // 2, seed, 3, 64)
        L = np.concatenate([L, sL, [0, n - 1, 5]]).astype(np.int32)
        R = np.concatenate([R, sR, [n - 1, n - 1, 5]]).astype(np.int32)
        for fn in (lambda: orc.rmq_scan(A, L, R),
                   lambda: orc.rmq_sparse_table(A, L, R, 1),
                   lambda: orc.rmq_sparse_table(A, L, R, 32)):
            out = fn()
            assert np.all((L <= out) & (out <= R))
            for l, r, o in zip(L, R, out):
                seg = A[l:r + 1]
                m = seg.min()
                assert A[o] == m
                assert not np.any(A[l:o] == m), "not leftmost"


def check_whole_array(orc):
    rng = np.random.default_rng(9)
    for n in (1, 5, 1000, 65537):
        A = rng.integers(-50, 50, n).astype(np.int32)
        L = np.array([0], dtype=np.int32)
        R = np.array([n - 1], dtype=np.int32)
        assert orc.rmq_scan(A, L, R)[0] == int(np.argmin(A))
        assert orc.rmq_sparse_table(A, L, R, 1)[0] == int(np.argmin(A))
        assert orc.rmq_sparse_table(A, L, R, 4)[0] == int(np.argmin(A))


def naive_lca(parent, depth_of, u, v):
    while depth_of[u] > depth_of[v]:
        u = parent[u]
    while depth_of[v] > depth_of[u]:
        v = parent[v]
    while u != v:
        u, v = parent[u], parent[v]
    return u


def node_depths(parent):
    d = np.zeros(parent.shape[0], dtype=np.int64)
    for i in range(1, parent.shape[0]):
        d[i] = d[parent[i]] + 1  # parent[i] < i
    return d


def check_lca(orc):
    for N, seed in ((1, 1), (2, 2), (10, 3), (100, 4), (1000, 5), (4000, 6)):
        parent = W.random_recursive_tree(N, seed)
        tour = orc.euler_tour(parent)
        assert tour is not None, (N, seed)
        depth, node, first = tour
        assert np.all(np.abs(np.diff(depth)) == 1)
        dn = node_depths(parent)
        u, v, L, R = W.lca_queries(first, 500, seed)
        for out in (orc.rmq_scan(depth, L, R), orc.rmq_sparse_table(depth, L, R, 1),
                    orc.rmq_sparse_table(depth, L, R, 8)):
            for a, b, o in zip(u, v, out):
                lca = naive_lca(parent, dn, int(a), int(b))
                assert node[o] == lca, (N, a, b, node[o], lca)
                assert depth[o] == dn[lca]


def first_occurrence(node, N):
    f = np.full(N, -1, dtype=np.int64)
    for i in range(node.shape[0] - 1, -1, -1):
        f[node[i]] = i
    return f


def check_euler_tour(orc):
    """The oracle's Euler tour (Section 1): hand-worked tour, structure of the
    tour (2N-1 steps of +-1, node depths, first occurrences, every edge
    walked down and up once), LCA by parent climbing, and None for inputs
    that are not one tree."""
    with open(GOLDEN) as f:
        lg = json.load(f)["lca"]
    res = orc.euler_tour(np.array(lg["parent"], dtype=np.int32))
    assert res is not None
    depth, node, first = res
    assert depth.tolist() == lg["euler_depth"] and node.tolist() == lg["euler_node"]
    assert first.tolist() == lg["first"]
    rng = np.random.default_rng(21)
    trees = [W.random_recursive_tree(N, N + 1) for N in (1, 2, 3, 50, 3000)]
    trees.append(np.arange(-1, 999, dtype=np.int32))        # a path, depth 999
    trees.append(np.r_[-1, np.zeros(500, dtype=np.int32)])   # a star
    perm = rng.permutation(700)                                # relabelled random tree
    base = W.random_recursive_tree(700, 5)
    relab = np.empty(700, dtype=np.int32)
    relab[perm] = np.where(base < 0, -1, perm[np.maximum(base, 0)])
    trees.append(relab)
    for parent in trees:
        N = parent.shape[0]
        res = orc.euler_tour(parent)
        assert res is not None, N
        depth, node, first = res
        assert depth.shape[0] == 2 * N - 1 and node.shape[0] == 2 * N - 1
        assert np.all(np.abs(np.diff(depth)) == 1)
        root = int(np.nonzero(parent < 0)[0][0])
        assert node[0] == root and node[-1] == root and depth[0] == 0
        dn = np.zeros(N, dtype=np.int64)
        for v in range(N):  # depth by climbing
            x, d = v, 0
            while parent[x] >= 0:
                x, d = parent[x], d + 1
            dn[v] = d
        assert np.array_equal(depth, dn[node])
        assert np.array_equal(first, first_occurrence(node, N))
        steps = [(int(node[i]), int(node[i + 1])) for i in range(2 * N - 2)]
        down = [(a, b) for i, (a, b) in enumerate(steps) if depth[i + 1] == depth[i] + 1]
        up = [(b, a) for i, (a, b) in enumerate(steps) if depth[i + 1] == depth[i] - 1]
        edges = sorted((int(parent[b]), b) for b in range(N) if parent[b] >= 0)
        assert sorted(down) == edges and sorted(up) == edges  # each edge down once, up once
        for v in range(N):  # children in increasing id
            kids = [b for a, b in down if a == v]
            assert kids == sorted(kids)
        if N > 1:
            u = rng.integers(0, N, 300)
            w = rng.integers(0, N, 300)
            L = np.minimum(first[u], first[w]).astype(np.int32)
            R = np.maximum(first[u], first[w]).astype(np.int32)
            out = orc.rmq_scan(depth, L, R)
            for a, b, o in zip(u, w, out):
                assert node[o] == naive_lca(parent, dn, int(a), int(b))
    for bad in ([-1, -1, 0], [-1, 2, 1], [0], [-1, 5], [-1, 0, 3, 2], [1, 0, -1]):
        assert orc.euler_tour(np.array(bad, dtype=np.int32)) is None, bad


def check_golden(orc):
    with open(GOLDEN) as f:
        g = json.load(f)
    A = np.array(g["A"], dtype=np.int32)
    L = np.array([e["l"] for e in g["rmq"]], dtype=np.int32)
    R = np.array([e["r"] for e in g["rmq"]], dtype=np.int32)
    exp = np.array([e["out"] for e in g["rmq"]], dtype=np.int32)
    assert np.array_equal(orc.rmq_scan(A, L, R), exp)
    for b in (1, 2, 3):
        assert np.array_equal(orc.rmq_sparse_table(A, L, R, b), exp)
    blk = g["blocks"]
    pos = orc.block_argmin(A, blk["k"])
    assert pos.tolist() == blk["argmin"]
    st = orc.block_sparse_table(A, pos, len(blk["levels"]))
    assert st.tolist() == blk["levels"]
    c = g["contraction"]
    sp, st_ = orc.sort_endpoints(c["L"], c["R"])
    assert sp.tolist() == c["sorted_pos"] and st_.tolist() == c["sorted_tag"]
    Lc, Rc = orc.remap(st_)
    assert Lc.tolist() == c["Lc"] and Rc.tolist() == c["Rc"]
    aq = orc.contract(A, sp)
    assert aq.tolist() == c["aq_pos"]
    assert orc.contracted_answer(A, aq, Lc, Rc).tolist() == c["answers"]
    lg = g["lca"]
    tour = orc.euler_tour(np.array(lg["parent"], dtype=np.int32))
    assert tour is not None
    depth, node, first = tour
    assert depth.tolist() == lg["euler_depth"] and node.tolist() == lg["euler_node"]
    assert first.tolist() == lg["first"]
    u = np.array([e["u"] for e in lg["queries"]])
    v = np.array([e["v"] for e in lg["queries"]])
    Lq = np.minimum(first[u], first[v]).astype(np.int32)
    Rq = np.maximum(first[u], first[v]).astype(np.int32)
    out = orc.rmq_scan(depth, Lq, Rq)
    assert [int(node[o]) for o in out] == [e["lca"] for e in lg["queries"]]


def check_blocks(orc):
    rng = np.random.default_rng(11)
    for n in (1, 7, 64, 1000, 4099):
        A = rng.integers(0, 6, n).astype(np.int32)
        for k in (1, 3, 16, 1000):
            nb = (n + k - 1) // k
            pos = orc.block_argmin(A, k)
            exp = [j * k + int(np.argmin(A[j * k:min(n, (j + 1) * k)])) for j in range(nb)]
            assert pos.tolist() == exp, (n, k)
            levels = max(1, int(np.floor(np.log2(nb))) + 2)
            st = orc.block_sparse_table(A, pos, levels)
            for i in range(levels):
                for j in range(nb):
                    lo, hi = j * k, min(n, (j + (1 << i)) * k)
                    assert st[i, j] == lo + int(np.argmin(A[lo:hi])), (n, k, i, j)


def contraction_cases():
    rng = np.random.default_rng(21)
    cases = []
    for n, q in ((1, 1), (5, 3), (64, 40), (1000, 7), (5000, 300)):
        A = rng.integers(0, 8, n).astype(np.int32)
        L, R = W.uniform_queries(n, q, 100 + n)
        cases.append((A, L, R))
    # duplicate endpoints, single-point queries, whole-array queries
    A = rng.integers(0, 3, 200).astype(np.int32)
    L = np.array([5, 5, 5, 0, 199, 10, 10, 0, 7], dtype=np.int32)
    R = np.array([5, 9, 9, 199, 199, 10, 50, 0, 7], dtype=np.int32)
    cases.append((A, L, R))
    return cases


def check_contraction(orc):
    for A, L, R in contraction_cases():
        q = L.shape[0]
        pos, tag = orc.sort_endpoints(L, R)
        # the order numpy.lexsort gives on (position, tag)
        allpos = np.empty(2 * q, dtype=np.int64)
        allpos[0::2], allpos[1::2] = L, R
        order = np.lexsort((np.arange(2 * q), allpos))
        assert np.array_equal(pos, allpos[order]) and np.array_equal(tag, order)
        Lc, Rc = orc.remap(tag)
        assert np.all(Lc <= Rc)
        assert np.array_equal(pos[Lc], L) and np.array_equal(pos[Rc + 1], R)
        aq = orc.contract(A, pos)
        assert aq.shape[0] == 2 * q - 1
        for s in range(2 * q - 1):
            lo, hi = pos[s], pos[s + 1]
            assert aq[s] == lo + int(np.argmin(A[lo:hi + 1]))
        direct = orc.rmq_scan(A, L, R)
        assert np.array_equal(orc.contracted_answer(A, aq, Lc, Rc), direct)
        for l, r, o in zip(L, R, direct):
            assert o == brute(A, int(l), int(r))


def check_invalid(orc):
    A = np.arange(10, dtype=np.int32)
    L = np.array([-1, 3, 0, 9, 2], dtype=np.int32)
    R = np.array([3, 2, 10, 9, 2], dtype=np.int32)
    for out in (orc.rmq_scan(A, L, R), orc.rmq_sparse_table(A, L, R, 1),
                orc.rmq_sparse_table(A, L, R, 4)):
        assert out.tolist() == [-1, -1, -1, 9, 2]


ALL = [check_scan_bruteforce, check_sparse_table_bruteforce, check_whole_array, check_golden,
       check_blocks, check_contraction, check_invalid, check_lca, check_invariants,
       check_euler_tour]


def run_all(orc):
    for fn in ALL:
        fn(orc)
