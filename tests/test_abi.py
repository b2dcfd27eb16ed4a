"""The C ABI on the host (CPU only): symbols, status codes, sizes, planner.

None of these calls touches a device: invalid arguments are rejected before
any HIP call, and the size/plan functions are pure host logic."""
import ctypes
import json
import math
import os
import re

import pytest

import paper_1706_06940_amd as rmq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rmq.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rmq_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = rmq.lib()
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name


def test_status_strings():
    L = rmq.lib()
    for code in range(7):
        assert L.rmq_status_string(code).decode() == rmq.STATUS[code]


def test_index_bytes_reproduces_table2():
    """Section 4, Table 2: the BbST footprint 8 * nb * levels bytes."""
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "table2_memory.json")))
    for n in (10 ** 8, 10 ** 9):
        got = [round(100 * rmq.index_bytes(n, k) / (4 * n), 2) for k in g["bbst"]["k"]]
        assert got == g["bbst"][f"n={n}"], (n, got)


def test_con_footprint_reading_matches_table2():
    """Reading of the paper's BbST_CON footprint: 40 bytes per query plus the
    block Sparse Table over 2q/512 blocks reproduces all six cells."""
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "table2_memory.json")))
    for n in (10 ** 8, 10 ** 9):
        row = g["bbst_con"][f"n={n}"]
        for q, pct in zip(row["q"], row["pct"]):
            nb = math.ceil(2 * q / 512)
            b = 40 * q + 8 * nb * math.ceil(math.log2(nb))
            assert round(100 * b / (4 * n), 2) == pct


def test_table_levels():
    # levels = floor(log2(nb - 2)) + 1: the widest span strictly inside A
    assert [rmq.table_levels(nb) for nb in (1, 2, 3, 4, 5, 6, 10, 1024, 1026)] == \
        [1, 1, 1, 2, 2, 3, 4, 10, 11]


def test_table_levels_over_powers_of_l():
    # Section 3.1 over powers of l = 2^a: level i spans l^i blocks, and the
    # levels needed are those with l^i <= nb - 2 (the widest inner span)
    for a in (1, 2, 3, 4, 5):
        for nb in (1, 2, 3, 4, 5, 6, 17, 18, 19, 33, 34, 257, 258, 1025, 1026, 4099, 1 << 20,
                   (1 << 25) + 3):
            exp = 1
            while nb > 3 and (1 << (exp * a)) <= nb - 2:
                exp += 1
            assert rmq.table_levels(nb, a) == exp, (nb, a)
    assert rmq.table_levels(1 << 20, 4) == 5 and rmq.table_levels(18, 4) == 2
    L = rmq.lib()
    assert L.rmq_table_levels_ary(10, 6) == 0 and L.rmq_table_levels_ary(0, 2) == 0
    assert L.rmq_table_levels_ary(1000, 0) == L.rmq_table_levels(1000)
    # the table over powers of 16 takes a quarter of the doubling table's levels
    n, q = 10 ** 8, 10 ** 7
    two = rmq.workspace_bytes(n, q, "full", 32)
    sixteen = rmq.workspace_bytes(n, q, "full", 32, arity_log2=4)
    nb = -(-n // 32)
    assert two - sixteen == 8 * nb * (rmq.table_levels(nb) - rmq.table_levels(nb, 4))


def test_query_record_bytes():
    # two records per block, one 16-byte pair per level, while they take at
    # most 8 MiB
    for nb in (1, 2, 3, 4, 100, 16_384, 17_476, 17_477, 32_768, 10 ** 6):
        exp = 2 * nb * rmq.table_levels(nb) * 16
        assert rmq.query_record_bytes(nb) == (exp if exp <= 8 << 20 else 0), nb
    assert rmq.query_record_bytes(12_208) == 2 * 12_208 * 14 * 16  # n = 1e8, k = 8192
    assert rmq.query_record_bytes(17_476) > 0 and rmq.query_record_bytes(17_477) == 0
    assert rmq.query_record_bytes(24_415) == 0 and rmq.query_record_bytes(0) == 0
    # the offline workspace holds them unless asked not to
    n, q = 10 ** 8, 10 ** 7
    nb = -(-n // 8192)
    on = rmq.workspace_bytes(n, q, "full", 8192)
    off = rmq.workspace_bytes(n, q, "full", 8192, records=False)
    assert off < on <= off + rmq.query_record_bytes(nb) + 512


def test_invalid_arguments_rejected_on_host():
    L = rmq.lib()
    fake = ctypes.c_void_p(256)  # never dereferenced: rejected before any device work
    out = ctypes.c_void_p(512)
    assert L.rmq_query_batch(fake, 0, fake, fake, 1, out, None) == 1        # n < 1
    assert L.rmq_query_batch(fake, 10, fake, fake, -1, out, None) == 1      # q < 0
    assert L.rmq_query_batch(None, 10, fake, fake, 1, out, None) == 1       # A null
    assert L.rmq_query_batch(fake, 10, None, fake, 1, out, None) == 1       # L null
    assert L.rmq_query_batch(fake, 2 ** 31, fake, fake, 1, out, None) == 1  # n too big
    assert L.rmq_query_batch(ctypes.c_void_p(258), 10, fake, fake, 1, out, None) == 5
    o = rmq._Options()
    o.block_size = 1000  # not a power of two
    assert L.rmq_query_batch_ex(fake, 10, fake, fake, 1, out, None, ctypes.byref(o)) == 1
    o.block_size = 8     # below the minimum
    assert L.rmq_query_batch_ex(fake, 10, fake, fake, 1, out, None, ctypes.byref(o)) == 1
    o.block_size = 0
    o.path = 7
    assert L.rmq_query_batch_ex(fake, 10, fake, fake, 1, out, None, ctypes.byref(o)) == 1
    o.path = 0
    for a in (-1, 6):  # table arity l = 2^a outside 2..32
        o.table_arity_log2 = a
        assert L.rmq_query_batch_ex(fake, 10, fake, fake, 1, out, None, ctypes.byref(o)) == 1
        h = ctypes.c_void_p()
        assert L.rmq_build(fake, 10, ctypes.byref(o), None, ctypes.byref(h)) == 1
    assert L.rmq_index_bytes(0, 1024) == 0 and L.rmq_index_bytes(100, 1000) == 0
    assert L.rmq_workspace_bytes(10, -1, None) == 0


def test_workspace_sizes():
    n, q = 10 ** 8, 10 ** 7
    full = rmq.workspace_bytes(n, q, "full", 1024)
    nb = -(-n // 1024)
    assert full >= 8 * nb * rmq.table_levels(nb)
    con = rmq.workspace_bytes(n, q, "contracted", 512)
    m = 2 * q - 1
    nbq = -(-m // 512)
    # endpoint list, sort scratch, remapped ranges, A_Q and its table
    assert con >= 8 * 2 * q + 8 * 2 * q + 8 * q + 8 * m + 8 * nbq * rmq.table_levels(nbq)
    assert con < 60 * q + n // 256 + 8 * nbq * rmq.table_levels(nbq) + (1 << 20)


def test_plan():
    k, p = rmq.plan(10 ** 8, 10 ** 6)
    assert p in ("full", "contracted") and k >= 16 and (k & (k - 1)) == 0
    with pytest.raises(rmq.RMQError):
        rmq.plan(0, 5)


def test_plan_table_roundtrip():
    """Measured plans (host only): the nearest entry in (log2 n, log2 q)."""
    rmq.set_plan_table([(10 ** 6, 10 ** 3, 4096, "full"), (10 ** 6, 10 ** 6, 64, "contracted")])
    try:
        assert rmq.plan(10 ** 6, 900) == (4096, "full")
        assert rmq.plan(2 * 10 ** 6, 2 * 10 ** 6) == (64, "contracted")
        with pytest.raises(rmq.RMQError):
            rmq.set_plan_table([(10, 10, 1000, "full")])  # not a power of two
    finally:
        rmq.set_plan_table([])
    k, p = rmq.plan(10 ** 6, 10)
    assert p == "full" and k == rmq.default_block(10 ** 6, 10, "full")


def test_plan_table_two_levels():
    """A two-level entry (Section 3.3) is what path="auto" takes; rmq_plan
    (and batches) get the entry's one-level block size instead."""
    rmq.set_plan_table([(10 ** 8, 10 ** 7, 65536, "full", 1024, 8192),
                        (10 ** 8, 10 ** 3, 4096, "full")])
    try:
        assert rmq.plan_ex(10 ** 8, 10 ** 7) == (65536, "full", 1024)
        assert rmq.plan(10 ** 8, 10 ** 7) == (8192, "full")
        assert rmq.plan_ex(10 ** 8, 10 ** 3) == (4096, "full", 0)
        # an array smaller than the entry's k: one level
        assert rmq.plan_ex(30_000, 10 ** 7) == (8192, "full", 0)
        # the workspace of an auto call follows the two-level plan
        two = rmq.workspace_bytes(10 ** 8, 10 ** 7, "auto")
        assert two == rmq.workspace_bytes(10 ** 8, 10 ** 7, "full", 65536, 1024)
        for bad in ((10, 10, 1024, "full", 2048, 0), (10, 10, 1024, "contracted", 256, 0),
                    (10, 10, 1024, "full", 100, 0), (10, 10, 1024, "full", 256, 1000)):
            with pytest.raises(rmq.RMQError):
                rmq.set_plan_table([bad])
    finally:
        rmq.set_plan_table([])


def test_contracted_default_block_and_workspace():
    """sub_block_size alone picks k from the length of A_Q; the workspace
    holds the k1-block minima of A_Q beside its table (no query records)."""
    n, q = 1_000_003, 100_000
    one = rmq.workspace_bytes(n, q, "contracted", 4096, records=False)
    two = rmq.workspace_bytes(n, q, "contracted", 4096, sub_block_size=64)
    m = 2 * q - 1
    assert two - one >= 8 * (-(-m // 64)) and two - one <= 8 * (-(-m // 64)) + 512
    assert rmq.workspace_bytes(n, q, "contracted", 0, sub_block_size=64) > 0


def test_contracted_default_plan():
    """The contracted method's default: one block level with k about sqrt(2q)/2
    below 2^22 queries; from there two levels, k1 = 256 under the smallest
    block from 16384 whose table over the 2q - 1 entries of A_Q fits 144 KiB
    (levels = floor(log2(nb - 2)) + 1 of 8-byte keys)."""
    n = 10 ** 8
    for q in (1, 1000, 10 ** 6, (1 << 22) - 1):
        assert rmq.default_sub_block(n, q, "contracted") == 0
    for q in (1, 1000, 10 ** 6, 10 ** 7):
        assert rmq.default_sub_block(n, q, "full") == 0
    assert rmq.default_block(n, 10 ** 6, "contracted") == 512
    for q in (1 << 22, 10 ** 7, 5 * 10 ** 7, 3 * 10 ** 8):
        assert rmq.default_sub_block(n, q, "contracted") == 256
        k = rmq.default_block(n, q, "contracted")
        nb = -(-2 * q // k)
        levels = 1 if nb <= 3 else (nb - 2).bit_length()
        assert k >= 16384 and nb * levels * 8 <= 144 * 1024
        if k > 16384:  # the smallest such block
            nb2 = -(-2 * q // (k // 2))
            assert nb2 * (nb2 - 2).bit_length() * 8 > 144 * 1024
    assert rmq.default_block(n, 10 ** 7, "contracted") == 16384
    k = rmq.default_block(n, 10 ** 7, "contracted")
    k1 = rmq.default_sub_block(n, 10 ** 7, "contracted")
    assert rmq.workspace_bytes(n, 10 ** 7, "contracted") == \
        rmq.workspace_bytes(n, 10 ** 7, "contracted", k, sub_block_size=k1)


def test_build_bytes_is_the_index_footprint():
    """rmq_build_bytes: the table (Table 2's 8 * nb * levels for one block
    level), plus the k1-block minima with two levels (Section 3.3), plus the
    query records when they are built."""
    for n in (1, 1000, 10 ** 6 + 3, 10 ** 8):
        for k in (256, 4096, 65536):
            assert rmq.build_bytes(n, k, records=False) == rmq.index_bytes(n, k)
            rec = rmq.query_record_bytes(-(-n // k))
            with_rec = rmq.build_bytes(n, k)
            if rec:
                base = -(-rmq.index_bytes(n, k) // 256) * 256  # records start on 256 B
                assert with_rec == base + rec
            else:
                assert with_rec == rmq.index_bytes(n, k)
        assert rmq.build_bytes(n, 65536, 1024) == rmq.index_bytes(n, 65536) + 8 * (-(-n // 1024))
    assert rmq.build_bytes(0) == 0 and rmq.build_bytes(10, 100) == 0


def test_st_con_workspace_and_options():
    """The comparison system ST-RMQ_CON (Section 2): its workspace holds the
    element table over A_Q's 4q - 1 entries (floor(log2(4q - 1)) + 1 levels)
    beside the sort's; block sizes, two levels, another arity or more than
    2^29 queries are refused; the planner never picks it."""
    n, q = 10 ** 8, 10 ** 6
    m = 4 * q - 1
    levels = m.bit_length()
    w = rmq.workspace_bytes(n, q, "st_con")
    con = rmq.workspace_bytes(n, q, "contracted", 512, records=False)
    assert w >= 8 * m * levels
    assert w <= 8 * m * levels + con + 16 * q + n // 256 + (1 << 20)
    assert rmq.workspace_bytes(n, 1, "st_con") > 0
    assert rmq.workspace_bytes(n, q, "st_con", 256) == 0
    assert rmq.workspace_bytes(n, q, "st_con", sub_block_size=64) == 0
    assert rmq.workspace_bytes(n, q, "st_con", arity_log2=2) == 0
    assert rmq.workspace_bytes(n, (1 << 29) + 1, "st_con") == 0
    for qq in (10, 10 ** 4, 10 ** 7):
        assert rmq.plan_ex(n, qq)[1] in ("full", "contracted")


def test_three_block_levels_workspace_and_options():
    """Three block levels (Section 3.3, h = 3): the workspace adds the
    k2-block minima to the two-level one; k2 needs k1 > k2, the plain method
    and a single call (the resident index refuses it)."""
    n, q = 10 ** 8, 10 ** 6
    two = rmq.workspace_bytes(n, q, "full", 65536, sub_block_size=1024)
    three = rmq.workspace_bytes(n, q, "full", 65536, sub_block_size=1024, sub_block_size2=64)
    nb2 = -(-n // 64)
    assert 8 * nb2 <= three - two <= 8 * nb2 + 512
    assert rmq.workspace_bytes(n, q, "auto", 65536, sub_block_size=1024, sub_block_size2=64) == three
    assert rmq.workspace_bytes(n, q, "full", 65536, sub_block_size2=64) == 0            # no k1
    assert rmq.workspace_bytes(n, q, "full", 65536, sub_block_size=1024,
                               sub_block_size2=1024) == 0                              # k2 >= k1
    assert rmq.workspace_bytes(n, q, "full", 65536, sub_block_size=1024,
                               sub_block_size2=100) == 0                               # not a power of 2
    assert rmq.workspace_bytes(n, q, "contracted", 4096, sub_block_size=256,
                               sub_block_size2=64) == 0                                # plain only
    assert rmq.workspace_bytes(n, q, "st_con", sub_block_size2=64) == 0
    o = rmq._options(65536, "full", sub_block_size=1024, sub_block_size2=64)
    assert rmq.lib().rmq_build_bytes(n, ctypes.byref(o)) == 0
