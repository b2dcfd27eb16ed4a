"""CPU oracle for batched range-minimum queries -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps `liboracle.so`, built from `oracle.c`, which
shares no code with the HIP library.  Each wrapper cites the passage of
Grabowski & Kowalski, "Faster batched range minimum queries", whose plain
definition it computes; see `oracle.c` for the definitions themselves.

Parity pinning: every function here is pinned by `tests/test_oracle_pins.py`
against brute force, library routines, invariants, the Euler-tour LCA
reduction and planted-mistake checks.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib_path() -> str:
    return os.path.join(HERE, "liboracle.so")


def load(path: str | None = None, fresh: bool = False):
    """Load the oracle library (building it if absent)."""
    global _LIB
    if _LIB is not None and path is None and not fresh:
        return _LIB
    p = path or lib_path()
    if not os.path.exists(p):
        from . import build as _b

        _b.build()
    lib = ctypes.CDLL(p)
    v, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.oracle_num_threads.restype = i32
    lib.oracle_set_threads.argtypes = [i32]
    lib.oracle_rmq_scan.argtypes = [v, i64, v, v, i64, v]
    lib.oracle_rmq_scan.restype = i64
    lib.oracle_rmq_sparse_table.argtypes = [v, i64, i64, v, v, i64, v]
    lib.oracle_rmq_sparse_table.restype = i64
    lib.oracle_block_argmin.argtypes = [v, i64, i64, v]
    lib.oracle_block_sparse_table.argtypes = [v, v, i64, i32, v]
    lib.oracle_sort_endpoints.argtypes = [v, v, i64, v, v]
    lib.oracle_sort_endpoints.restype = ctypes.c_int
    lib.oracle_remap.argtypes = [v, i64, v, v]
    lib.oracle_contract.argtypes = [v, v, i64, v]
    lib.oracle_contracted_answer.argtypes = [v, v, v, v, i64, v]
    lib.oracle_euler_tour.argtypes = [v, i64, v, v, v]
    lib.oracle_euler_tour.restype = ctypes.c_int
    if path is None:
        _LIB = lib
    return lib


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


class Oracle:
    """Typed wrappers over one loaded copy of the library."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load()

    def num_threads(self) -> int:
        return int(self.lib.oracle_num_threads())

    def set_threads(self, t: int) -> None:
        self.lib.oracle_set_threads(int(t))

    def rmq_scan(self, A, L, R):
        """Section 1 definition: leftmost argmin of A[L[i]..R[i]]; -1 if invalid."""
        A, L, R = _i32(A), _i32(L), _i32(R)
        out = np.empty(L.shape[0], dtype=np.int32)
        self.lib.oracle_rmq_scan(_p(A), A.shape[0], _p(L), _p(R), L.shape[0], _p(out))
        return out

    def rmq_sparse_table(self, A, L, R, b: int = 1):
        """Section 2 Sparse Table over blocks of b elements (b = 1: textbook)."""
        A, L, R = _i32(A), _i32(L), _i32(R)
        out = np.empty(L.shape[0], dtype=np.int32)
        rc = self.lib.oracle_rmq_sparse_table(_p(A), A.shape[0], int(b), _p(L), _p(R),
                                              L.shape[0], _p(out))
        if rc < 0:
            raise MemoryError("oracle sparse table allocation failed")
        return out

    def block_argmin(self, A, k: int):
        """Section 3.2: argmin position of each block of k elements."""
        A = _i32(A)
        nb = (A.shape[0] + k - 1) // k
        pos = np.empty(nb, dtype=np.int32)
        self.lib.oracle_block_argmin(_p(A), A.shape[0], int(k), _p(pos))
        return pos

    def block_sparse_table(self, A, blk, levels: int):
        """Section 3.1 step 3: argmin over spans of 2^i blocks, level-major."""
        A, blk = _i32(A), _i32(blk)
        nb = blk.shape[0]
        st = np.empty(levels * nb, dtype=np.int32)
        self.lib.oracle_block_sparse_table(_p(A), _p(blk), nb, int(levels), _p(st))
        return st.reshape(levels, nb)

    def sort_endpoints(self, L, R):
        """Section 3.1 step 1: sorted (position, tag) endpoint list."""
        L, R = _i32(L), _i32(R)
        q = L.shape[0]
        pos = np.empty(2 * q, dtype=np.int32)
        tag = np.empty(2 * q, dtype=np.int32)
        if self.lib.oracle_sort_endpoints(_p(L), _p(R), q, _p(pos), _p(tag)) != 0:
            raise MemoryError("oracle sort allocation failed")
        return pos, tag

    def remap(self, tag):
        """Section 3.1 step 1: contracted index ranges [Lc[i], Rc[i]]."""
        tag = _i32(tag)
        q = tag.shape[0] // 2
        Lc = np.empty(q, dtype=np.int32)
        Rc = np.empty(q, dtype=np.int32)
        self.lib.oracle_remap(_p(tag), q, _p(Lc), _p(Rc))
        return Lc, Rc

    def contract(self, A, pos):
        """Section 3.1 step 2: position map of A_Q (argmin of each closed area)."""
        A, pos = _i32(A), _i32(pos)
        m = pos.shape[0]
        aq = np.empty(max(m - 1, 0), dtype=np.int32)
        self.lib.oracle_contract(_p(A), _p(pos), m, _p(aq))
        return aq

    def euler_tour(self, parent):
        """Section 1 (LCA reduces to RMQ): (depth, node, first) of the Euler
        tour, children in increasing id; None if parent[] is not one tree."""
        parent = _i32(parent)
        N = parent.shape[0]
        depth = np.empty(2 * N - 1, dtype=np.int32)
        node = np.empty(2 * N - 1, dtype=np.int32)
        first = np.empty(N, dtype=np.int32)
        if self.lib.oracle_euler_tour(_p(parent), N, _p(depth), _p(node), _p(first)) != 0:
            return None
        return depth, node, first

    def contracted_answer(self, A, aq, Lc, Rc):
        """Section 3.1 step 4 (without blocks): minimum over A_Q[Lc..Rc]."""
        A, aq, Lc, Rc = _i32(A), _i32(aq), _i32(Lc), _i32(Rc)
        out = np.empty(Lc.shape[0], dtype=np.int32)
        self.lib.oracle_contracted_answer(_p(A), _p(aq), _p(Lc), _p(Rc), Lc.shape[0], _p(out))
        return out
