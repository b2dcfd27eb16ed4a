"""Python binding of librmq: batched offline range minimum queries on MI355X.

Argument marshalling only -- every step of both methods runs in the HIP
kernels of librmq.so (see include/rmq.h for the C ABI this mirrors).  Tensors
are torch CUDA (HIP) tensors; calls enqueue on the current stream of the
tensor's device and return without synchronising.

Methods (Grabowski & Kowalski, "Faster batched range minimum queries"):
  path="full"        Section 3.2, block Sparse Table over all of A (BbST)
  path="contracted"  Section 3.1, contraction of A to A_Q first (BbST_CON)
  path="auto"        the library's planner
Answers are the LEFTMOST position of the minimum of A[L[i]..R[i]] (0-based,
inclusive), -1 for an invalid query.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librmq.so")

OK = 0
STATUS = {0: "ok", 1: "invalid argument", 2: "out of device memory", 3: "HIP runtime error",
          4: "workspace too small", 5: "misaligned device pointer",
          6: "needs more than the fixed scratch array"}
PATHS = {"auto": 0, "full": 1, "contracted": 2, "st_con": 3}
MIN_BLOCK = 16
MAX_BLOCK = 1 << 24
NUM_STAGES = 4
STAGE_NAMES = ("sort", "contract_or_blockmin", "sparse_table", "query")


class RMQError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn}: {STATUS.get(status, status)} (status {status})")
        self.status = status


class _Options(ctypes.Structure):
    _fields_ = [
        ("block_size", ctypes.c_int32),
        ("path", ctypes.c_int32),
        ("bad_count", ctypes.c_void_p),
        ("stats", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
        ("timer", ctypes.c_void_p),
        ("sub_block_size", ctypes.c_int32),
        ("table_arity_log2", ctypes.c_int32),
        ("no_query_records", ctypes.c_int32),
        ("sub_block_size2", ctypes.c_int32),
    ]


_LIB = None


def lib() -> ctypes.CDLL:
    """The loaded librmq.so.  Raises if it has not been built: there is no
    fallback implementation."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1706_06940_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    v, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    opt = ctypes.POINTER(_Options)
    sigs = {
        "rmq_status_string": ([i32], ctypes.c_char_p),
        "rmq_version": ([], ctypes.c_char_p),
        "rmq_query_batch": ([v, i64, v, v, i64, v, v], i32),
        "rmq_query_batch_ex": ([v, i64, v, v, i64, v, v, opt], i32),
        "rmq_query_batch_noalloc": ([v, i64, v, v, i64, v, v, opt], i32),
        "rmq_workspace_bytes": ([i64, i64, opt], sz),
        "rmq_plan": ([i64, i64, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "rmq_plan_ex": ([i64, i64, ctypes.POINTER(i32), ctypes.POINTER(i32),
                         ctypes.POINTER(i32)], i32),
        "rmq_default_block": ([i64, i64, i32], i32),
        "rmq_default_sub_block": ([i64, i64, i32], i32),
        "rmq_build": ([v, i64, opt, v, ctypes.POINTER(v)], i32),
        "rmq_query_index": ([v, v, v, i64, v, v], i32),
        "rmq_query_index_ex": ([v, v, v, i64, v, v, opt], i32),
        "rmq_index_free": ([v], i32),
        "rmq_build_bytes": ([i64, opt], sz),
        "rmq_lca_build": ([v, i64, opt, v, ctypes.POINTER(v)], i32),
        "rmq_lca_query": ([v, v, v, i64, v, v, opt], i32),
        "rmq_lca_copy_tour": ([v, v, v, v, v], i32),
        "rmq_lca_info": ([v, ctypes.POINTER(i64), ctypes.POINTER(sz)], i32),
        "rmq_lca_free": ([v], i32),
        "rmq_index_info": ([v, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i64),
                            ctypes.POINTER(i32), ctypes.POINTER(sz)], i32),
        "rmq_index_copy_table": ([v, v, v], i32),
        "rmq_index_bytes": ([i64, i32], sz),
        "rmq_table_levels": ([i64], i32),
        "rmq_table_levels_ary": ([i64, i32], i32),
        "rmq_query_record_bytes": ([i64], sz),
        "rmq_block_minima": ([v, i64, i32, v, v], i32),
        "rmq_block_minima_keys": ([v, i64, i32, v, v], i32),
        "rmq_sparse_table_build": ([v, i64, i32, v], i32),
        "rmq_sort_endpoints": ([v, v, i64, i64, v, v, v, sz, v], i32),
        "rmq_sort_workspace_bytes": ([i64], sz),
        "rmq_contract": ([v, i64, v, v, i64, v, v, v], i32),
        "rmq_planner_set_table": ([v, i32], i32),
        "rmq_batch_create": ([v, i32, ctypes.POINTER(v)], i32),
        "rmq_batch_run": ([v, i32, i32, v], i32),
        "rmq_batch_item_plan": ([v, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "rmq_batch_item_plan_ex": ([v, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                    ctypes.POINTER(i32)], i32),
        "rmq_batch_workspace_bytes": ([v], sz),
        "rmq_batch_free": ([v], i32),
        "rmq_test_sort_abort": ([i32], i32),
        "rmq_timer_create": ([ctypes.POINTER(v)], i32),
        "rmq_timer_read": ([v, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)], i32),
        "rmq_timer_destroy": ([v], i32),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _LIB = L
    return L


def _check(fn: str, status: int) -> None:
    if status != OK:
        raise RMQError(fn, status)


def _dev_i32(t: torch.Tensor, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.int32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous int32 tensor")
    return t.data_ptr()


def _dev_u64(t: torch.Tensor, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype not in (torch.int64, torch.uint64) or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous 64-bit tensor")
    return t.data_ptr()


def _stream(device: torch.device, stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return int(s.cuda_stream)


class Timer:
    """Per-stage timing of one batch (Table 1's four stages)."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check("rmq_timer_create", lib().rmq_timer_create(ctypes.byref(h)))
        self.handle = h

    def read(self):
        """Wait for the last timed call; returns (stage_ms[4], total_ms)."""
        st = (ctypes.c_float * NUM_STAGES)()
        tot = ctypes.c_float()
        _check("rmq_timer_read", lib().rmq_timer_read(self.handle, st, ctypes.byref(tot)))
        return list(st), tot.value

    def __del__(self):
        if getattr(self, "handle", None) and _LIB is not None:
            _LIB.rmq_timer_destroy(self.handle)
            self.handle = None


def _options(block_size=0, path="auto", bad_count=None, stats=None, workspace=None,
             timer: Optional[Timer] = None, sub_block_size: int = 0,
             arity_log2: int = 0, records: bool = True, sub_block_size2: int = 0) -> _Options:
    o = _Options()
    o.no_query_records = 0 if records else 1
    o.block_size = int(block_size)
    o.sub_block_size = int(sub_block_size)
    o.sub_block_size2 = int(sub_block_size2)
    o.table_arity_log2 = int(arity_log2)
    o.path = PATHS[path] if isinstance(path, str) else int(path)
    o.bad_count = _dev_u64(bad_count, "bad_count") if bad_count is not None else None
    o.stats = _dev_u64(stats, "stats") if stats is not None else None
    if workspace is not None:
        if not workspace.is_cuda or not workspace.is_contiguous():
            raise TypeError("workspace must be a contiguous CUDA tensor")
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    o.timer = timer.handle if timer is not None else None
    return o


class _PlanEntry(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("q", ctypes.c_int64), ("block_size", ctypes.c_int32),
                ("path", ctypes.c_int32), ("sub_block_size", ctypes.c_int32),
                ("one_level_block_size", ctypes.c_int32)]


class _BatchItem(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("n", ctypes.c_int64), ("L", ctypes.c_void_p),
                ("R", ctypes.c_void_p), ("q", ctypes.c_int64), ("out", ctypes.c_void_p),
                ("block_size", ctypes.c_int32), ("path", ctypes.c_int32)]


def set_plan_table(entries) -> None:
    """Install measured plans: iterable of (n, q, block_size, path name) or
    (n, q, block_size, path name, sub_block_size, one_level_block_size); a
    sub_block_size > 0 is a two-level plan (Section 3.3).  An empty iterable
    restores the built-in rule."""
    entries = list(entries)
    arr = (_PlanEntry * max(len(entries), 1))()
    for i, e in enumerate(entries):
        n, q, k, p = e[:4]
        k1, k_one = (e[4], e[5]) if len(e) > 4 else (0, 0)
        arr[i] = _PlanEntry(int(n), int(q), int(k), PATHS[p] if isinstance(p, str) else int(p),
                            int(k1), int(k_one))
    _check("rmq_planner_set_table", lib().rmq_planner_set_table(arr, len(entries)))


TUNE_TABLE = os.path.join(HERE, "tune_table.json")


def load_plan_table(path: str = TUNE_TABLE) -> bool:
    """Install the autotuner's table if it exists; returns whether it did."""
    import json

    if not os.path.exists(path):
        return False
    with open(path) as f:
        data = json.load(f)
    set_plan_table((e["n"], e["q"], e["block_size"], e["path"], e.get("sub_block_size", 0),
                    e.get("one_level_block_size", 0)) for e in data["entries"])
    return True


def test_sort_abort(on: bool) -> None:
    """For tests of the failure report only: every later device sort starts
    as if a bounded wait had run out (rmq_test_sort_abort)."""
    _check("rmq_test_sort_abort", lib().rmq_test_sort_abort(1 if on else 0))


def version() -> str:
    return lib().rmq_version().decode()


def plan(n: int, q: int):
    """(block_size, path name) the planner picks for (n, q) among one-level
    plans."""
    k, p = ctypes.c_int32(), ctypes.c_int32()
    _check("rmq_plan", lib().rmq_plan(n, q, ctypes.byref(k), ctypes.byref(p)))
    return k.value, {v: k_ for k_, v in PATHS.items()}[p.value]


def plan_ex(n: int, q: int):
    """(block_size, path name, sub_block_size) of a path="auto" call without
    block sizes; sub_block_size > 0 means two block levels."""
    k, p, k1 = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check("rmq_plan_ex", lib().rmq_plan_ex(n, q, ctypes.byref(k), ctypes.byref(p),
                                            ctypes.byref(k1)))
    return k.value, {v: k_ for k_, v in PATHS.items()}[p.value], k1.value


def default_block(n: int, q: int, path: str) -> int:
    """Block size a call with block_size=0 uses on the given path."""
    return int(lib().rmq_default_block(n, q, PATHS[path]))


def default_sub_block(n: int, q: int, path: str) -> int:
    """Sub-block size a call with block_size=0 and sub_block_size=0 uses on
    the given path (0: one block level)."""
    return int(lib().rmq_default_sub_block(n, q, PATHS[path]))


def workspace_bytes(n: int, q: int, path="auto", block_size: int = 0,
                    sub_block_size: int = 0, arity_log2: int = 0, records: bool = True,
                    sub_block_size2: int = 0) -> int:
    o = _options(block_size, path, sub_block_size=sub_block_size, arity_log2=arity_log2,
                 records=records, sub_block_size2=sub_block_size2)
    return int(lib().rmq_workspace_bytes(n, q, ctypes.byref(o)))


def index_bytes(n: int, block_size: int) -> int:
    return int(lib().rmq_index_bytes(n, block_size))


def build_bytes(n: int, block_size: int = 0, sub_block_size: int = 0, arity_log2: int = 0,
                records: bool = True) -> int:
    """Device bytes Index(A, ...) of n elements allocates (0: invalid)."""
    o = _options(block_size, "full", sub_block_size=sub_block_size, arity_log2=arity_log2,
                 records=records)
    return int(lib().rmq_build_bytes(n, ctypes.byref(o)))


def query_record_bytes(num_blocks: int) -> int:
    """Bytes of the query records kept beside a doubling table of
    num_blocks blocks (0 if none)."""
    return int(lib().rmq_query_record_bytes(num_blocks))


def table_levels(num_blocks: int, arity_log2: int = 0) -> int:
    """Levels of the block table: doubling, or over powers of
    l = 2^arity_log2 (Section 3.1)."""
    if arity_log2 <= 1:
        return int(lib().rmq_table_levels(num_blocks))
    return int(lib().rmq_table_levels_ary(num_blocks, arity_log2))


def query_batch(A: torch.Tensor, L: torch.Tensor, R: torch.Tensor, *, path="auto",
                block_size: int = 0, sub_block_size: int = 0, arity_log2: int = 0,
                out: Optional[torch.Tensor] = None, bad_count=None, stats=None, workspace=None,
                timer: Optional[Timer] = None, stream=None, records: bool = True,
                sub_block_size2: int = 0) -> torch.Tensor:
    """Answer all queries of one offline batch (Section 1); returns int32 out.
    sub_block_size > 0 selects two block levels (Section 3.3), and
    sub_block_size2 > 0 a third (plain method); arity_log2 in 2..5 builds the
    block table over powers of l = 2^arity_log2 instead of 2 (Section 3.1)."""
    n, q = A.numel(), L.numel()
    if R.numel() != q:
        raise ValueError("L and R differ in length")
    if out is None:
        out = torch.empty(q, dtype=torch.int32, device=A.device)
    o = _options(block_size, path, bad_count, stats, workspace, timer, sub_block_size,
                 arity_log2, records, sub_block_size2)
    st = lib().rmq_query_batch_ex(_dev_i32(A, "A"), n, _dev_i32(L, "L") if q else None,
                                  _dev_i32(R, "R") if q else None, q,
                                  _dev_i32(out, "out") if q else None,
                                  _stream(A.device, stream), ctypes.byref(o))
    _check("rmq_query_batch_ex", st)
    return out


# Bytes of the fixed device scratch array behind query_batch_noalloc.
NOALLOC_SCRATCH_BYTES = 128 << 20


def query_batch_noalloc(A: torch.Tensor, L: torch.Tensor, R: torch.Tensor, out: torch.Tensor,
                        *, path="auto", block_size: int = 0, sub_block_size: int = 0,
                        arity_log2: int = 0, bad_count=None, stats=None, stream=None,
                        records: bool = True, sub_block_size2: int = 0) -> torch.Tensor:
    """query_batch through rmq_query_batch_noalloc: the scratch is the
    library's fixed device array, so the call allocates nothing (out must be
    given).  Raises RMQError (status 6) when the batch needs more scratch
    than NOALLOC_SCRATCH_BYTES.  Calls overlapping on one device race."""
    n, q = A.numel(), L.numel()
    if R.numel() != q or out.numel() != q:
        raise ValueError("L, R and out differ in length")
    o = _options(block_size, path, bad_count, stats, None, None, sub_block_size, arity_log2,
                 records, sub_block_size2)
    st = lib().rmq_query_batch_noalloc(_dev_i32(A, "A"), n, _dev_i32(L, "L") if q else None,
                                       _dev_i32(R, "R") if q else None, q,
                                       _dev_i32(out, "out") if q else None,
                                       _stream(A.device, stream), ctypes.byref(o))
    _check("rmq_query_batch_noalloc", st)
    return out


class Index:
    """Resident block Sparse Table of A (Section 3.2) for repeated batches,
    with the k1-block minima too when sub_block_size > 0 (Section 3.3), and
    the table over powers of l = 2^arity_log2 when arity_log2 > 1 (Section
    3.1).  Keeps a reference to A, which partial-block scans read."""

    def __init__(self, A: torch.Tensor, block_size: int = 0, stream=None,
                 sub_block_size: int = 0, arity_log2: int = 0, records: bool = True):
        h = ctypes.c_void_p()
        o = _options(block_size, "full", sub_block_size=sub_block_size, arity_log2=arity_log2,
                     records=records)
        _check("rmq_build", lib().rmq_build(_dev_i32(A, "A"), A.numel(), ctypes.byref(o),
                                            _stream(A.device, stream), ctypes.byref(h)))
        self.handle = h
        self.A = A
        n, k, nb, lv, by = (ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64(),
                            ctypes.c_int32(), ctypes.c_size_t())
        _check("rmq_index_info", lib().rmq_index_info(h, ctypes.byref(n), ctypes.byref(k),
                                                      ctypes.byref(nb), ctypes.byref(lv),
                                                      ctypes.byref(by)))
        self.n, self.block_size, self.num_blocks = n.value, k.value, nb.value
        self.levels, self.bytes = lv.value, by.value

    def query(self, L: torch.Tensor, R: torch.Tensor, out: Optional[torch.Tensor] = None,
              bad_count=None, stats=None, stream=None) -> torch.Tensor:
        q = L.numel()
        if out is None:
            out = torch.empty(q, dtype=torch.int32, device=self.A.device)
        o = _options(0, "full", bad_count, stats)
        _check("rmq_query_index_ex", lib().rmq_query_index_ex(
            self.handle, _dev_i32(L, "L") if q else None, _dev_i32(R, "R") if q else None, q,
            _dev_i32(out, "out") if q else None, _stream(self.A.device, stream), ctypes.byref(o)))
        return out

    def table(self, stream=None) -> torch.Tensor:
        """The Sparse Table as a (levels, num_blocks) int64 tensor of keys."""
        st = torch.empty(self.levels * self.num_blocks, dtype=torch.int64, device=self.A.device)
        _check("rmq_index_copy_table", lib().rmq_index_copy_table(
            self.handle, st.data_ptr(), _stream(self.A.device, stream)))
        return st.view(self.levels, self.num_blocks)

    def free(self) -> None:
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.A.device)
            _check("rmq_index_free", lib().rmq_index_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---- single stages ----------------------------------------------------------
def block_minima(A: torch.Tensor, block_size: int, stream=None) -> torch.Tensor:
    nb = (A.numel() + block_size - 1) // block_size
    keys = torch.empty(nb, dtype=torch.int64, device=A.device)
    _check("rmq_block_minima", lib().rmq_block_minima(_dev_i32(A, "A"), A.numel(), block_size,
                                                      keys.data_ptr(), _stream(A.device, stream)))
    return keys


def block_minima_keys(S: torch.Tensor, block_size: int, stream=None) -> torch.Tensor:
    nb = (S.numel() + block_size - 1) // block_size
    keys = torch.empty(nb, dtype=torch.int64, device=S.device)
    _check("rmq_block_minima_keys", lib().rmq_block_minima_keys(
        _dev_u64(S, "src"), S.numel(), block_size, keys.data_ptr(), _stream(S.device, stream)))
    return keys


def sparse_table(level0: torch.Tensor, levels: Optional[int] = None, stream=None) -> torch.Tensor:
    """(levels, nb) table built on the device from its level 0."""
    nb = level0.numel()
    levels = table_levels(nb) if levels is None else levels
    st = torch.empty(levels * nb, dtype=torch.int64, device=level0.device)
    st[:nb].copy_(level0)
    _check("rmq_sparse_table_build", lib().rmq_sparse_table_build(
        st.data_ptr(), nb, levels, _stream(level0.device, stream)))
    return st.view(levels, nb)


def sort_endpoints(L: torch.Tensor, R: torch.Tensor, n: int, stream=None):
    """Sorted (position, tag) endpoint list of Section 3.1 step 1."""
    q = L.numel()
    pos = torch.empty(2 * q, dtype=torch.int32, device=L.device)
    tag = torch.empty(2 * q, dtype=torch.int32, device=L.device)
    wsb = int(lib().rmq_sort_workspace_bytes(q))
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=L.device)
    _check("rmq_sort_endpoints", lib().rmq_sort_endpoints(
        _dev_i32(L, "L"), _dev_i32(R, "R"), q, n, _dev_i32(pos, "pos"), _dev_i32(tag, "tag"),
        ws.data_ptr(), wsb, _stream(L.device, stream)))
    return pos, tag


def contract(A: torch.Tensor, pos: torch.Tensor, tag: torch.Tensor, stream=None):
    """Remapped ranges (Lc, Rc) and A_Q keys of Section 3.1 steps 1-2."""
    q = pos.numel() // 2
    LR = torch.empty(2 * q, dtype=torch.int32, device=A.device)
    aq = torch.empty(max(2 * q - 1, 0), dtype=torch.int64, device=A.device)
    if q:
        _check("rmq_contract", lib().rmq_contract(
            _dev_i32(A, "A"), A.numel(), _dev_i32(pos, "pos"), _dev_i32(tag, "tag"), q,
            _dev_i32(LR, "LR"), aq.data_ptr(), _stream(A.device, stream)))
    return LR[0::2], LR[1::2], aq


class LCA:
    """Lowest common ancestors through RMQ (Section 1): the Euler tour of the
    tree given by `parent` (int32 on the device, parent[root] = -1) and an
    RMQ index over its depths, built on the device."""

    def __init__(self, parent: torch.Tensor, block_size: int = 0, sub_block_size: int = 0,
                 stream=None, arity_log2: int = 0, records: bool = True):
        h = ctypes.c_void_p()
        o = _options(block_size, "full", sub_block_size=sub_block_size, arity_log2=arity_log2,
                     records=records)
        _check("rmq_lca_build", lib().rmq_lca_build(_dev_i32(parent, "parent"), parent.numel(),
                                                    ctypes.byref(o),
                                                    _stream(parent.device, stream),
                                                    ctypes.byref(h)))
        self.handle = h
        self.device = parent.device
        self.num_nodes = parent.numel()
        by = ctypes.c_size_t()
        _check("rmq_lca_info", lib().rmq_lca_info(h, None, ctypes.byref(by)))
        self.bytes = by.value

    def query(self, u: torch.Tensor, v: torch.Tensor, out: Optional[torch.Tensor] = None,
              bad_count=None, stream=None) -> torch.Tensor:
        q = u.numel()
        if v.numel() != q:
            raise ValueError("u and v differ in length")
        if out is None:
            out = torch.empty(q, dtype=torch.int32, device=self.device)
        o = _options(0, "full", bad_count)
        _check("rmq_lca_query", lib().rmq_lca_query(
            self.handle, _dev_i32(u, "u") if q else None, _dev_i32(v, "v") if q else None, q,
            _dev_i32(out, "out") if q else None, _stream(self.device, stream), ctypes.byref(o)))
        return out

    def tour(self, stream=None):
        """(depth, node, first) of the Euler tour, copied to new tensors."""
        N = self.num_nodes
        depth = torch.empty(2 * N - 1, dtype=torch.int32, device=self.device)
        node = torch.empty(2 * N - 1, dtype=torch.int32, device=self.device)
        first = torch.empty(N, dtype=torch.int32, device=self.device)
        _check("rmq_lca_copy_tour", lib().rmq_lca_copy_tour(
            self.handle, depth.data_ptr(), node.data_ptr(), first.data_ptr(),
            _stream(self.device, stream)))
        return depth, node, first

    def free(self) -> None:
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            _check("rmq_lca_free", lib().rmq_lca_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Batch:
    """Many arrays, each with its own query batch (rmq_batch_* in rmq.h).
    `arrays`: int32 CUDA tensors; `queries`: (L, R) pairs; `outs`: optional
    int32 outputs.  Keeps references to every tensor it was given."""

    def __init__(self, arrays, queries, outs=None, block_sizes=None, paths=None):
        count = len(arrays)
        if len(queries) != count:
            raise ValueError("one (L, R) pair per array")
        if outs is None:
            outs = [torch.empty(L.numel(), dtype=torch.int32, device=A.device)
                    for A, (L, _) in zip(arrays, queries)]
        self.arrays, self.queries, self.outs = list(arrays), list(queries), list(outs)
        items = (_BatchItem * count)()
        for i, (A, (L, R), out) in enumerate(zip(self.arrays, self.queries, self.outs)):
            q = L.numel()
            items[i] = _BatchItem(
                _dev_i32(A, "A"), A.numel(), _dev_i32(L, "L") if q else None,
                _dev_i32(R, "R") if q else None, q, _dev_i32(out, "out") if q else None,
                int(block_sizes[i]) if block_sizes else 0,
                PATHS[paths[i]] if paths else 0)
        h = ctypes.c_void_p()
        _check("rmq_batch_create", lib().rmq_batch_create(items, count, ctypes.byref(h)))
        self.handle = h
        self.device = self.arrays[0].device

    MODES = {"fused": 0, "per_item": 1}

    def run(self, mode: str = "fused", graph: bool = False, stream=None):
        """Enqueue one run; `graph` replays a captured hipGraph (needs a
        non-default stream)."""
        s = _stream(self.device, stream)
        _check("rmq_batch_run", lib().rmq_batch_run(self.handle, self.MODES[mode],
                                                    1 if graph else 0, s))
        return self.outs

    def plan(self, i: int):
        k, p = ctypes.c_int32(), ctypes.c_int32()
        _check("rmq_batch_item_plan", lib().rmq_batch_item_plan(self.handle, i, ctypes.byref(k),
                                                                ctypes.byref(p)))
        return k.value, {v: k_ for k_, v in PATHS.items()}[p.value]

    def plan_ex(self, i: int):
        """(block_size, path name, sub_block_size) of item i; sub_block_size
        > 0 means two block levels."""
        k, p, k1 = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check("rmq_batch_item_plan_ex", lib().rmq_batch_item_plan_ex(
            self.handle, i, ctypes.byref(k), ctypes.byref(p), ctypes.byref(k1)))
        return k.value, {v: k_ for k_, v in PATHS.items()}[p.value], k1.value

    def workspace_bytes(self) -> int:
        return int(lib().rmq_batch_workspace_bytes(self.handle))

    def free(self) -> None:
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            _check("rmq_batch_free", lib().rmq_batch_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
