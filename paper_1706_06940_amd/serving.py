"""Serving: resident arrays, continuous batching, latency statistics.

Binding of the native server (rmq_server_* in include/rmq.h) plus the
load-generation helpers used by the tests and the benchmark:

* `Server`: resident block Sparse Tables of device arrays, submit / wait.
* `poisson_schedule`: seeded Poisson arrival times for a list of requests.
* `run_schedule`: submit requests at their arrival times (native load
  generator), wait for all, return per-request latencies and throughput.

The plain per-request form to compare against is the same server with one
slot and one request per batch: every request is its own copy-in, launch and
copy-out, served strictly one after another.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _check, _dev_i32, lib

_i32p = ctypes.POINTER(ctypes.c_int32)


COPY_QUERIES = 1  # queries and answers through device buffers and the copy engines


class _Config(ctypes.Structure):
    _fields_ = [("num_streams", ctypes.c_int32), ("max_tables", ctypes.c_int32),
                ("max_requests_per_batch", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("budget_bytes", ctypes.c_size_t), ("hbm_budget_bytes", ctypes.c_size_t),
                ("sub_block_size", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("queries", ctypes.c_int64),
                ("slot_capacity", ctypes.c_int64), ("max_inflight", ctypes.c_int64),
                ("index_bytes", ctypes.c_size_t), ("hbm_bytes", ctypes.c_size_t)]


class _Info(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_launch", ctypes.c_double),
                ("t_done", ctypes.c_double), ("batch_requests", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _Spec(ctypes.Structure):
    _fields_ = [("table_id", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("L", ctypes.c_void_p), ("R", ctypes.c_void_p), ("q", ctypes.c_int64),
                ("out", ctypes.c_void_p), ("t_arrival", ctypes.c_double)]


# rmq_request_spec as a numpy record (same offsets as _Spec), so that a whole
# schedule's arrival times are set in one vector operation
_SPEC_DTYPE = np.dtype([("table_id", "<i4"), ("reserved", "<i4"), ("L", "<u8"), ("R", "<u8"),
                        ("q", "<i8"), ("out", "<u8"), ("t_arrival", "<f8")])
assert _SPEC_DTYPE.itemsize == ctypes.sizeof(_Spec) and all(
    _SPEC_DTYPE.fields[f][1] == getattr(_Spec, f).offset for f, _ in _Spec._fields_)


_SIGS_DONE = False


def _lib():
    global _SIGS_DONE
    L = lib()
    if not _SIGS_DONE:
        v, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.rmq_server_create.argtypes = [ctypes.POINTER(_Config), ctypes.POINTER(v)]
        L.rmq_server_add_array.argtypes = [v, v, i64, i32, _i32p]
        L.rmq_server_submit.argtypes = [v, i32, v, v, i64, v, ctypes.POINTER(ctypes.c_uint64)]
        L.rmq_server_submit_schedule.argtypes = [v, i32, v, v]
        L.rmq_server_wait.argtypes = [v, ctypes.c_uint64, ctypes.POINTER(_Info)]
        L.rmq_server_stats_get.argtypes = [v, ctypes.POINTER(_Stats)]
        L.rmq_server_clock.argtypes = []
        L.rmq_server_clock.restype = ctypes.c_double
        L.rmq_server_destroy.argtypes = [v]
        for name in ("rmq_server_create", "rmq_server_add_array", "rmq_server_submit",
                     "rmq_server_submit_schedule", "rmq_server_wait", "rmq_server_stats_get",
                     "rmq_server_destroy"):
            getattr(L, name).restype = i32
        _SIGS_DONE = True
    return L


def clock() -> float:
    """The server clock (seconds), shared by every timestamp it reports."""
    return float(_lib().rmq_server_clock())


def _host_i32(a: np.ndarray, name: str) -> np.ndarray:
    if not isinstance(a, np.ndarray) or a.dtype != np.int32 or not a.flags.c_contiguous:
        raise TypeError(f"{name} must be a contiguous int32 numpy array")
    return a


class Server:
    def __init__(self, num_streams: int = 3, max_tables: int = 64,
                 max_requests_per_batch: int = 1024, budget_bytes: int = 256 << 20,
                 copy_queries: bool = False, hbm_budget_bytes: int = 0,
                 sub_block_size: int = 0):
        """budget_bytes: in-flight query buffers (pinned host memory, and as
        much device memory with copy_queries).  hbm_budget_bytes: device
        memory the resident tables and device buffers may take (0: no
        limit); add_array refuses a table beyond it.  sub_block_size > 0:
        every table has two block levels (Section 3.3) with that k1."""
        cfg = _Config(num_streams, max_tables, max_requests_per_batch,
                      COPY_QUERIES if copy_queries else 0, budget_bytes, hbm_budget_bytes,
                      sub_block_size)
        h = ctypes.c_void_p()
        _check("rmq_server_create", _lib().rmq_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self.arrays = []
        self._keep = {}

    def add_array(self, A: torch.Tensor, block_size: int = 0) -> int:
        tid = ctypes.c_int32()
        _check("rmq_server_add_array", _lib().rmq_server_add_array(
            self.handle, _dev_i32(A, "A"), A.numel(), int(block_size), ctypes.byref(tid)))
        self.arrays.append(A)
        return tid.value

    def submit(self, table: int, L: np.ndarray, R: np.ndarray, out: np.ndarray) -> int:
        L, R, out = _host_i32(L, "L"), _host_i32(R, "R"), _host_i32(out, "out")
        t = ctypes.c_uint64()
        _check("rmq_server_submit", _lib().rmq_server_submit(
            self.handle, int(table), L.ctypes.data, R.ctypes.data, L.shape[0], out.ctypes.data,
            ctypes.byref(t)))
        self._keep[t.value] = (L, R, out)
        return t.value

    def submit_schedule(self, requests, arrivals, lead_s: float = 1e-3):
        """requests: list of (table, L, R, out); arrivals: server-clock times.
        The request table is built first; if that took the schedule's start
        closer than lead_s to now, the whole schedule is shifted later by the
        same amount (gaps unchanged), so that no request is submitted behind
        its arrival time because of this set-up.  Returns the tickets and the
        arrival times used."""
        n = len(requests)
        specs = np.zeros(max(n, 1), dtype=_SPEC_DTYPE)
        for i, (tab, L, R, out) in enumerate(requests):
            L, R, out = _host_i32(L, "L"), _host_i32(R, "R"), _host_i32(out, "out")
            specs[i] = (int(tab), 0, L.ctypes.data, R.ctypes.data, L.shape[0], out.ctypes.data, 0.0)
        arr = np.array(arrivals, dtype=np.float64)
        if n:
            arr += max(0.0, clock() + lead_s - float(arr.min()))
            specs["t_arrival"][:n] = arr
        tickets = np.zeros(max(n, 1), dtype=np.uint64)
        _check("rmq_server_submit_schedule",
               _lib().rmq_server_submit_schedule(self.handle, n, specs.ctypes.data,
                                                 tickets.ctypes.data))
        out = [int(t) for t in tickets[:n]]
        for t, r in zip(out, requests):
            self._keep[t] = r
        return out, arr

    def wait(self, ticket: int) -> dict:
        info = _Info()
        _check("rmq_server_wait", _lib().rmq_server_wait(self.handle, ticket, ctypes.byref(info)))
        self._keep.pop(ticket, None)
        return {"t_submit": info.t_submit, "t_launch": info.t_launch, "t_done": info.t_done,
                "batch_requests": info.batch_requests}

    def stats(self) -> dict:
        s = _Stats()
        _check("rmq_server_stats_get", _lib().rmq_server_stats_get(self.handle, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in _Stats._fields_}

    def close(self) -> None:
        if getattr(self, "handle", None):
            _check("rmq_server_destroy", _lib().rmq_server_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def poisson_schedule(count: int, rate: float, seed: int, t0: float) -> np.ndarray:
    """Arrival times of a Poisson process of the given rate (per second),
    starting at t0 on the server clock; exponential gaps from seeded draws."""
    import workloads as W

    u = W.unit_floats(count, seed, 41)
    gaps = -np.log1p(-u) / rate
    return t0 + np.cumsum(gaps)


@dataclass
class RunResult:
    latencies_s: np.ndarray
    queries: int
    makespan_s: float
    mean_batch_requests: float
    queued_s: np.ndarray = None  # arrival -> launch of the request's batch

    def summary(self) -> dict:
        lat = self.latencies_s
        out = {"requests": int(lat.shape[0]), "queries": int(self.queries),
               "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
               "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4),
               "max_ms": round(float(lat.max()) * 1e3, 4),
               "mean_ms": round(float(lat.mean()) * 1e3, 4),
               "queries_per_s": round(self.queries / self.makespan_s, 1),
               "mean_requests_per_batch": round(self.mean_batch_requests, 2)}
        if self.queued_s is not None:
            out["queued_p99_ms"] = round(float(np.percentile(self.queued_s, 99)) * 1e3, 4)
        return out


def run_schedule(server: Server, requests, arrivals) -> RunResult:
    """Submit each request at its arrival time, wait for all; latency =
    completion - arrival (the schedule shifted as a whole past the set-up of
    its request table, see Server.submit_schedule)."""
    tickets, arr = server.submit_schedule(requests, arrivals)
    infos = [server.wait(t) for t in tickets]
    done = np.array([i["t_done"] for i in infos])
    launch = np.array([i["t_launch"] for i in infos])
    q = sum(int(r[1].shape[0]) for r in requests)
    return RunResult(done - arr, q, float(done.max() - arr.min()),
                     float(np.mean([i["batch_requests"] for i in infos])), launch - arr)


def make_requests(ns, count: int, q_lo: float, q_hi: float, seed: int):
    """Requests (table, L, R, out): table uniform over the arrays, q
    log-uniform in [q_lo, q_hi], uniform queries over [0, n_table)."""
    import workloads as W

    tables = W.uniform_index(len(ns), count, seed, 51)
    qs = W.loguniform_ints(count, q_lo, q_hi, seed, 52)
    reqs = []
    for i, (t, q) in enumerate(zip(tables, qs)):
        L, R = W.uniform_queries(int(ns[t]), int(q), seed + 7919 * (i + 1), 53)
        reqs.append((int(t), L, R, np.full(int(q), -2, dtype=np.int32)))
    return reqs
