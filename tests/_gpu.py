"""Helpers for the GPU parity tests: device transfer, reference answers from
the CPU oracle, and named input families."""
from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

import workloads as W

INT_MIN = np.iinfo(np.int32).min
INT_MAX = np.iinfo(np.int32).max


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def say(*a):
    """Name the case on stdout before touching the GPU (flushed)."""
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(a: np.ndarray, device) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy()


def reference(orc, A, L, R):
    """Oracle answers: the linear scan when the total scan length is small,
    else the block Sparse Table over 32-element blocks (both pinned)."""
    lens = (R.astype(np.int64) - L.astype(np.int64) + 1).clip(0)
    if lens.sum() <= 5e8:
        return orc.rmq_scan(A, L, R)
    return orc.rmq_sparse_table(A, L, R, 32)


def arrays(n: int, seed: int):
    """Named value families for A."""
    rng = np.random.default_rng(seed)
    yield "uniform31", W.uniform_int31(n, seed)
    yield "ties8", rng.integers(0, 8, n).astype(np.int32)
    yield "equal", np.full(n, 3, dtype=np.int32)
    yield "increasing", np.arange(n, dtype=np.int32)
    yield "decreasing", (n - np.arange(n)).astype(np.int32)
    yield "pm1_walk", np.cumsum(rng.choice(np.array([-1, 1], dtype=np.int32), n)).astype(np.int32)
    yield "extremes", rng.choice(np.array([INT_MIN, INT_MAX, 0, -1], dtype=np.int64), n).astype(np.int32)


def query_sets(n: int, k: int, q: int, seed: int):
    """Named query families over [0, n), including block-aligned edges."""
    L, R = W.uniform_queries(n, q, seed)
    yield "uniform", L, R
    sl, sr = W.short_queries(n, q, seed, 5, max(1, min(n, 64)))
    yield "short", sl, sr
    p = W.uniform_index(n, q, seed, 9).astype(np.int32)
    yield "point", p, p.copy()
    # endpoints on block boundaries, adjacent blocks, whole array
    nb = (n + k - 1) // k
    b = W.uniform_index(nb, q, seed, 11)
    lo = np.minimum(b * k, n - 1)
    hi = np.minimum((b + 1) * k - 1, n - 1)
    hi2 = np.minimum((b + 2) * k - 1, n - 1)
    yield "block_exact", lo.astype(np.int32), hi.astype(np.int32)
    yield "two_blocks", np.minimum(lo + k // 2, n - 1).astype(np.int32), hi2.astype(np.int32)
    yield "edges", np.array([0, 0, n - 1, 0], dtype=np.int32), \
        np.array([n - 1, 0, n - 1, min(n - 1, k)], dtype=np.int32)
