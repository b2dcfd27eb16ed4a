"""Seeded synthetic inputs for batched range-minimum queries.

This module only draws inputs: arrays, query endpoints, batch sizes and
trees.  It holds none of the arithmetic of the query method itself, and both
the CPU oracle and the GPU library are fed from the same bytes it produces.

Random numbers come from a counter-based generator: the SplitMix64 output
function (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) applied to

    x(seed, stream, i) = (seed XOR stream * 0xD1B54A32D192ED03) + (i + 1) * 0x9E3779B97F4A7C15

so draw i of a stream is independent of how many draws precede it and can be
regenerated piecewise.  Derived draws:

* value in [0, 2^31):  h >> 33
* index in [0, m):     ((h >> 32) * m) >> 32          (Lemire's multiply-shift)
* unit float in [0,1): (h >> 11) * 2^-53

Workload shapes follow the experiments section of the paper (uniform query
endpoints drawn over the whole array and swapped when the left one is larger)
and the configurations the library is benchmarked on (uniform int32 values,
short/long query mixes, log-uniform batch sizes, random recursive trees as
parent arrays for the LCA reduction of the introduction).  Tours of those
trees are not drawn here: tests take them from the oracle.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
STREAM_MUL = np.uint64(0xD1B54A32D192ED03)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)

#: base seed; a configuration adds its own number to it
BASE_SEED = 1706069400

_CHUNK = 1 << 22  # draws per numpy chunk, bounds temporary memory


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function, in place on a uint64 array."""
    z ^= z >> np.uint64(30)
    z *= M1
    z ^= z >> np.uint64(27)
    z *= M2
    z ^= z >> np.uint64(31)
    return z


def hashes(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """Draws start .. start+count-1 of (seed, stream) as uint64."""
    out = np.empty(count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        base = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) ^ (np.uint64(stream) * STREAM_MUL)
        for c0 in range(0, count, _CHUNK):
            c1 = min(count, c0 + _CHUNK)
            z = np.arange(start + c0 + 1, start + c1 + 1, dtype=np.uint64)
            z *= GAMMA
            z += base
            out[c0:c1] = _mix(z)
    return out


def hash_one(seed: int, stream: int, i: int) -> int:
    """Scalar form of draw i, for checks and for tiny callers."""
    mask = (1 << 64) - 1
    x = ((seed ^ (stream * 0xD1B54A32D192ED03)) + (i + 1) * 0x9E3779B97F4A7C15) & mask
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & mask
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & mask
    return x ^ (x >> 31)


def _index_from(h: np.ndarray, m) -> np.ndarray:
    """Map uint64 draws to [0, m); m may be a scalar or an array, m <= 2^32."""
    with np.errstate(over="ignore"):
        return ((h >> np.uint64(32)) * np.asarray(m, dtype=np.uint64)) >> np.uint64(32)


def uniform_int31(n: int, seed: int, stream: int = 0) -> np.ndarray:
    """n int32 values uniform in [0, 2^31)."""
    out = np.empty(n, dtype=np.int32)
    for c0 in range(0, n, _CHUNK * 4):
        c1 = min(n, c0 + _CHUNK * 4)
        out[c0:c1] = (hashes(seed, stream, c0, c1 - c0) >> np.uint64(33)).astype(np.int32)
    return out


def uniform_index(m: int, count: int, seed: int, stream: int, start: int = 0) -> np.ndarray:
    """count indices uniform in [0, m), as int64."""
    if m < 1 or m > (1 << 32):
        raise ValueError("m must be in [1, 2^32]")
    return _index_from(hashes(seed, stream, start, count), m).astype(np.int64)


def unit_floats(count: int, seed: int, stream: int) -> np.ndarray:
    """count doubles uniform in [0, 1)."""
    return (hashes(seed, stream, 0, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_queries(n: int, q: int, seed: int, stream: int = 1):
    """q queries with both endpoints uniform over [0, n), swapped so l <= r.

    This is the query distribution of the paper's experiments (0-based here).
    Returns (L, R) as int32 arrays.
    """
    a = uniform_index(n, q, seed, stream)
    b = uniform_index(n, q, seed, stream + 1)
    L = np.minimum(a, b).astype(np.int32)
    R = np.maximum(a, b).astype(np.int32)
    return L, R


def short_queries(n: int, q: int, seed: int, stream: int, max_len: int = 1024):
    """q queries of length uniform in [1, max_len] at uniform start positions."""
    max_len = min(max_len, n)
    length = uniform_index(max_len, q, seed, stream) + 1
    start = _index_from(hashes(seed, stream + 1, 0, q), n - length + 1).astype(np.int64)
    return start.astype(np.int32), (start + length - 1).astype(np.int32)


def permutation(count: int, seed: int, stream: int) -> np.ndarray:
    """A seeded uniform permutation of range(count): argsort of fresh draws."""
    return np.argsort(hashes(seed, stream, 0, count), kind="stable")


def skewed_queries(n: int, q: int, seed: int, stream: int = 1, max_len: int = 1024):
    """Half short queries (length uniform in [1, max_len]), half uniform long
    ones, interleaved by a seeded permutation."""
    qs = q // 2
    Ls, Rs = short_queries(n, qs, seed, stream, max_len)
    Ll, Rl = uniform_queries(n, q - qs, seed, stream + 2)
    L = np.concatenate([Ls, Ll])
    R = np.concatenate([Rs, Rl])
    p = permutation(q, seed, stream + 4)
    return np.ascontiguousarray(L[p]), np.ascontiguousarray(R[p])


def loguniform_ints(count: int, lo: float, hi: float, seed: int, stream: int) -> np.ndarray:
    """count integers log-uniform in [lo, hi] (rounded, clipped to [lo, hi])."""
    u = unit_floats(count, seed, stream)
    v = np.rint(np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo))))
    return np.clip(v, lo, hi).astype(np.int64)


# ------------------------------------------------------------ torch form
# The same draws computed with torch int64 tensor arithmetic (two's-complement
# wrap-around gives the uint64 products mod 2^64; logical shifts are masked
# arithmetic shifts), so large inputs can be drawn where they are used,
# e.g. in device memory.  Bit-identical to the numpy form above.
def _signed(x: int) -> int:
    x &= (1 << 64) - 1
    return x - (1 << 64) if x >= (1 << 63) else x


def _lshr(z, s: int):
    import torch

    return (z >> s) & ((1 << (64 - s)) - 1)


def hashes_torch(seed: int, stream: int, start: int, count: int, device="cpu"):
    import torch

    base = _signed((seed ^ (stream * 0xD1B54A32D192ED03)) & ((1 << 64) - 1))
    z = torch.arange(start + 1, start + count + 1, dtype=torch.int64, device=device)
    z.mul_(_signed(0x9E3779B97F4A7C15)).add_(base)
    z ^= _lshr(z, 30)
    z.mul_(_signed(0xBF58476D1CE4E5B9))
    z ^= _lshr(z, 27)
    z.mul_(_signed(0x94D049BB133111EB))
    z ^= _lshr(z, 31)
    return z


def uniform_int31_torch(n: int, seed: int, stream: int = 0, device="cpu", chunk: int = 1 << 26):
    """uniform_int31 drawn with torch on `device` (identical values)."""
    import torch

    out = torch.empty(n, dtype=torch.int32, device=device)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        out[c0:c1] = _lshr(hashes_torch(seed, stream, c0, c1 - c0, device), 33).to(torch.int32)
    return out


def uniform_queries_torch(n: int, q: int, seed: int, stream: int = 1, device="cpu"):
    """uniform_queries drawn with torch on `device` (identical values)."""
    import torch

    def idx(st):
        return (_lshr(hashes_torch(seed, st, 0, q, device), 32) * n) >> 32

    a, b = idx(stream), idx(stream + 1)
    return torch.minimum(a, b).to(torch.int32), torch.maximum(a, b).to(torch.int32)


# ---------------------------------------------------------------- native part
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libworkloads.so")
        if not os.path.exists(path):
            from . import build as _b

            _b.build()
        lib = ctypes.CDLL(path)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        lib.wl_swap_permutation.argtypes = [p, i64, p, p, i64]
        lib.wl_swap_permutation.restype = None
        _LIB = lib
    return _LIB


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def random_recursive_tree(N: int, seed: int, stream: int = 7) -> np.ndarray:
    """Parent array of a random recursive tree: node 0 is the root and the
    parent of node i >= 1 is uniform in [0, i)."""
    parent = np.empty(N, dtype=np.int32)
    parent[0] = -1
    for c0 in range(1, N, _CHUNK * 4):
        c1 = min(N, c0 + _CHUNK * 4)
        i = np.arange(c0, c1, dtype=np.uint64)
        parent[c0:c1] = _index_from(hashes(seed, stream, c0, c1 - c0), i).astype(np.int32)
    return parent


def lca_queries(first: np.ndarray, q: int, seed: int, stream: int = 9):
    """q LCA queries (u, v uniform over the nodes) and their ranges
    [min(first[u], first[v]), max(...)] over a tour's depth array, where
    `first` (first visit of each node) comes from the caller's tour.
    Returns (u, v, L, R)."""
    N = int(first.shape[0])
    u = uniform_index(N, q, seed, stream)
    v = uniform_index(N, q, seed, stream + 1)
    fu, fv = first[u], first[v]
    return (u.astype(np.int32), v.astype(np.int32),
            np.minimum(fu, fv).astype(np.int32), np.maximum(fu, fv).astype(np.int32))


def paper_permutation(n: int, seed: int, stream: int = 11) -> np.ndarray:
    """The paper's array workload: the increasing sequence 1..n after n/2
    swaps of uniformly drawn position pairs, applied in draw order."""
    a = np.arange(1, n + 1, dtype=np.int32)
    m = n // 2
    done = 0
    while done < m:
        c = min(_CHUNK, m - done)
        i = uniform_index(n, c, seed, stream, done).astype(np.int64)
        j = uniform_index(n, c, seed, stream + 1, done).astype(np.int64)
        _lib().wl_swap_permutation(_ptr(a), n, _ptr(i), _ptr(j), c)
        done += c
    return a
