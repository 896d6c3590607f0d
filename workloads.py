"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only builds inputs; it holds none of the shuffle's arithmetic.
The paper evaluates on synthetic 64-bit integers (arXiv 2302.03317, Sec. 6);
these generators produce arrays of the same kind at the sizes the benchmark
and tests use.
"""
from __future__ import annotations

import numpy as np

GOLDEN_GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output for state x + gamma (Steele, Lea, Flood, OOPSLA'14,
    as popularised by Vigna): two xor-shift-multiply rounds and a final
    xor-shift.  Vectorised over a uint64 array."""
    z = (x.astype(np.uint64) + np.uint64(GOLDEN_GAMMA))
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def identity(n: int, elem_bytes: int) -> np.ndarray:
    """Identity-initialised array: element i holds i.

    4 -> uint32, 8 -> uint64, 16 -> (n, 2) uint64 records {key = i,
    payload = splitmix64(i)}."""
    if elem_bytes == 4:
        if n > (1 << 32):
            raise ValueError("uint32 identity needs n <= 2^32")
        return np.arange(n, dtype=np.uint32)
    if elem_bytes == 8:
        return np.arange(n, dtype=np.uint64)
    if elem_bytes == 16:
        rec = np.empty((n, 2), dtype=np.uint64)
        rec[:, 0] = np.arange(n, dtype=np.uint64)
        rec[:, 1] = splitmix64(rec[:, 0])
        return rec
    raise ValueError("elem_bytes must be 4, 8 or 16")


def random_values(n: int, elem_bytes: int, seed: int) -> np.ndarray:
    """Arbitrary (non-identity) contents, for data-independence checks."""
    rng = np.random.default_rng(seed)
    words = max(1, elem_bytes // 8)
    if elem_bytes == 4:
        return rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    arr = rng.integers(0, MASK64, size=(n, words), dtype=np.uint64, endpoint=True)
    return arr[:, 0].copy() if elem_bytes == 8 else arr


def log_uniform_sizes(count: int, lo_log2: int, hi_log2: int, seed: int) -> np.ndarray:
    """Array sizes floor(2^(lo + (hi - lo) * U)) with U uniform in [0, 1)."""
    rng = np.random.default_rng(seed)
    u = rng.random(count)
    return np.floor(np.exp2(lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)


def csr_offsets(sizes: np.ndarray) -> np.ndarray:
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    np.cumsum(sizes, out=off[1:])
    return off


def batched_identity(sizes: np.ndarray) -> np.ndarray:
    """Arrays packed back to back, each identity-initialised (uint32)."""
    total = int(np.sum(sizes))
    out = np.empty(total, dtype=np.uint32)
    pos = 0
    for s in sizes:
        out[pos:pos + s] = np.arange(s, dtype=np.uint32)
        pos += int(s)
    return out


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of `rate` per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def identity_mod32(n: int) -> np.ndarray:
    """uint32 array whose element i holds i mod 2^32 (an identity that wraps,
    for uint32 arrays of more than 2^32 elements)."""
    out = np.empty(n, dtype=np.uint32)
    chunk = 1 << 28
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        out[a:b] = (np.arange(a, b, dtype=np.uint64) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    return out
