"""Seeded synthetic inputs (no shuffle arithmetic here).

Both the GPU path and the CPU oracle are fed from these generators, so a
test compares the two on identical bytes.  All randomness comes from numpy's
PCG64 with a fixed seed; the recipes follow the workloads the shuffle is
measured on (arrays of length 2^w + 1 and 2^w, uniform 32-bit payloads,
batches of log-uniform sizes, a Poisson request stream).
"""
from __future__ import annotations

import math

import numpy as np


def arange_u32(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.uint32)


def uniform_u32(n: int, seed: int) -> np.ndarray:
    """n values uniform on [0, 2^32) from PCG64(seed)."""
    return np.random.Generator(np.random.PCG64(seed)).integers(0, 2**32, size=n, dtype=np.uint32)


def normal_records_f32(n: int, width: int, seed: int) -> np.ndarray:
    """n records of `width` float32 values drawn N(0, 1) from PCG64(seed)."""
    g = np.random.Generator(np.random.PCG64(seed))
    return g.standard_normal(size=(n, width), dtype=np.float32)


def random_bytes(nbytes: int, seed: int) -> np.ndarray:
    return np.random.Generator(np.random.PCG64(seed)).integers(0, 256, size=nbytes, dtype=np.uint8)


def log_uniform_sizes(count: int, lo: int, hi: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """`count` sizes floor(exp(U(ln lo, ln hi))) and one 64-bit seed per size,
    both from PCG64(seed) (sizes first, then seeds)."""
    g = np.random.Generator(np.random.PCG64(seed))
    sizes = np.floor(np.exp(g.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)
    seeds = g.integers(0, 2**63, size=count, dtype=np.int64).astype(np.uint64) * np.uint64(2) + g.integers(
        0, 2, size=count, dtype=np.int64
    ).astype(np.uint64)
    return sizes, seeds


def batch(count: int, lo: int, hi: int, seed: int) -> dict:
    """A packed batch: offsets (int64, count+1), per-segment seeds (uint64),
    payload = global arange as uint32."""
    sizes, seeds = log_uniform_sizes(count, lo, hi, seed)
    offsets = np.zeros(count + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    return {"sizes": sizes, "offsets": offsets, "seeds": seeds, "total": int(offsets[-1])}


def request_stream(count: int, lo: int, hi: int, qps: float, seed: int,
                   dtypes=("uint32", "int64", "float32")) -> list[dict]:
    """Serving requests: exponential inter-arrival times at rate qps,
    log-uniform sizes in [lo, hi], a dtype drawn uniformly, a 64-bit seed."""
    g = np.random.Generator(np.random.PCG64(seed))
    gaps = g.exponential(1.0 / qps, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    sizes = np.floor(np.exp(g.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)
    kinds = g.integers(0, len(dtypes), size=count)
    seeds = g.integers(0, 2**63, size=count, dtype=np.int64)
    return [
        {"id": i, "arrival": float(arrivals[i]), "n": int(sizes[i]), "dtype": dtypes[int(kinds[i])],
         "seed": int(seeds[i])}
        for i in range(count)
    ]
