"""Shared test helpers: oracle slices of large shuffles, computed in parallel
threads (the oracle itself stays sequential; ctypes releases the GIL)."""
from __future__ import annotations

import concurrent.futures
import os

import numpy as np

import oracle

THREADS = min(16, os.cpu_count() or 1)


def kept_before(n: int, seed: int, rounds: int, i: int) -> int:
    """Number of kept padded indices below i (the rank of the first output
    produced at or after i), split across threads."""
    if i == 0:
        return 0
    chunks = max(1, min(THREADS * 4, i // 65536))
    bounds = np.linspace(0, i, chunks + 1, dtype=np.int64)
    with concurrent.futures.ThreadPoolExecutor(THREADS) as ex:
        parts = ex.map(lambda ab: oracle.count_kept(n, seed, rounds, int(ab[0]), int(ab[1])),
                       zip(bounds[:-1], bounds[1:]))
        return int(sum(parts))


def oracle_window(x: np.ndarray, seed: int, rounds: int, i_begin: int, i_end: int) -> tuple[int, np.ndarray]:
    """(first output position, oracle outputs) for padded indices [i_begin, i_end)."""
    n = x.shape[0]
    rank = kept_before(n, seed, rounds, i_begin)
    return rank, oracle.shuffle_window(x, seed, rounds, i_begin, i_end)


def kept_before_fast(n: int, seed: int, rounds: int, i: int) -> int:
    """Same as kept_before, counting from whichever end of the domain is nearer."""
    domain = 1 << oracle.domain_bits(n)
    if i > domain // 2:
        rest = domain - i
        chunks = max(1, min(THREADS * 4, rest // 65536))
        bounds = np.linspace(i, domain, chunks + 1, dtype=np.int64)
        with concurrent.futures.ThreadPoolExecutor(THREADS) as ex:
            parts = ex.map(lambda ab: oracle.count_kept(n, seed, rounds, int(ab[0]), int(ab[1])),
                           zip(bounds[:-1], bounds[1:]))
            return n - int(sum(parts))
    return kept_before(n, seed, rounds, i)


def check_slices(x_np: np.ndarray, y_np: np.ndarray, seed: int, rounds: int, starts, span: int = 1 << 20):
    """Compares the GPU output y with the oracle on padded-index slices."""
    n = x_np.shape[0]
    for s in starts:
        rank = kept_before_fast(n, seed, rounds, s)
        want = oracle.shuffle_window(x_np, seed, rounds, s, s + span)
        got = y_np[rank:rank + len(want)]
        assert np.array_equal(got, want), (n, s)


def oracle_whole(x_np: np.ndarray, seed: int, rounds: int, chunks: int = 64) -> np.ndarray:
    """The oracle's whole output, its padded domain split into `chunks`
    consecutive windows run on parallel threads and concatenated in order
    (each window's outputs are the ranks that follow the previous window's)."""
    n = x_np.shape[0]
    domain = 1 << oracle.domain_bits(n)
    bounds = np.linspace(0, domain, chunks + 1, dtype=np.int64)
    with concurrent.futures.ThreadPoolExecutor(THREADS) as ex:
        parts = list(ex.map(lambda ab: oracle.shuffle_window(x_np, seed, rounds, int(ab[0]), int(ab[1])),
                            zip(bounds[:-1], bounds[1:])))
    out = np.concatenate(parts)
    assert out.shape[0] == n
    return out
