"""Pins for the oracle's Algorithm 1 (Sec. 4, "Bijection Shuffle").

The shuffle keeps the padded indices i with f(i) < n and writes
out[rank(i)] = in[f(i)], rank being the exclusive scan of the flags.  The
checks: the output is a permutation of the input; zero rounds reduces to a
plain copy; the compaction of a longer permutation restricted to values < n
is the shorter shuffle (the construction of Sec. 4); batching is a set of
independent single shuffles; the slice helpers agree with the full run.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n", [1, 2, 3, 5, 15, 16, 17, 100, 1000, 4097, 100_000])
@pytest.mark.parametrize("rounds", [1, 4, 24])
def test_output_is_permutation_of_input(n, rounds):
    x = np.arange(n, dtype=np.uint32)
    out = oracle.shuffle(x, 42 + n, rounds)
    assert np.array_equal(np.sort(out), x)


def test_zero_rounds_is_copy():
    for n in (1, 7, 100, 5000):
        x = np.random.default_rng(n).integers(0, 2**32, size=n, dtype=np.uint32)
        assert np.array_equal(oracle.shuffle(x, 3, 0), x)


@pytest.mark.parametrize("eb_dtype,shape", [(np.uint8, ()), (np.uint16, ()), (np.uint32, ()),
                                             (np.uint64, ()), (np.float32, (4,))])
def test_element_sizes_move_whole_records(eb_dtype, shape):
    n = 3000
    rng = np.random.default_rng(5)
    x = rng.integers(0, 200, size=(n,) + shape).astype(eb_dtype)
    out = oracle.shuffle(x, 11, 24)
    perm = oracle.shuffle_sources(n, 11, 24).astype(np.int64)
    assert np.array_equal(out, x[perm])


def test_compaction_of_longer_permutation():
    """Sec. 4: the shuffle of n items is the 2^k-domain permutation with the
    values >= n deleted, for every n sharing the same domain."""
    seed, rounds = 2718, 24
    k = 12
    full = oracle.Cipher(k, seed, rounds).table()
    for n in (2049, 2050, 3000, 4095, 4096):
        assert oracle.domain_bits(n) == k
        want = full[full < n]
        got = oracle.shuffle(np.arange(n, dtype=np.uint32), seed, rounds)
        assert np.array_equal(got, want)


def test_sources_match_shuffle_of_arange():
    for n in (5, 1000, 12345):
        assert np.array_equal(
            oracle.shuffle_sources(n, 9, 24).astype(np.uint32),
            oracle.shuffle(np.arange(n, dtype=np.uint32), 9, 24),
        )


def test_deterministic_and_seed_sensitive():
    x = np.arange(5000, dtype=np.uint32)
    a = oracle.shuffle(x, 1, 24)
    assert np.array_equal(a, oracle.shuffle(x, 1, 24))
    assert not np.array_equal(a, oracle.shuffle(x, 2, 24))
    assert not np.array_equal(a, oracle.shuffle(x, 1, 23))


def test_batched_is_independent_singles():
    rng = np.random.default_rng(3)
    sizes = [0, 1, 5, 100, 257, 4096, 4097, 10000]
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    seeds = rng.integers(0, 2**63, size=len(sizes), dtype=np.uint64)
    x = rng.integers(0, 2**32, size=offsets[-1], dtype=np.uint32)
    out = oracle.shuffle_batched(x, offsets, seeds, 24)
    for s in range(len(sizes)):
        a, b = offsets[s], offsets[s + 1]
        assert np.array_equal(out[a:b], oracle.shuffle(x[a:b], int(seeds[s]), 24))


def test_window_and_count_agree_with_full_run():
    n, seed, rounds = 50_001, 17, 24
    x = np.arange(n, dtype=np.uint32)
    full = oracle.shuffle(x, seed, rounds)
    domain = 1 << oracle.domain_bits(n)
    assert oracle.count_kept(n, seed, rounds, 0, domain) == n
    for lo, hi in [(0, 1000), (30_000, 40_000), (domain - 777, domain)]:
        r = oracle.count_kept(n, seed, rounds, 0, lo)
        win = oracle.shuffle_window(x, seed, rounds, lo, hi)
        assert np.array_equal(win, full[r : r + len(win)])


def test_kept_fraction_matches_padding():
    # Exactly n of the 2^k padded indices are kept, whatever the seed.
    for n in (100_000, 65_537):
        d = 1 << oracle.domain_bits(n)
        for seed in (1, 2):
            assert oracle.count_kept(n, seed, 4, 0, d) == n


def test_golden_outputs_unchanged():
    """Regression pin: digests written by tests/golden/make_golden.py (which
    calls only the oracle).  The paper prints no test vectors, so these pin
    the oracle to itself over time, not to the paper."""
    with open(os.path.join(GOLDEN, "oracle_outputs.json")) as fh:
        golden = json.load(fh)
    for case in golden["cases"]:
        n, seed, rounds = case["n"], case["seed"], case["rounds"]
        out = oracle.shuffle(np.arange(n, dtype=np.uint32), seed, rounds)
        assert hashlib.sha256(out.tobytes()).hexdigest() == case["sha256"], case
        assert out[: len(case["head"])].tolist() == case["head"], case


def test_std_shuffle_reference_is_a_permutation():
    x = np.arange(10_000, dtype=np.uint32)
    y = oracle.std_shuffle_u32(x, 7)
    assert np.array_equal(np.sort(y), x) and not np.array_equal(y, x)
    assert np.array_equal(y, oracle.std_shuffle_u32(x, 7))
