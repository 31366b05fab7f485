"""Pins for the oracle's LCG bijection (Sec. 3.1): y = (a*x + c) mod 2^k with
a odd is a bijection of [0, 2^k); for a fixed modulus the keyed family holds
at most 2^(k-1) * 2^k permutations; at n = 5 its chi-square is in the region
the paper reports (hundreds of thousands), far above VariablePhilox's."""
import numpy as np

import oracle
from oracle import stats


def test_lcg_is_a_bijection_and_matches_its_definition():
    for n in (5, 16, 17, 1000, 65_537):
        k = oracle.domain_bits(n)
        for seed in (1, 2, 3):
            a, c = oracle.lcg_params(n, seed)
            assert a % 2 == 1 and a < (1 << k) and c < (1 << k)
            out = oracle.lcg_shuffle(np.arange(n, dtype=np.uint32), seed)
            assert np.array_equal(np.sort(out), np.arange(n, dtype=np.uint32))
            # independent restatement: keep the images below n, in index order
            y = (np.arange(1 << k, dtype=np.uint64) * np.uint64(a) + np.uint64(c)) % np.uint64(1 << k)
            assert np.array_equal(out.astype(np.uint64), y[y < n])


def test_lcg_family_is_small():
    k = 4
    tables = {oracle.lcg_shuffle(np.arange(16, dtype=np.uint32), s).tobytes() for s in range(5000)}
    assert len(tables) <= (1 << (k - 1)) * (1 << k)


def test_lcg_chi_square_n5_is_huge():
    perms = oracle.lcg_permutations(5, range(1, 100_001))
    chi, dof = stats.chi_square(perms)
    assert chi > 200_000
    assert chi > 1000 * stats.chi_square_critical(dof, 0.05)
