"""Statistical pins (Sec. 5): chi-square over all 120 orderings at n = 5 and
the Mallows-kernel MMD test.

The paper reports, without printing the plotted values, that VariablePhilox
fails the n = 5 chi-square test below 20 rounds and passes at 24, and that the
MMD test with the normal threshold agrees.  Those outcomes pin the oracle's
cipher as a whole.  The closed forms for E[K] and Var K are checked against
brute force over S_n, and the test machinery itself against numpy's own
permutation generator (which must pass).

Seed blocks are fixed (seeds 1..100000 unless stated), so each statistic is
deterministic.  The MMD assertions use alpha = 0.01 on those blocks; the
first block at 24 rounds sits at z = +2.29, inside alpha = 0.01 but outside
0.05, while the next block sits at z = +1.13.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import stats

P = 100_000


def _perms(n, rounds, first_seed=1, count=P):
    return oracle.permutations(n, np.arange(first_seed, first_seed + count, dtype=np.uint64), rounds)


# ------------------------------------------------------- closed forms ----
@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_expected_kernel_closed_form_matches_enumeration(n):
    assert math.isclose(stats.expected_kernel(n), stats.expected_kernel_brute(n), rel_tol=1e-12)
    assert math.isclose(stats.expected_kernel(n, 10.0), stats.expected_kernel_brute(n, 10.0), rel_tol=1e-12)


def test_kernel_variance_matches_enumeration():
    import itertools

    n = 5
    c = n * (n - 1) / 2
    ks = []
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        ks.append(math.exp(-stats.LAMBDA * inv / c))
    assert math.isclose(stats.kernel_variance(n), float(np.var(ks)), rel_tol=1e-12)


def test_discordant_pairs_merge_equals_brute():
    rng = np.random.default_rng(0)
    for n in (2, 3, 10, 57, 200):
        for _ in range(20):
            a, b = rng.permutation(n), rng.permutation(n)
            assert oracle.discordant_pairs(a, b) == oracle.discordant_pairs(a, b, brute=True)
    # reversal is discordant on every pair
    n = 30
    assert oracle.discordant_pairs(np.arange(n), np.arange(n)[::-1]) == n * (n - 1) // 2


def test_lehmer_index_is_a_bijection_on_s5():
    import itertools

    perms = np.array(list(itertools.permutations(range(5))))
    idx = stats.lehmer_index(perms)
    assert sorted(idx.tolist()) == list(range(120))
    assert idx[0] == 0 and idx[-1] == 119


# ----------------------------------------------------------- controls ----
def test_numpy_permutations_pass_both_tests():
    rng = np.random.default_rng(20210611)
    perms = np.stack([rng.permutation(5) for _ in range(P)])
    chi, dof = stats.chi_square(perms)
    assert chi < stats.chi_square_critical(dof, 0.05)
    m = stats.mmd2(perms)
    assert abs(m) < stats.normal_threshold(5, P, 0.01)


def test_identity_sample_fails_mmd():
    perms = np.tile(np.arange(100, dtype=np.uint32), (1000, 1))
    m = stats.mmd2(perms)
    assert m > stats.hoeffding_threshold(1000, 0.05)


# ------------------------------------------------- paper's outcomes ----
def test_chi_square_critical_value():
    assert stats.chi_square_critical(119, 0.05) == pytest.approx(145.46, abs=0.01)


@pytest.mark.parametrize("rounds", [4, 8, 12, 16])
def test_chi_square_fails_below_twenty_rounds(rounds):
    chi, dof = stats.chi_square(_perms(5, rounds))
    assert chi > stats.chi_square_critical(dof, 0.05)


@pytest.mark.parametrize("rounds", [24, 32])
def test_chi_square_passes_at_24_rounds_and_above(rounds):
    chi, dof = stats.chi_square(_perms(5, rounds))
    assert chi < stats.chi_square_critical(dof, 0.05)


@pytest.mark.parametrize("first_seed", [1, 100_001])
def test_mmd_n5_passes_at_24_rounds(first_seed):
    m = stats.mmd2(_perms(5, 24, first_seed))
    assert abs(m) < stats.normal_threshold(5, P, 0.01)
    assert abs(m) < stats.hoeffding_threshold(P, 0.05)


def test_mmd_n5_fails_at_4_rounds():
    m = stats.mmd2(_perms(5, 4))
    assert abs(m) > stats.normal_threshold(5, P, 0.05)
    assert stats.mmd_z(5, m, P) > 50


@pytest.mark.slow
def test_mmd_n100_pass_at_24_fail_at_4():
    m24 = stats.mmd2(_perms(100, 24))
    assert abs(m24) < stats.normal_threshold(100, P, 0.01)
    m4 = stats.mmd2(_perms(100, 4))
    assert abs(m4) > stats.normal_threshold(100, P, 0.05)
