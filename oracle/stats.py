"""Statistical tests on samples of permutations (TEST INFRASTRUCTURE ONLY).

Sec. 5 of the paper: a chi-square test over all orderings at n = 5, and a
one-sample maximum-mean-discrepancy test with the Mallows kernel
K(s, s') = exp(-lambda * n_dis(s, s') / C(n, 2)), lambda = 5.

Under the uniform distribution E[K(s, s')] has a closed form (a product over
j = 1..n), E[K^2] is the same product at 2*lambda, and the MMD^2 estimate over
disjoint consecutive pairs of the sample has mean 0 and variance
2 Var(K) / |Pi|.  Acceptance regions: Hoeffding, |MMD^2| < sqrt(log(2/a)/|Pi|);
central limit, |MMD^2| < sqrt(2 Var(MMD^2)) * erfinv(1 - a).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy import special, stats

from . import pair_discordances

LAMBDA = 5.0


# ------------------------------------------------------------ chi-square --
def lehmer_index(perms: np.ndarray) -> np.ndarray:
    """Map each row (a permutation of 0..n-1) to its rank in 0..n!-1."""
    perms = np.asarray(perms, dtype=np.int64)
    p, n = perms.shape
    idx = np.zeros(p, dtype=np.int64)
    for i in range(n):
        smaller_after = (perms[:, i + 1 :] < perms[:, i : i + 1]).sum(axis=1)
        idx = idx * (n - i) + smaller_after
    return idx


def chi_square(perms: np.ndarray) -> tuple[float, int]:
    """Pearson chi-square of the ordering counts against the uniform law.

    Returns (statistic, degrees of freedom = n! - 1)."""
    n = perms.shape[1]
    cells = math.factorial(n)
    counts = np.bincount(lehmer_index(perms), minlength=cells).astype(np.float64)
    expected = perms.shape[0] / cells
    return float(((counts - expected) ** 2 / expected).sum()), cells - 1


def chi_square_critical(dof: int, alpha: float = 0.05) -> float:
    return float(stats.chi2.ppf(1.0 - alpha, dof))


# ------------------------------------------------------------------- MMD --
def expected_kernel(n: int, lam: float = LAMBDA) -> float:
    """E[K(I, s)] for s uniform on S_n: prod_j (1 - e^{-lam j/C}) / (j (1 - e^{-lam/C}))."""
    if n < 2:
        return 1.0
    c = n * (n - 1) / 2.0
    j = np.arange(1, n + 1, dtype=np.float64)
    # log-domain product, expm1 for accuracy when lam/C is small
    terms = np.log(-np.expm1(-lam * j / c)) - np.log(j) - math.log(-math.expm1(-lam / c))
    return float(np.exp(terms.sum()))


def expected_kernel_brute(n: int, lam: float = LAMBDA) -> float:
    """E[K(I, s)] by enumerating S_n (small n only)."""
    c = n * (n - 1) / 2.0
    total = 0.0
    count = 0
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        total += math.exp(-lam * inv / c)
        count += 1
    return total / count


def kernel_variance(n: int, lam: float = LAMBDA) -> float:
    """Var K = E[K^2] - E[K]^2, with E[K^2] the closed form at 2*lam."""
    return expected_kernel(n, 2 * lam) - expected_kernel(n, lam) ** 2


def mmd2(perms: np.ndarray, lam: float = LAMBDA) -> float:
    """Unbiased one-sample MMD^2 estimate: mean over pairs (2i, 2i+1) of
    K(Pi_2i, Pi_2i+1), minus E[K] under the uniform law."""
    p, n = perms.shape
    if p % 2:
        raise ValueError("|Pi| must be even")
    c = n * (n - 1) / 2.0
    ndis = pair_discordances(perms).astype(np.float64)
    return float(np.exp(-lam * ndis / c).mean() - expected_kernel(n, lam))


def hoeffding_threshold(sample_size: int, alpha: float) -> float:
    return math.sqrt(math.log(2.0 / alpha) / sample_size)


def normal_threshold(n: int, sample_size: int, alpha: float, lam: float = LAMBDA) -> float:
    var_mmd = 2.0 * kernel_variance(n, lam) / sample_size
    return math.sqrt(2.0 * var_mmd) * float(special.erfinv(1.0 - alpha))


def mmd_z(n: int, value: float, sample_size: int, lam: float = LAMBDA) -> float:
    """The estimate in standard deviations of its null distribution."""
    return value / math.sqrt(2.0 * kernel_variance(n, lam) / sample_size)
