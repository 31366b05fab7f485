"""The paper's statistical experiments (Sec. 5) with permutations generated
on the GPU: 100,000 shuffles of arange(n) with seeds 1..100,000 in one
batched launch, then chi-square over all 120 orderings at n = 5 and the
Mallows-kernel MMD test at n = 5, 100 and 1,000."""
import numpy as np
import pytest
import torch

import oracle
import paper_2106_06161_amd as bs
from oracle import stats

pytestmark = pytest.mark.gpu

P = 100_000


def gpu_permutations(n, rounds, first_seed=1, count=P):
    x = torch.arange(n, dtype=torch.int32, device="cuda:0").repeat(count)
    off = torch.arange(count + 1, dtype=torch.int64, device="cuda:0") * n
    sd = torch.arange(first_seed, first_seed + count, dtype=torch.int64, device="cuda:0")
    y = bs.shuffle_batched(x, off, sd, rounds)
    torch.cuda.synchronize()
    return y.view(count, n).cpu().numpy().astype(np.uint32)


@pytest.mark.parametrize("rounds,passes", [(16, False), (24, True)])
def test_chi_square_n5(rounds, passes):
    perms = gpu_permutations(5, rounds)
    chi, dof = stats.chi_square(perms)
    assert (chi < stats.chi_square_critical(dof, 0.05)) == passes, chi
    # the same sample as the oracle's
    assert np.array_equal(perms[:2000], oracle.permutations(5, np.arange(1, 2001, dtype=np.uint64), rounds))


@pytest.mark.parametrize("n", [5, 100, 1000])
def test_mmd_pass_at_24_fail_at_4(n):
    p24 = gpu_permutations(n, 24)
    m24 = stats.mmd2(p24)
    assert abs(m24) < stats.normal_threshold(n, P, 0.01), stats.mmd_z(n, m24, P)
    m4 = stats.mmd2(gpu_permutations(n, 4))
    assert abs(m4) > stats.normal_threshold(n, P, 0.05), stats.mmd_z(n, m4, P)
    # the sample the statistic was taken on is the oracle's
    rows = 1000 if n == 1000 else 2000
    assert np.array_equal(p24[:rows], oracle.permutations(n, np.arange(1, rows + 1, dtype=np.uint64), 24))


def test_lcg_chi_square_n5_is_huge():
    """Sec. 5: the LCG bijection fails the n = 5 chi-square test by a wide
    margin (hundreds of thousands against a critical value near 145)."""
    x = torch.arange(5, dtype=torch.int32, device="cuda:0")
    seeds = range(1, 20_001)
    perms = np.stack([bs.shuffle_lcg(x, s).cpu().numpy() for s in seeds]).astype(np.uint32)
    assert np.array_equal(perms, oracle.lcg_permutations(5, seeds))
    chi, dof = stats.chi_square(perms)
    # the statistic grows with the sample: ~5.6e5 at 100,000 permutations,
    # ~1.1e5 at these 20,000
    assert chi > 500 * stats.chi_square_critical(dof, 0.05)
