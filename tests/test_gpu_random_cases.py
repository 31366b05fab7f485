"""Seeded random parity cases: n log-uniform over [1, 2^21], every element
size, rounds in [0, 32], 64-bit seeds and every compiled launch shape (both
tile schedules, every grid choice), each bit-exact against the oracle; half
of the cases also run as a batch of several segments."""
import numpy as np
import pytest
import torch

import oracle
import paper_2106_06161_amd as bs
from paper_2106_06161_amd import autotune
from paper_2106_06161_amd import binding as B

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SHAPES = [tuple(s) for s in autotune.SHAPES + autotune.COMPACT_SHAPES]
DTYPES = {1: (np.uint8, 0), 2: (np.uint16, 0), 4: (np.uint32, 0), 8: (np.uint64, 0), 16: (np.uint32, 4)}


def _case(i):
    rng = np.random.default_rng(9000 + i)
    n = int(np.exp(rng.uniform(0, np.log(1 << 21))))
    eb = int(rng.choice(list(DTYPES)))
    rounds = int(rng.integers(0, 33))
    seed = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
    shape = SHAPES[int(rng.integers(0, len(SHAPES)))]
    grid = int(rng.choice(autotune.GRIDS))
    dt, width = DTYPES[eb]
    x = rng.integers(0, np.iinfo(dt).max, size=(n,) if width == 0 else (n, width), dtype=dt)
    return n, eb, rounds, seed, shape + (grid,), x, rng


@pytest.fixture(autouse=True)
def _default_config():
    yield
    B.bs_set_config(0, 0, 0, 0)
    assert bs.workspace_error() == B.BS_OK


@pytest.mark.parametrize("i", range(48))
def test_random_case(i):
    n, eb, rounds, seed, cfg, x, rng = _case(i)
    assert B.bs_set_config(*cfg) == B.BS_OK
    xt = torch.from_numpy(x).to(DEV)
    y = bs.shuffle(xt, seed, rounds)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), oracle.shuffle(x, seed, rounds)), (n, eb, rounds, seed, cfg)
    if i % 2 == 0:
        cuts = np.sort(rng.integers(0, n + 1, size=int(rng.integers(1, 8))))
        offsets = np.concatenate([[0], cuts, [n]]).astype(np.int64)
        seeds = rng.integers(0, 2**63, size=len(offsets) - 1, dtype=np.uint64)
        off = torch.from_numpy(offsets).to(DEV)
        sd = torch.from_numpy(seeds.view(np.int64)).to(DEV)
        yb = bs.shuffle_batched(xt, off, sd, rounds)
        torch.cuda.synchronize()
        want = oracle.shuffle_batched(x, offsets, seeds, rounds)
        assert np.array_equal(yb.cpu().numpy(), want), (n, eb, rounds, cfg, offsets.tolist())
