"""GPU parity of bs_bijection, the keyed bijection applied elementwise:

- forward values equal the oracle's encrypt, inverse values its decrypt,
  for even and odd widths from 1 to 40 bits and 0, 1, 2 and 24 rounds;
- on small domains the forward map over every value is the oracle's table
  and a permutation;
- inverse(forward(x)) == x and forward(inverse(y)) == y;
- on the shuffle's own domain, the images below n in index order are the
  gather map bs_permutation writes (same cipher as the fused kernels);
- inputs are reduced modulo 2^k; in-place calls work.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2106_06161_amd as bs
from paper_2106_06161_amd import binding as B

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
WIDTHS = [1, 2, 3, 4, 5, 7, 8, 15, 16, 17, 26, 27, 28, 32, 33, 38, 39, 40]


def _values(k: int, count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    v = rng.integers(0, 1 << k, size=count, dtype=np.uint64)
    v[:4] = [0, (1 << k) - 1, (1 << k) // 2, 1 % (1 << k)]
    return v


def _run(v: np.ndarray, k: int, seed: int, rounds: int, inverse: bool) -> np.ndarray:
    x = torch.from_numpy(v.view(np.int64)).to(DEV)
    y = bs.bijection(x, k, seed, rounds, inverse=inverse)
    torch.cuda.synchronize()
    return y.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("rounds", [0, 1, 2, 24])
@pytest.mark.parametrize("k", WIDTHS)
def test_forward_and_inverse_match_oracle(k, rounds):
    seed = 1000 * k + rounds
    v = _values(k, 600, seed)
    c = oracle.Cipher(k, seed, rounds)
    fwd = _run(v, k, seed, rounds, False)
    inv = _run(v, k, seed, rounds, True)
    assert np.array_equal(fwd, np.array([c.encrypt(int(x)) for x in v], dtype=np.uint64))
    assert np.array_equal(inv, np.array([c.decrypt(int(x)) for x in v], dtype=np.uint64))
    assert np.array_equal(_run(fwd, k, seed, rounds, True), v)
    assert np.array_equal(_run(inv, k, seed, rounds, False), v)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 9, 12, 16, 19])
def test_whole_domain_is_the_oracle_table(k):
    seed = 77 + k
    v = np.arange(1 << k, dtype=np.uint64)
    fwd = _run(v, k, seed, 24, False)
    assert np.array_equal(fwd, oracle.Cipher(k, seed, 24).table().astype(np.uint64))
    assert np.array_equal(np.sort(fwd), v)
    assert np.array_equal(_run(fwd, k, seed, 24, True), v)


@pytest.mark.parametrize("n", [5, 1000, 16385, (1 << 20) + 1])
def test_kept_images_are_the_shuffle_gather_map(n):
    seed, rounds = 4242 + n, 24
    k = bs.bs_domain_bits(n)
    f = _run(np.arange(1 << k, dtype=np.uint64), k, seed, rounds, False)
    perm = bs.permutation(n, seed, rounds, index_dtype=torch.int64, device=DEV)
    torch.cuda.synchronize()
    assert np.array_equal(f[f < n], perm.cpu().numpy().astype(np.uint64))


def test_inputs_are_reduced_and_in_place_works():
    k, seed = 21, 9
    v = _values(k, 4096, 3)
    high = v | (np.uint64(0xABC) << np.uint64(40))
    x = torch.from_numpy(high.view(np.int64)).to(DEV)
    want = _run(v, k, seed, 24, False)
    bs.bijection(x, k, seed, 24, out=x)
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy().view(np.uint64), want)


def test_large_count_grid_stride():
    # more elements than one grid pass covers (65536 workgroups of 256)
    k, seed, count = 34, 5, (1 << 24) + 777
    x = torch.randint(0, 1 << k, (count,), dtype=torch.int64, device=DEV)
    y = bs.bijection(x, k, seed, 24)
    z = bs.bijection(y, k, seed, 24, inverse=True)
    torch.cuda.synchronize()
    assert torch.equal(z, x)
    c = oracle.Cipher(k, seed, 24)
    idx = np.random.default_rng(1).integers(0, count, 256)
    xs, ys = x.cpu().numpy()[idx], y.cpu().numpy()[idx]
    assert all(c.encrypt(int(a)) == int(b) for a, b in zip(xs, ys))
    tail = np.arange(count - 64, count)
    assert all(c.encrypt(int(a)) == int(b) for a, b in zip(x.cpu().numpy()[tail], y.cpu().numpy()[tail]))


def test_argument_errors():
    x = torch.zeros(8, dtype=torch.int64, device=DEV)
    for k, rounds, inv in [(0, 24, 0), (41, 24, 0), (10, 65, 0), (10, 24, 2)]:
        assert B.bs_bijection(x.data_ptr(), x.data_ptr(), 8, k, 1, rounds, inv, None) == B.BS_EINVAL
    assert B.bs_bijection(x.data_ptr() + 4, x.data_ptr(), 1, 10, 1, 24, 0, None) == B.BS_EELEM
    with pytest.raises(ValueError):
        bs.bijection(torch.zeros(8, dtype=torch.int32, device=DEV), 10, 1)
