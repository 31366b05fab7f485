"""Full-size single shuffles: 10^9 uint32 records, 2.5*10^8 records of 16
bytes, and a domain past 2^32 (64-bit index path, with the un-shuffle forms,
the index output and the LCG bijection).  Checked on oracle slices at the start, middle and end
of the padded domain, and by properties that hold at any size (the output is a
permutation of the input)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2106_06161_amd as bs
from paper_2106_06161_amd import workloads as W
from _helpers import check_slices

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def test_billion_uint32_arange():
    n, seed, rounds = 10**9, 1, 24
    x = torch.arange(n, dtype=torch.int64, device=DEV).to(torch.int32)
    y = bs.shuffle(x, seed, rounds)
    torch.cuda.synchronize()
    assert bs.workspace_error() == 0
    assert torch.equal(torch.sort(y)[0], x)  # a permutation of arange(n)
    del x
    y_np = y.cpu().numpy().view(np.uint32)
    x_np = np.arange(n, dtype=np.uint32)
    domain = 1 << oracle.domain_bits(n)
    check_slices(x_np, y_np, seed, rounds, [0, domain - (1 << 20)])


def test_16_byte_records():
    n, seed, rounds = 250_000_000, 11, 24
    x_np = W.normal_records_f32(n, 4, seed=11)
    x = torch.from_numpy(x_np).to(DEV)
    y = bs.shuffle(x, seed, rounds)
    torch.cuda.synchronize()
    assert bs.workspace_error() == 0
    # same multiset of records: two order-independent checksums over the 4 words
    xi, yi = x.view(torch.int32).to(torch.int64), y.view(torch.int32).to(torch.int64)
    for w in (torch.tensor([1, 3, 5, 7], device=DEV), torch.tensor([11, -13, 17, 19], device=DEV)):
        assert torch.equal((xi * w).sum(dim=1).sum(), (yi * w).sum(dim=1).sum())
    del x, xi, yi
    y_np = y.cpu().numpy()
    domain = 1 << oracle.domain_bits(n)
    check_slices(x_np, y_np, seed, rounds, [0, domain // 2, domain - (1 << 20)], span=1 << 19)


def test_domain_beyond_32_bits():
    """n = 2^32 + 1 one-byte records: k = 33, 64-bit indices (shuffle, and
    both un-shuffle forms back to the input)."""
    n, seed, rounds = (1 << 32) + 1, 3, 4
    x_np = W.random_bytes(n, seed=3)
    x = torch.from_numpy(x_np).to(DEV)
    y = bs.shuffle(x, seed, rounds)
    torch.cuda.synchronize()
    assert bs.workspace_error() == 0
    def histogram(t):
        h = torch.zeros(256, dtype=torch.int64, device=DEV)
        for c in torch.split(t, 1 << 28):
            h += torch.bincount(c.to(torch.int32), minlength=256)
        return h

    assert torch.equal(histogram(x), histogram(y))
    # both un-shuffle forms invert it on the 64-bit index path
    z = bs.unshuffle(y, seed, rounds)
    torch.cuda.synchronize()
    assert torch.equal(z, x)
    z.zero_()
    z = bs.unshuffle_inverse(y, seed, rounds, out=z)
    torch.cuda.synchronize()
    assert torch.equal(z, x)
    del x, z
    y_np = y.cpu().numpy()
    domain = 1 << oracle.domain_bits(n)
    assert domain == 1 << 33
    check_slices(x_np, y_np, seed, rounds, [0, domain - (1 << 20)])


def _lcg_ends(x_np, n, seed, count):
    """The first and last `count` outputs of Algorithm 1 with the LCG bijection
    (oracle parameters), walking the padded domain from each end: the kept
    indices in order give consecutive output slots."""
    a, c = oracle.lcg_params(n, seed)
    domain = 1 << oracle.domain_bits(n)
    head, i = [], 0
    while len(head) < count:
        y = (a * i + c) % domain
        if y < n:
            head.append(x_np[y])
        i += 1
    tail, i = [], domain - 1
    while len(tail) < count:
        y = (a * i + c) % domain
        if y < n:
            tail.append(x_np[y])
        i -= 1
    return np.array(head), np.array(tail[::-1])


def test_lcg_beyond_32_bits():
    """The LCG form on the 64-bit index path (k = 33): a permutation of the
    input whose first and last 4,096 outputs follow Algorithm 1 exactly."""
    n, seed = (1 << 32) + 1, 21
    x_np = W.random_bytes(n, seed=21)
    x = torch.from_numpy(x_np).to(DEV)
    y = bs.shuffle_lcg(x, seed)
    torch.cuda.synchronize()
    assert bs.workspace_error() == 0
    hx = torch.zeros(256, dtype=torch.int64, device=DEV)
    hy = torch.zeros(256, dtype=torch.int64, device=DEV)
    for cx, cy in zip(torch.split(x, 1 << 28), torch.split(y, 1 << 28)):
        hx += torch.bincount(cx.to(torch.int32), minlength=256)
        hy += torch.bincount(cy.to(torch.int32), minlength=256)
    assert torch.equal(hx, hy)
    head, tail = _lcg_ends(x_np, n, seed, 4096)
    assert np.array_equal(y[:4096].cpu().numpy(), head)
    assert np.array_equal(y[-4096:].cpu().numpy(), tail)


def test_permutation_beyond_32_bits():
    """bs_permutation on the 64-bit index path (k = 33, 8-byte indices): its
    first and last 4,096 entries are the kept images of the padded indices
    walked from each end (oracle cipher), and all n entries sum and xor to
    the values of 0 .. n-1."""
    n, seed, rounds = (1 << 32) + 1, 8, 4
    idx = bs.permutation(n, seed, rounds, index_dtype=torch.int64, device=DEV)
    torch.cuda.synchronize()
    assert bs.workspace_error() == 0
    c = oracle.Cipher(oracle.domain_bits(n), seed, rounds)
    head, i = [], 0
    while len(head) < 4096:
        y = c.encrypt(i)
        if y < n:
            head.append(y)
        i += 1
    tail, i = [], (1 << oracle.domain_bits(n)) - 1
    while len(tail) < 4096:
        y = c.encrypt(i)
        if y < n:
            tail.append(y)
        i -= 1
    assert idx[:4096].cpu().tolist() == head
    assert idx[-4096:].cpu().tolist() == tail[::-1]
    total, xor = 0, 0
    for chunk in torch.split(idx, 1 << 28):
        assert int(chunk.min()) >= 0 and int(chunk.max()) < n
        total += int(chunk.sum())
        x = chunk
        while x.numel() > 1:  # xor-reduce by halves
            if x.numel() % 2:
                x = torch.cat([x, torch.zeros(1, dtype=x.dtype, device=x.device)])
            x = torch.bitwise_xor(x[: x.numel() // 2], x[x.numel() // 2:])
        xor ^= int(x[0])
    assert total == n * (n - 1) // 2
    want_xor = [n - 1, 1, n, 0][(n - 1) % 4]  # xor of 0 .. n-1
    assert xor == want_xor


def test_batch_with_a_32_bit_segment():
    """A batch whose largest segment needs all 32 index bits (2^31 + 1 one-byte
    records, domain 2^32) between small segments: the small ones equal the
    oracle, the large one matches oracle slices at both ends of its domain and
    is a permutation of its input."""
    big = (1 << 31) + 1
    sizes = np.array([5, 1000, big, 3, 70_001], dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    seeds = np.array([11, 12, 13, 14, 15], dtype=np.uint64)
    total = int(offsets[-1])
    x_np = W.random_bytes(total, seed=31)
    x = torch.from_numpy(x_np).to(DEV)
    off = torch.from_numpy(offsets).to(DEV)
    sd = torch.from_numpy(seeds.view(np.int64)).to(DEV)
    rounds = 4
    y = bs.shuffle_batched(x, off, sd, rounds)
    torch.cuda.synchronize()
    assert bs.workspace_error() == 0
    lo, hi = int(offsets[2]), int(offsets[3])
    hx = torch.bincount(x[lo:hi].to(torch.int32), minlength=256)
    hy = torch.bincount(y[lo:hi].to(torch.int32), minlength=256)
    assert torch.equal(hx, hy)
    y_np = y.cpu().numpy()
    for s in (0, 1, 3, 4):
        a, b = int(offsets[s]), int(offsets[s + 1])
        assert np.array_equal(y_np[a:b], oracle.shuffle(x_np[a:b], int(seeds[s]), rounds)), s
    assert oracle.domain_bits(big) == 32
    check_slices(x_np[lo:hi], y_np[lo:hi], int(seeds[2]), rounds, [0, (1 << 32) - (1 << 20)])
