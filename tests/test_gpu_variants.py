"""GPU parity of the permutation outputs and the less-fused variants:

- bs_permutation writes the gather map itself (oracle: shuffle_sources);
- bs_unshuffle inverts bs_shuffle (and matches the oracle's inverse map);
- the two-pass-scan and unfused forms (Sec. 6, Bijective1 / Bijective0)
  produce exactly bs_shuffle's output.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2106_06161_amd as bs
from paper_2106_06161_amd import binding as B
from paper_2106_06161_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SIZES = [1, 2, 5, 16, 17, 1000, 4097, 16383, 16384, 16385, 100_000, 300_001, 1 << 20, (1 << 20) + 1]


@pytest.fixture(autouse=True)
def _check_device_errors():
    yield
    assert bs.workspace_error() == B.BS_OK


@pytest.mark.parametrize("rounds", [24, 4])
@pytest.mark.parametrize("index_dtype", [torch.int32, torch.int64])
def test_permutation_matches_oracle(rounds, index_dtype):
    for n in SIZES:
        got = bs.permutation(n, 100 + n, rounds, index_dtype=index_dtype, device=DEV)
        torch.cuda.synchronize()
        want = oracle.shuffle_sources(n, 100 + n, rounds)
        assert np.array_equal(got.cpu().numpy().astype(np.uint64), want), n


@pytest.mark.parametrize("dtype,width", [(np.uint8, 0), (np.uint16, 0), (np.uint32, 0), (np.uint64, 0),
                                         (np.float32, 4)])
def test_unshuffle_inverts_shuffle(dtype, width):
    rng = np.random.default_rng(1)
    for n in (5, 4097, 70_001, 300_001):
        shape = (n,) if width == 0 else (n, width)
        x_np = rng.integers(0, 250, size=shape).astype(dtype)
        x = torch.from_numpy(x_np).to(DEV)
        y = bs.shuffle(x, 9, 24)
        z = bs.unshuffle(y, 9, 24)
        torch.cuda.synchronize()
        assert torch.equal(z, x), n
        # against the oracle: the record at output j came from position perm[j]
        perm = oracle.shuffle_sources(n, 9, 24).astype(np.int64)
        y_np = y.cpu().numpy()
        want = np.empty_like(y_np)
        want[perm] = y_np
        assert np.array_equal(z.cpu().numpy(), want), n


@pytest.mark.parametrize("dtype,width", [(np.uint8, 0), (np.uint16, 0), (np.uint32, 0), (np.uint64, 0),
                                         (np.uint64, 2)])
@pytest.mark.parametrize("rounds", [24, 3, 0])
def test_unshuffle_through_inverse_matches_oracle(dtype, width, rounds):
    """Gather form through f^-1: the oracle's inverse map, sizes spanning
    several rank tiles (8192 indices) with ragged ends, odd and even k."""
    rng = np.random.default_rng(2)
    for n in (1, 2, 5, 16, 17, 1000, 8191, 8193, 70_001, 300_001, 1 << 20):
        shape = (n,) if width == 0 else (n, width)
        y_np = rng.integers(0, 250, size=shape).astype(dtype)
        y = torch.from_numpy(y_np).to(DEV)
        z = bs.unshuffle_inverse(y, 31 + n, rounds)
        torch.cuda.synchronize()
        perm = oracle.shuffle_sources(n, 31 + n, rounds).astype(np.int64)
        want = np.empty_like(y_np)
        want[perm] = y_np
        assert np.array_equal(z.cpu().numpy(), want), n


def test_unshuffle_forms_agree_and_scratch_is_reused():
    n = 2_000_003
    x = torch.from_numpy(W.uniform_u32(n, seed=5)).to(DEV)
    y = bs.shuffle(x, 12, 24)
    scratch = torch.full((B.bs_unshuffle_inverse_scratch_bytes(n),), 0xAB, dtype=torch.uint8, device=DEV)
    a = bs.unshuffle(y, 12, 24)
    b = bs.unshuffle_inverse(y, 12, 24, scratch=scratch)
    # a smaller call on the same (now dirty) scratch
    small = bs.unshuffle_inverse(y[:1000], 4, 24, scratch=scratch)
    torch.cuda.synchronize()
    assert torch.equal(a, x) and torch.equal(b, x)
    assert torch.equal(small, bs.unshuffle(y[:1000], 4, 24))
    st = B.bs_unshuffle_inverse(y.data_ptr(), a.data_ptr(), n, 4, 12, 24, scratch.data_ptr(), scratch.numel() - 1,
                                None)
    assert st == B.BS_ENOMEM


@pytest.mark.parametrize("rounds", [24, 5])
def test_two_pass_and_unfused_equal_fused(rounds):
    for n in SIZES:
        x_np = W.uniform_u32(n, seed=n)
        x = torch.from_numpy(x_np).to(DEV)
        want = oracle.shuffle(x_np, 77, rounds)
        y2 = torch.empty_like(x)
        st = B.bs_probe_shuffle_two_pass(x.data_ptr(), y2.data_ptr(), n, 4, 77, rounds, None, 0,
                                         torch.cuda.current_stream().cuda_stream)
        assert st == B.BS_OK
        scratch = torch.empty(B.bs_probe_unfused_scratch_bytes(n), dtype=torch.uint8, device=DEV)
        y0 = torch.empty_like(x)
        st = B.bs_probe_shuffle_unfused(x.data_ptr(), y0.data_ptr(), n, 4, 77, rounds, scratch.data_ptr(),
                                        scratch.numel(), None, 0, torch.cuda.current_stream().cuda_stream)
        assert st == B.BS_OK
        torch.cuda.synchronize()
        assert np.array_equal(y2.cpu().numpy(), want), ("two-pass", n)
        assert np.array_equal(y0.cpu().numpy(), want), ("unfused", n)


def test_two_pass_other_element_sizes():
    for eb, dt in ((8, np.uint64), (16, np.uint32)):
        n = 123_457
        shape = (n,) if eb == 8 else (n, 4)
        x_np = np.random.default_rng(eb).integers(0, 2**31, size=shape).astype(dt)
        x = torch.from_numpy(x_np).to(DEV)
        y = torch.empty_like(x)
        assert B.bs_probe_shuffle_two_pass(x.data_ptr(), y.data_ptr(), n, eb, 3, 24, None, 0,
                                           torch.cuda.current_stream().cuda_stream) == B.BS_OK
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), oracle.shuffle(x_np, 3, 24))


def test_workspace_shared_by_variants_and_fused():
    """Two-pass leaves counts in the status words; a fused launch on the same
    workspace afterwards must still be exact."""
    n = 1 << 20
    ws = bs.make_workspace(bs.workspace_bytes(n), device=DEV)
    x_np = W.uniform_u32(n, seed=5)
    x = torch.from_numpy(x_np).to(DEV)
    want = oracle.shuffle(x_np, 5, 24)
    for _ in range(3):
        y = torch.empty_like(x)
        B.bs_probe_shuffle_two_pass(x.data_ptr(), y.data_ptr(), n, 4, 5, 24, ws.data_ptr(), ws.numel(),
                                    torch.cuda.current_stream().cuda_stream)
        z = bs.shuffle(x, 5, 24, workspace=ws)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), want) and np.array_equal(z.cpu().numpy(), want)
    assert bs.workspace_error(ws) == B.BS_OK


@pytest.mark.parametrize("dtype,width", [(np.uint8, 0), (np.uint32, 0), (np.uint64, 0), (np.float32, 4)])
def test_lcg_shuffle_matches_oracle(dtype, width):
    rng = np.random.default_rng(2)
    for n in SIZES:
        shape = (n,) if width == 0 else (n, width)
        x_np = rng.integers(0, 250, size=shape).astype(dtype)
        x = torch.from_numpy(x_np).to(DEV)
        y = bs.shuffle_lcg(x, 31 + n)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), oracle.lcg_shuffle(x_np, 31 + n)), n
