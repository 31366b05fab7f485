"""bs_shuffle_staged (the streaming-pass form) against the oracle: the same
output as Algorithm 1 for every record size, both parities of k, one and two
distribution passes, the single-window case, ragged tails, zero and few
rounds, repeated calls on one scratch and graph replay; the headline
workload whole; 10^9 records and a domain of 2^31 (above the tuned table) on
oracle slices.  bs_unshuffle_staged (the same passes keyed by output
position) against the oracle's shuffle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2106_06161_amd as bs
from paper_2106_06161_amd import binding as B
from paper_2106_06161_amd import workloads as W

from _helpers import check_slices, oracle_whole

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
NP = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}


def records(n, eb, seed):
    rng = np.random.default_rng(seed)
    if eb == 16:
        return rng.integers(0, 2**63, size=(n, 2), dtype=np.int64)
    return rng.integers(0, np.iinfo(NP[eb]).max, size=n, dtype=NP[eb], endpoint=True)


def to_dev(x_np):
    if x_np.dtype == np.uint16:
        return torch.from_numpy(x_np.view(np.int16)).to(DEV)
    if x_np.dtype == np.uint32:
        return torch.from_numpy(x_np.view(np.int32)).to(DEV)
    if x_np.dtype == np.uint64:
        return torch.from_numpy(x_np.view(np.int64)).to(DEV)
    return torch.from_numpy(x_np).to(DEV)


def staged(x_np, seed, rounds):
    x = to_dev(x_np)
    y = bs.shuffle_staged(x, seed, rounds)
    torch.cuda.synchronize()
    return y.cpu().numpy().view(x_np.dtype).reshape(x_np.shape)


# (n, elem_bytes): single window (k <= s), one pass, the widest one-pass split,
# two passes; odd and even k (at 24 rounds, records of at most 4 bytes with
# 2^b1 <= 256 take the first pass's two-workgroups-per-CU shape, one pass or
# two); ragged tails
CASES = [(1, 4), (5, 4), (1000, 4), (4097, 4), (100_000, 4), ((1 << 20) + 1, 4), ((1 << 22) + 3, 4),
         ((1 << 23) + 1, 4), ((1 << 24) - 5, 4), ((1 << 24) + 1, 4), (70_001, 1), ((1 << 22) + 1, 1),
         (100_003, 2), ((1 << 23) + 7, 2), ((1 << 24) + 3, 2), (65_537, 8), ((1 << 21) + 1, 8),
         ((1 << 23) + 1, 8), (3000, 16), ((1 << 20) + 1, 16), ((1 << 22) + 1, 16)]


@pytest.mark.parametrize("n,eb", CASES)
def test_staged_equals_oracle(n, eb):
    x = records(n, eb, seed=n + eb)
    assert np.array_equal(staged(x, 1000 + n, 24), oracle.shuffle(x, 1000 + n, 24)), (n, eb)


@pytest.mark.parametrize("rounds", [0, 1, 4, 64])
def test_staged_round_counts(rounds):
    x = records((1 << 23) + 1, 4, seed=3)
    assert np.array_equal(staged(x, 9, rounds), oracle.shuffle(x, 9, rounds))


# The first pass takes its two-workgroups-per-CU shape once the inverse cipher
# is long (rounds x 5 instructions for even k, x 8 for odd k, at least 80) and
# the larger one-workgroup shape below that: both sides of the switch, both
# parities of k, 4-, 2- and 1-byte records.
@pytest.mark.parametrize("n,eb,rounds", [((1 << 23) + 1, 4, 15), ((1 << 23) + 1, 4, 16), ((1 << 24) + 1, 4, 9),
                                         ((1 << 24) + 1, 4, 10), ((1 << 21) + 5, 2, 15), ((1 << 21) + 5, 2, 16),
                                         ((1 << 24) + 3, 2, 9), ((1 << 23) + 1, 1, 15), ((1 << 23) + 1, 1, 16),
                                         ((1 << 22) + 1, 1, 10)])
def test_staged_first_pass_shapes(n, eb, rounds):
    x = records(n, eb, seed=rounds)
    assert np.array_equal(staged(x, 77, rounds), oracle.shuffle(x, 77, rounds)), (n, eb, rounds)


def test_staged_splits():
    """The pass structure the cases above cover."""
    for n, eb in CASES:
        assert bs.staged_scratch_bytes(n, eb) > 0
    assert bs.staged_scratch_bytes((1 << 32) + 1, 4) == 0  # k = 33
    assert bs.staged_scratch_bytes(1 << 31, 16) == 0  # k = 31 > 12 + 18


def test_staged_repeated_calls_and_sizes_on_one_scratch():
    sizes = [(1 << 23) + 1, 1000, (1 << 22) + 3, 100_000, (1 << 23) + 1]
    need = max(bs.staged_scratch_bytes(n, 4) for n in sizes)
    scratch = torch.empty(need, dtype=torch.uint8, device=DEV)
    for i, n in enumerate(sizes):
        x_np = records(n, 4, seed=i)
        x = to_dev(x_np)
        y = bs.shuffle_staged(x, 50 + i, 24, scratch=scratch)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy().view(np.uint32), oracle.shuffle(x_np, 50 + i, 24)), n


def test_staged_under_graph_replay():
    n = (1 << 23) + 1
    x_np = records(n, 4, seed=11)
    want = oracle.shuffle(x_np, 77, 24)
    x = to_dev(x_np)
    y = torch.empty_like(x)
    scratch = torch.empty(bs.staged_scratch_bytes(n, 4), dtype=torch.uint8, device=DEV)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bs.shuffle_staged(x, 77, 24, out=y, scratch=scratch)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        bs.shuffle_staged(x, 77, 24, out=y, scratch=scratch)
    for rep in range(4):
        y.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy().view(np.uint32), want), rep
        bs.shuffle_staged(x[: n // 2], 3, 24, out=y[: n // 2], scratch=scratch)  # eager work between replays
        torch.cuda.synchronize()


def test_staged_equals_fused_on_the_headline_workload_whole():
    """n = 2^27 + 1 uniform uint32 (PCG64 seed 7), seed 7, 24 rounds: the
    whole staged output equals the oracle's and the fused kernel's."""
    x_np = W.uniform_u32((1 << 27) + 1, seed=7)
    x = torch.from_numpy(x_np).to(DEV)
    y = bs.shuffle_staged(x, 7, 24)
    z = bs.shuffle(x, 7, 24)
    torch.cuda.synchronize()
    assert torch.equal(y, z)
    assert np.array_equal(y.cpu().numpy(), oracle_whole(x_np, 7, 24))


def test_staged_billion_uint32_slices():
    """n = 10^9 uint32 (domain 2^30: digits 9 + 7, the one-workgroup first
    pass): a permutation of the input, equal to the oracle on slices at both
    ends of the padded domain."""
    n, seed, rounds = 10**9, 1, 24
    x = torch.arange(n, dtype=torch.int64, device=DEV).to(torch.int32)
    y = bs.shuffle_staged(x, seed, rounds)
    torch.cuda.synchronize()
    assert torch.equal(torch.sort(y)[0], x)
    del x
    y_np = y.cpu().numpy().view(np.uint32)
    domain = 1 << oracle.domain_bits(n)
    check_slices(np.arange(n, dtype=np.uint32), y_np, seed, rounds, [0, domain - (1 << 20)])


def test_bs_shuffle_staged_past_the_tuned_table():
    """n = 2^30 + 1 uint32 (domain 2^31, digits 9 + 8), above the largest
    tuned class: bs_shuffle with a workspace that holds the staged scratch
    takes the staged form, and its output equals the fused kernel's and the
    oracle's slices."""
    n, seed, rounds = (1 << 30) + 1, 5, 24
    assert B.bs_query_config(0, 4, n) == (0, 0, B.DEPTH_STAGED, 0)
    x = torch.arange(n, dtype=torch.int64, device=DEV).to(torch.int32)
    ws = bs.make_workspace(B.bs_workspace_bytes_staged(n, 4), device=DEV)
    y = bs.shuffle(x, seed, rounds, workspace=ws)
    torch.cuda.synchronize()
    del ws
    torch.cuda.empty_cache()
    z = bs.shuffle(x, seed, rounds)  # default workspace: the fused kernel
    torch.cuda.synchronize()
    assert torch.equal(y, z)
    del x, z
    y_np = y.cpu().numpy().view(np.uint32)
    domain = 1 << oracle.domain_bits(n)
    check_slices(np.arange(n, dtype=np.uint32), y_np, seed, rounds, [0, domain - (1 << 20)])


def unstaged(y_np, seed, rounds):
    y = to_dev(y_np)
    x = bs.unshuffle_staged(y, seed, rounds)
    torch.cuda.synchronize()
    return x.cpu().numpy().view(y_np.dtype).reshape(y_np.shape)


# the staged un-shuffle inverts the oracle's shuffle: every record size, one
# and two distribution passes, both parities of k, a domain smaller than one
# key tile, ragged tails
UNSHUFFLE_CASES = [(1, 4), (1000, 4), (100_000, 4), ((1 << 20) + 1, 4), ((1 << 23) + 1, 4), ((1 << 24) + 1, 4),
                   (70_001, 1), ((1 << 22) + 1, 1), (100_003, 2), ((1 << 23) + 7, 2), (65_537, 8),
                   ((1 << 21) + 1, 8), (3000, 16), ((1 << 20) + 1, 16)]


@pytest.mark.parametrize("n,eb", UNSHUFFLE_CASES)
def test_unshuffle_staged_inverts_the_oracle_shuffle(n, eb):
    x = records(n, eb, seed=n + 2 * eb)
    y = oracle.shuffle(x, 500 + n, 24)
    assert np.array_equal(unstaged(y, 500 + n, 24), x), (n, eb)


@pytest.mark.parametrize("rounds", [0, 1, 4, 9, 16])
def test_unshuffle_staged_round_counts(rounds):
    x = records((1 << 22) + 3, 4, seed=rounds)
    assert np.array_equal(unstaged(oracle.shuffle(x, 13, rounds), 13, rounds), x)


def test_unshuffle_staged_headline_equals_the_scatter_form():
    """n = 2^27 + 1 uniform uint32, seed 7, 24 rounds: the staged un-shuffle of
    the shuffle is the input, and equals bs_unshuffle's output."""
    x = torch.from_numpy(W.uniform_u32((1 << 27) + 1, seed=7)).to(DEV)
    y = bs.shuffle(x, 7, 24)
    z = bs.unshuffle_staged(y, 7, 24)
    w = bs.unshuffle(y, 7, 24)
    torch.cuda.synchronize()
    assert torch.equal(z, x)
    assert torch.equal(w, x)


def test_unshuffle_staged_under_graph_replay():
    """Captured once, replayed with other work on the same scratch between
    replays: every replay inverts the oracle's shuffle."""
    n = (1 << 23) + 1
    x_np = records(n, 4, seed=12)
    y = to_dev(oracle.shuffle(x_np, 78, 24))
    z = torch.empty_like(y)
    scratch = torch.empty(bs.unshuffle_staged_scratch_bytes(n, 4), dtype=torch.uint8, device=DEV)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bs.unshuffle_staged(y, 78, 24, out=z, scratch=scratch)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        bs.unshuffle_staged(y, 78, 24, out=z, scratch=scratch)
    for rep in range(4):
        z.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(z.cpu().numpy().view(np.uint32), x_np), rep
        bs.unshuffle_staged(y[: n // 2], 5, 24, out=z[: n // 2], scratch=scratch)  # eager work between replays
        torch.cuda.synchronize()


def test_staged_argument_errors_on_device():
    x = torch.zeros(1 << 20, dtype=torch.int32, device=DEV)
    y = torch.empty_like(x)
    need = bs.staged_scratch_bytes(1 << 20, 4)
    small = torch.empty(need - 256, dtype=torch.uint8, device=DEV)
    sp = torch.cuda.current_stream().cuda_stream
    assert B.bs_shuffle_staged(x.data_ptr(), y.data_ptr(), 1 << 20, 4, 1, 24, small.data_ptr(), small.numel(),
                               sp) == B.BS_ENOMEM
    big = torch.empty(need, dtype=torch.uint8, device=DEV)
    assert B.bs_shuffle_staged(x.data_ptr(), y.data_ptr(), 1 << 20, 4, 1, 24, big.data_ptr() + 16, need,
                               sp) == B.BS_EINVAL
    # scratch overlapping the output
    assert B.bs_shuffle_staged(x.data_ptr(), big.data_ptr(), 1 << 18, 4, 1, 24, big.data_ptr(), need,
                               sp) == B.BS_EALIAS


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_bs_shuffle_with_room_for_the_staged_form(mode):
    """bs_shuffle with a workspace of bs_workspace_bytes_staged: policy 1 takes
    the staged form, 0 the fused kernel, 2 what the shipped table says; the
    bytes are the oracle's every time, also after a call with a fused-size
    workspace on the same buffers."""
    n = (1 << 23) + 1
    x_np = records(n, 4, seed=21)
    x = to_dev(x_np)
    want = oracle.shuffle(x_np, 5, 24)
    ws = bs.make_workspace(bs.workspace_bytes(n, staged=True), device=DEV)
    small = bs.make_workspace(bs.workspace_bytes(n), device=DEV)
    assert B.bs_probe_set_staged_policy(mode) == B.BS_OK
    try:
        if mode == 1:
            assert B.bs_query_config(0, 4, n)[2] == B.DEPTH_STAGED
        if mode == 0:
            assert B.bs_query_config(0, 4, n)[2] != B.DEPTH_STAGED
        for w in (ws, small, ws):
            y = bs.shuffle(x, 5, 24, workspace=w)
            torch.cuda.synchronize()
            assert np.array_equal(y.cpu().numpy().view(np.uint32), want)
        assert bs.workspace_error(ws) == B.BS_OK and bs.workspace_error(small) == B.BS_OK
    finally:
        B.bs_probe_set_staged_policy(2)
