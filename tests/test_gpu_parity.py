"""GPU parity: the HIP path, called through the C ABI, against the oracle.

The shuffle is integer-only and moves raw bytes, so every comparison is
bit-exact (np.array_equal).  Small and medium sizes are checked whole; the
full-size workloads are checked on oracle slices at the start, middle and
end of the padded domain plus properties that hold at any size (the output
is a permutation of the input).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2106_06161_amd as bs
from paper_2106_06161_amd import binding as B
from paper_2106_06161_amd import workloads as W
from _helpers import oracle_whole, oracle_window

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def gpu(x_np, seed, rounds, **kw):
    x = torch.from_numpy(np.ascontiguousarray(x_np)).to(DEV)
    y = bs.shuffle(x, seed, rounds, **kw)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.fixture(autouse=True)
def _default_config():
    B.bs_set_config(0, 0, 0, 0)
    B.bs_probe_set_store_mode(0)
    yield
    B.bs_set_config(0, 0, 0, 0)
    B.bs_probe_set_store_mode(0)
    assert bs.workspace_error() == B.BS_OK


# --------------------------------------------------------- small sizes --
def test_small_workload_bitexact():
    """n = 100,000 uint32 arange, seed 42, 4 rounds (domain 2^17)."""
    x = W.arange_u32(100_000)
    assert np.array_equal(gpu(x, 42, 4), oracle.shuffle(x, 42, 4))


SWEEP = [1, 2, 3, 5, 8, 9, 15, 16, 17, 31, 32, 33, 63, 64, 65, 100, 127, 128, 129, 255, 256, 257,
         1000, 1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8193, 12345, 65535, 65536,
         65537, 100_000, 131_071, 131_073, 1 << 20, (1 << 20) + 1]


@pytest.mark.parametrize("rounds", [0, 1, 4, 7, 24])
def test_size_sweep(rounds):
    for n in SWEEP:
        x = W.uniform_u32(n, seed=n)
        seed = 1000 + n
        got, want = gpu(x, seed, rounds), oracle.shuffle(x, seed, rounds)
        assert np.array_equal(got, want), (n, rounds)


def test_many_seeds_small():
    x = W.arange_u32(5)
    for seed in range(200):
        assert np.array_equal(gpu(x, seed, 24), oracle.shuffle(x, seed, 24)), seed


@pytest.mark.parametrize("eb_dtype,width", [(np.uint8, 0), (np.uint16, 0), (np.uint32, 0), (np.uint64, 0),
                                            (np.float32, 4)])
@pytest.mark.parametrize("n", [40_000, 70_001])
def test_element_sizes(eb_dtype, width, n):
    rng = np.random.default_rng(n)
    shape = (n,) if width == 0 else (n, width)
    x = rng.integers(0, np.iinfo(np.uint8).max, size=shape).astype(eb_dtype) if eb_dtype != np.float32 \
        else rng.standard_normal(size=shape).astype(np.float32)
    assert np.array_equal(gpu(x, 77, 24), oracle.shuffle(x, 77, 24))


SHAPES = [(4, 16, 2), (8, 16, 2), (8, 16, 1), (16, 16, 1), (16, 8, 1), (8, 8, 2), (4, 16, 1), (16, 16, 2),
          (16, 8, 2)]
COMPACT = [(w, i, d) for d in (B.DEPTH_COMPACT, B.DEPTH_COMPACT_PIPE)  # LDS-compacted schedules
           for (w, i) in ((16, 16), (8, 16), (16, 8), (8, 8), (4, 16))]
CONFIGS = [s + (0,) for s in SHAPES + COMPACT] + [(8, 16, 2, 1), (4, 16, 1, 1000), (16, 8, 1, 3),
                                                  (16, 16, 8, 1000), (8, 16, 8, 1), (16, 8, 9, 1000), (16, 8, 9, 1)]


@pytest.mark.parametrize("cfg", CONFIGS)
@pytest.mark.parametrize("rounds", [24, 5])
def test_launch_configs_do_not_change_output(cfg, rounds):
    assert B.bs_set_config(*cfg) == B.BS_OK
    for n in (300_001, 262_144, 33):
        x = W.uniform_u32(n, seed=3)
        assert np.array_equal(gpu(x, 9, rounds), oracle.shuffle(x, 9, rounds)), (cfg, n)


@pytest.mark.parametrize("cfg", [(16, 16, 8, 0), (8, 8, 8, 0), (16, 8, 9, 0), (8, 16, 9, 0)])
def test_compact_schedule_element_sizes(cfg):
    assert B.bs_set_config(*cfg) == B.BS_OK
    rng = np.random.default_rng(8)
    for dt, width in ((np.uint8, 0), (np.uint16, 0), (np.uint64, 0), (np.float32, 4)):
        for n in (17, 16_385, 200_003):
            shape = (n,) if width == 0 else (n, width)
            x = rng.integers(0, 250, size=shape).astype(dt)
            assert np.array_equal(gpu(x, 12, 24), oracle.shuffle(x, 12, 24)), (cfg, dt, n)


def test_store_modes_agree():
    x = W.uniform_u32(200_003, seed=4)
    want = oracle.shuffle(x, 5, 24)
    B.bs_probe_set_store_mode(0)
    assert np.array_equal(gpu(x, 5, 24), want)
    B.bs_probe_set_store_mode(1)
    assert np.array_equal(gpu(x, 5, 24), want)


def test_caller_workspace_reused_across_sizes():
    ws = bs.make_workspace(bs.workspace_bytes(1 << 21), device=DEV)
    for i, n in enumerate([1 << 21, 7, 100_000, 1 << 21, 3, 555_555] * 3):
        x = W.uniform_u32(n, seed=i)
        assert np.array_equal(gpu(x, i, 24, workspace=ws), oracle.shuffle(x, i, 24)), (i, n)
    assert bs.workspace_error(ws) == B.BS_OK


def test_workspace_too_small_raises():
    ws = bs.make_workspace(512, device=DEV)
    x = torch.zeros(1 << 20, dtype=torch.int32, device=DEV)
    with pytest.raises(bs.BShuffleError):
        bs.shuffle(x, 1, 24, workspace=ws)


def test_many_launches_one_stream():
    """Hundreds of launches share the library workspace; every one must be
    exact (the per-launch generation tags keep stale tile words inert)."""
    xs = [torch.from_numpy(W.uniform_u32(n, seed=n)).to(DEV) for n in (4097, 100_000, 70_001)]
    want = [oracle.shuffle(x.cpu().numpy(), 11, 24) for x in xs]
    outs = []
    for it in range(300):
        j = it % 3
        outs.append((j, bs.shuffle(xs[j], 11, 24)))
    torch.cuda.synchronize()
    for j, y in outs:
        assert np.array_equal(y.cpu().numpy(), want[j])


def test_tensor_api_checks():
    x = torch.arange(10, dtype=torch.int32, device=DEV)
    with pytest.raises(ValueError):
        bs.shuffle(x.cpu(), 1)
    with pytest.raises(ValueError):
        bs.shuffle(x[::2], 1)
    with pytest.raises(bs.BShuffleError):
        bs.shuffle(x, 1, rounds=65)
    y = torch.empty(0, dtype=torch.int32, device=DEV)
    assert bs.shuffle(y, 1).numel() == 0


# ------------------------------------------------------ full-size single --
def _check_large(x_np, seed, rounds, windows=3, span=1 << 20):
    n = x_np.shape[0]
    x = torch.from_numpy(x_np).to(DEV)
    y = bs.shuffle(x, seed, rounds)
    torch.cuda.synchronize()
    domain = 1 << oracle.domain_bits(n)
    starts = [0, domain // 2, domain - span][:windows]
    y_np = y.cpu().numpy()
    for s in starts:
        rank, want = oracle_window(x_np, seed, rounds, s, s + span)
        assert np.array_equal(y_np[rank:rank + len(want)], want), (n, s)
    # permutation of the input: equal multisets
    xs = torch.sort(x.view(torch.int32) if x.dtype == torch.uint32 else x.view(-1))[0]
    ys = torch.sort(y.view(torch.int32) if y.dtype == torch.uint32 else y.view(-1))[0]
    assert torch.equal(xs, ys)


def test_headline_workload_4_rounds_whole():
    """n = 2^27 + 1 uniform uint32 (seed 7), domain 2^28, 4 rounds: whole output."""
    x = W.uniform_u32((1 << 27) + 1, seed=7)
    assert np.array_equal(gpu(x, 7, 4), oracle.shuffle(x, 7, 4))


def test_headline_workload_24_rounds_whole():
    """The benched configuration itself: n = 2^27 + 1 uniform uint32 (seed 7),
    domain 2^28, 24 rounds; the whole output against the oracle's (computed
    over 64 windows of the padded domain on parallel threads)."""
    x = W.uniform_u32((1 << 27) + 1, seed=7)
    assert np.array_equal(gpu(x, 7, 24), oracle_whole(x, 7, 24))


def test_headline_workload_24_rounds_slices():
    x = W.uniform_u32((1 << 27) + 1, seed=7)
    _check_large(x, 7, 24)


def test_power_of_two_control_24_rounds_slices():
    x = W.uniform_u32(1 << 27, seed=7)
    _check_large(x, 7, 24)


@pytest.mark.parametrize("cfg", [(0, 0, 0, 0), (16, 16, 9, 0), (16, 16, 1, 0)])
def test_single_shuffles_under_graph_replay(cfg):
    """Several bs_shuffle calls captured in one HIP graph and replayed: every
    replay, with eager launches on the same workspace between replays, equals
    the oracle."""
    assert B.bs_set_config(*cfg) == B.BS_OK
    sizes = [1000, 100_003, 1 << 20, (1 << 22) + 1]
    xs = [W.uniform_u32(n, seed=n) for n in sizes]
    want = [oracle.shuffle(x, 40 + i, 24) for i, x in enumerate(xs)]
    xd = [torch.from_numpy(x).to(DEV) for x in xs]
    outs = [torch.empty_like(x) for x in xd]
    ws = bs.make_workspace(bs.workspace_bytes(max(sizes)), device=DEV)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        for i, x in enumerate(xd):
            bs.shuffle(x, 40 + i, 24, out=outs[i], workspace=ws)
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        for i, x in enumerate(xd):
            bs.shuffle(x, 40 + i, 24, out=outs[i], workspace=ws)
    for rep in range(5):
        for o in outs:
            o.fill_(0)
        g.replay()
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            assert np.array_equal(o.cpu().numpy(), want[i]), (cfg, rep, sizes[i])
        bs.shuffle(xd[1], 7, 24, workspace=ws)  # eager work on the same workspace between replays
        torch.cuda.synchronize()
    assert bs.workspace_error(ws) == B.BS_OK


def test_capture_without_a_workspace_is_rejected():
    """During graph capture the library's own workspace cache is not used
    (a later call could regrow it under the graph): BS_EINVAL, nothing captured."""
    x = torch.arange(1000, dtype=torch.int32, device=DEV)
    y = torch.empty_like(x)
    stream = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        st = B.bs_shuffle(x.data_ptr(), y.data_ptr(), 1000, 4, 1, 24, None, 0, stream.cuda_stream)
        y.fill_(3)  # something to capture
    assert st == B.BS_EINVAL
    g.replay()
    torch.cuda.synchronize()
    assert bool((y == 3).all())


@pytest.mark.parametrize("cfg", [(16, 16, 8, 0), (16, 8, 9, 0), (16, 16, 1, 0)])
def test_cipher_scan_probe_under_each_schedule(cfg):
    """The no-payload probe (cipher, keep flags and scan only) runs with every
    tile schedule and leaves the workspace clean."""
    assert B.bs_set_config(*cfg) == B.BS_OK
    ws = bs.make_workspace(bs.workspace_bytes((1 << 22) + 1), device=DEV)
    sp = torch.cuda.current_stream().cuda_stream
    for n in (1, 1000, (1 << 22) + 1):
        assert B.bs_probe_cipher_scan(n, 3, 24, ws.data_ptr(), ws.numel(), sp) == B.BS_OK
    torch.cuda.synchronize()
    assert bs.workspace_error(ws) == B.BS_OK
