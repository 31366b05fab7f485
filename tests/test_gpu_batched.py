"""GPU parity of the batched shuffle: many independent shuffles of packed
segments in one launch sequence, each equal byte for byte to the oracle's
shuffle of that segment with its own seed, and to a single bs_shuffle call.
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


@pytest.fixture(autouse=True)
def _default_config():
    B.bs_set_config(0, 0, 0, 0)
    B.bs_probe_set_xcd_mode(2)
    B.bs_probe_set_batch_small(1)
    yield
    B.bs_set_config(0, 0, 0, 0)
    B.bs_probe_set_xcd_mode(2)
    B.bs_probe_set_batch_small(1)
    assert bs.workspace_error() == B.BS_OK


def run_batched(x_np, offsets, seeds, rounds, **kw):
    x = torch.from_numpy(np.ascontiguousarray(x_np)).to(DEV)
    off = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int64)).to(DEV)
    sd = torch.from_numpy(np.ascontiguousarray(seeds, dtype=np.uint64).view(np.int64)).to(DEV)
    y = bs.shuffle_batched(x, off, sd, rounds, **kw)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def test_small_batch_matches_oracle():
    b = W.batch(300, 100, 100_000, seed=3)
    x = W.arange_u32(b["total"])
    for rounds in (24, 4, 7):
        got = run_batched(x, b["offsets"], b["seeds"], rounds)
        want = oracle.shuffle_batched(x, b["offsets"], b["seeds"], rounds)
        assert np.array_equal(got, want), rounds


EDGE_SIZES = [0, 1, 2, 3, 5, 8, 9, 16, 17, 0, 100, 4095, 4096, 4097, 16383, 16384, 16385, 70_001, 0, 1]


def test_edge_sizes_in_one_batch():
    sizes = np.array(EDGE_SIZES, dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    seeds = np.arange(len(sizes), dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    x = W.uniform_u32(int(offsets[-1]), seed=5)
    got = run_batched(x, offsets, seeds, 24)
    assert np.array_equal(got, oracle.shuffle_batched(x, offsets, seeds, 24))


SMALL_SIZES = [0, 1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 31, 33, 64, 100, 255, 257, 511, 513, 1000, 1023, 1024,
               1025, 2048, 0, 1]


@pytest.mark.parametrize("small", [1, 0])
@pytest.mark.parametrize("dtype,width", [(np.uint8, 0), (np.uint16, 0), (np.uint32, 0), (np.uint64, 0),
                                         (np.uint64, 2)])
def test_small_segments_one_wavefront_each(small, dtype, width):
    """Segments of at most 2^10 padded indices (n <= 1024) go to the
    one-wavefront kernel by default: every size class from 1 to 1024, around
    the boundary (1025, 2048 take tiles), and empty segments, for every record
    size; the same bytes with the path switched off."""
    B.bs_probe_set_batch_small(small)
    rng = np.random.default_rng(17)
    sizes = np.array(SMALL_SIZES * 3 + list(rng.integers(1, 1025, size=300)), dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    seeds = rng.integers(0, 2**63, size=len(sizes), dtype=np.int64).view(np.uint64)
    total = int(offsets[-1])
    shape = (total,) if width == 0 else (total, width)
    x = rng.integers(0, 2**31, size=shape).astype(dtype)
    for rounds in (24, 0, 5):
        got = run_batched(x, offsets, seeds, rounds)
        assert np.array_equal(got, oracle.shuffle_batched(x, offsets, seeds, rounds)), rounds


def test_many_tiny_segments_like_a_permutation_test():
    """100,000 segments of n = 5 (the paper's chi-square setting) in one
    launch: each equals the oracle's shuffle with its own seed."""
    S, n = 100_000, 5
    offsets = (np.arange(S + 1, dtype=np.int64) * n)
    seeds = np.arange(1, S + 1, dtype=np.uint64)
    x = np.tile(np.arange(n, dtype=np.uint32), S)
    got = run_batched(x, offsets, seeds, 24).reshape(S, n)
    want = oracle.permutations(n, seeds[:2000], 24)
    assert np.array_equal(got[:2000], want.astype(np.uint32))
    assert np.array_equal(np.sort(got, axis=1), np.tile(np.arange(n, dtype=np.uint32), (S, 1)))


def test_batched_equals_single_calls():
    b = W.batch(64, 10, 300_000, seed=9)
    x_np = W.uniform_u32(b["total"], seed=1)
    got = run_batched(x_np, b["offsets"], b["seeds"], 24)
    x = torch.from_numpy(x_np).to(DEV)
    for s in range(64):
        lo, hi = int(b["offsets"][s]), int(b["offsets"][s + 1])
        if hi == lo:
            continue
        single = bs.shuffle(x[lo:hi], int(b["seeds"][s]), 24)
        assert np.array_equal(single.cpu().numpy(), got[lo:hi]), s


@pytest.mark.parametrize("cfg", [(0, 0, 0, 0), (16, 16, 9, 0), (16, 8, 8, 0)])
@pytest.mark.parametrize("dtype,width", [(np.uint8, 0), (np.uint16, 0), (np.uint64, 0), (np.float32, 4)])
def test_batched_element_sizes(dtype, width, cfg):
    assert B.bs_set_config(*cfg) == B.BS_OK
    b = W.batch(40, 50, 50_000, seed=11)
    n = b["total"]
    rng = np.random.default_rng(2)
    shape = (n,) if width == 0 else (n, width)
    x = (rng.standard_normal(size=shape).astype(np.float32) if dtype == np.float32
         else rng.integers(0, 250, size=shape).astype(dtype))
    got = run_batched(x, b["offsets"], b["seeds"], 24)
    assert np.array_equal(got, oracle.shuffle_batched(x, b["offsets"], b["seeds"], 24))


COMPACT = [(w, i, d, 0) for d in (B.DEPTH_COMPACT, B.DEPTH_COMPACT_PIPE)
           for (w, i) in ((16, 16), (8, 16), (16, 8), (8, 8), (4, 16))]


@pytest.mark.parametrize("cfg", [(16, 16, 1, 0), (4, 16, 2, 0), (8, 8, 2, 3), (16, 8, 1, 1000), (8, 16, 1, 1)] +
                         COMPACT + [(16, 16, 9, 1000), (16, 8, 8, 2)])
@pytest.mark.parametrize("xcd", [0, 1])
def test_batched_configs_do_not_change_output(cfg, xcd):
    assert B.bs_set_config(*cfg) == B.BS_OK
    assert B.bs_probe_set_xcd_mode(xcd) == B.BS_OK
    b = W.batch(100, 100, 200_000, seed=4)
    x = W.arange_u32(b["total"])
    got = run_batched(x, b["offsets"], b["seeds"], 24)
    assert np.array_equal(got, oracle.shuffle_batched(x, b["offsets"], b["seeds"], 24))


def test_malformed_offsets_rejected_on_device():
    n = 1000
    x = torch.arange(n, dtype=torch.int32, device=DEV)
    out = torch.full_like(x, -7)
    off = torch.tensor([0, 600, 400, 1000], dtype=torch.int64, device=DEV)  # decreasing
    sd = torch.tensor([1, 2, 3], dtype=torch.int64, device=DEV)
    bs.shuffle_batched(x, off, sd, 24, out=out)
    assert bs.workspace_error() == B.BS_EDEVICE
    assert bool((out == -7).all())
    off = torch.tensor([5, 600, 800, 1000], dtype=torch.int64, device=DEV)  # offsets[0] != 0
    bs.shuffle_batched(x, off, sd, 24, out=out)
    assert bs.workspace_error() == B.BS_EDEVICE
    assert bool((out == -7).all())
    off = torch.tensor([0, 600, 800, 1001], dtype=torch.int64, device=DEV)  # past the buffer
    bs.shuffle_batched(x, off, sd, 24, out=out)
    assert bs.workspace_error() == B.BS_EDEVICE
    assert bool((out == -7).all())


def test_batched_under_graph_replay():
    """One batched launch captured in a HIP graph and replayed: every replay,
    with eager work between replays, equals the eager result."""
    b = W.batch(200, 100, 100_000, seed=13)
    x = torch.from_numpy(W.arange_u32(b["total"])).to(DEV)
    off = torch.from_numpy(b["offsets"]).to(DEV)
    sd = torch.from_numpy(b["seeds"].view(np.int64)).to(DEV)
    want = torch.from_numpy(oracle.shuffle_batched(W.arange_u32(b["total"]), b["offsets"], b["seeds"], 24)).to(DEV)
    ws = bs.make_workspace(bs.workspace_bytes(b["total"], 200), device=DEV)
    out = torch.empty_like(x)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        bs.shuffle_batched(x, off, sd, 24, out=out, workspace=ws)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        bs.shuffle_batched(x, off, sd, 24, out=out, workspace=ws)
    for i in range(5):
        out.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, want), i
        # eager work between replays
        bs.shuffle(x[:1000], 5, 24)
        torch.cuda.synchronize()
    assert bs.workspace_error(ws) == B.BS_OK


def test_back_to_back_batches_rewrite_the_key_table():
    """Consecutive batched launches on one workspace and stream, no sync in
    between: each launch's prepare kernel rewrites the per-segment key table
    that the previous launch's tiles read through scalar loads; every output
    must follow its own seeds and offsets."""
    ws = bs.make_workspace(bs.workspace_bytes(300_000, 64), device=DEV)
    cases, outs = [], []
    for seed in (21, 22, 23):
        b = W.batch(64 if seed != 22 else 40, 100, 5_000, seed=seed)
        x_np = W.arange_u32(b["total"])
        x = torch.from_numpy(x_np).to(DEV)
        off = torch.from_numpy(b["offsets"]).to(DEV)
        sd = torch.from_numpy(b["seeds"].view(np.int64)).to(DEV)
        outs.append(bs.shuffle_batched(x, off, sd, 24, workspace=ws))
        cases.append((x_np, b))
    torch.cuda.synchronize()
    assert bs.workspace_error(ws) == B.BS_OK
    for (x_np, b), y in zip(cases, outs):
        want = oracle.shuffle_batched(x_np, b["offsets"], b["seeds"], 24)
        assert np.array_equal(y.cpu().numpy(), want)


def test_bootstrap_shaped_batch_sampled():
    """4,096 segments, sizes log-uniform in [100, 10^6] (seed 3), uint32
    payload = global index: every output value stays in its segment and the
    output is a permutation; sampled segments match the oracle exactly."""
    b = W.batch(4096, 100, 1_000_000, seed=3)
    total = b["total"]
    x = torch.arange(total, dtype=torch.int64, device=DEV).to(torch.int32)
    off = torch.from_numpy(b["offsets"]).to(DEV)
    sd = torch.from_numpy(b["seeds"].view(np.int64)).to(DEV)
    y = bs.shuffle_batched(x, off, sd, 24)
    torch.cuda.synchronize()
    pos = torch.arange(total, device=DEV)
    seg_of_pos = torch.searchsorted(off, pos, right=True) - 1
    seg_of_val = torch.searchsorted(off, y.to(torch.int64), right=True) - 1
    assert torch.equal(seg_of_pos, seg_of_val)
    assert torch.equal(torch.sort(y)[0], x)
    y_np = y.cpu().numpy().view(np.uint32)
    rng = np.random.default_rng(0)
    picks = set(rng.choice(4096, size=24, replace=False).tolist()) | {int(np.argmax(b["sizes"])), 0, 4095}
    for s in sorted(picks):
        lo, hi = int(b["offsets"][s]), int(b["offsets"][s + 1])
        want = oracle.shuffle(np.arange(lo, hi, dtype=np.uint32), int(b["seeds"][s]), 24)
        assert np.array_equal(y_np[lo:hi], want), s


def test_xcd_ranges_cover_whole_segments():
    """The batch's tiles are split into 8 XCD ranges made of whole segments,
    about equal in size; read back from the workspace header after a launch."""
    assert B.bs_probe_set_xcd_mode(1) == B.BS_OK  # ranges on (auto keeps one range below 4 tiles a segment)
    b = W.batch(300, 100, 100_000, seed=9)
    S, total = len(b["sizes"]), b["total"]
    x = torch.from_numpy(W.arange_u32(total)).to(DEV)
    off = torch.from_numpy(b["offsets"]).to(DEV)
    sd = torch.from_numpy(b["seeds"].view(np.int64)).to(DEV)
    ws = bs.make_workspace(bs.workspace_bytes(total, S), device=DEV)
    y = bs.shuffle_batched(x, off, sd, 24, workspace=ws)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), oracle.shuffle_batched(W.arange_u32(total), b["offsets"], b["seeds"], 24))
    hdr = ws[:256].cpu().numpy().view(np.uint32)
    batch_tiles, xcd_first = int(hdr[5]), hdr[14:23].astype(np.int64)
    waves, items, _, _ = B.bs_query_config(1, 4, total, S)
    tile = 64 * waves * items
    # empty segments and those of at most 2^10 padded indices (one wavefront
    # each) take no tile
    tiles = [0 if n == 0 or B.bs_domain_bits(int(n)) <= 10 else -(-(1 << B.bs_domain_bits(int(n))) // tile)
             for n in b["sizes"]]
    starts = np.concatenate([[0], np.cumsum(tiles)])
    assert batch_tiles == starts[-1]
    assert xcd_first[0] == 0 and xcd_first[8] == batch_tiles
    assert np.all(np.diff(xcd_first) >= 0)
    assert set(xcd_first.tolist()) <= set(starts.tolist())  # whole segments per range
    assert np.diff(xcd_first).max() <= -(-batch_tiles // 8) + max(tiles)
    # with ranges off, every tile is in the first range
    assert B.bs_probe_set_xcd_mode(0) == B.BS_OK
    y = bs.shuffle_batched(x, off, sd, 24, workspace=ws)
    torch.cuda.synchronize()
    hdr = ws[:256].cpu().numpy().view(np.uint32)
    assert hdr[14] == 0 and np.all(hdr[15:23] == batch_tiles)
    assert np.array_equal(y.cpu().numpy(), oracle.shuffle_batched(W.arange_u32(total), b["offsets"], b["seeds"], 24))
    assert bs.workspace_error(ws) == B.BS_OK
