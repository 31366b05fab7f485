"""bs_shuffle_noalloc (the entry point for callers that cannot allocate)
against bs_shuffle, through the C ABI: byte-equal outputs on consecutive
calls (the second smaller than the first), for several record sizes, and
from a captured graph replayed with eager work in between."""
import numpy as np
import pytest
import torch

from paper_2106_06161_amd import binding as B
from paper_2106_06161_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _noalloc(x, y, seed, rounds, stream):
    n = x.shape[0]
    eb = x.element_size() * (x[0].numel() if x.dim() > 1 else 1)
    B._check(B.bs_shuffle_noalloc(x.data_ptr(), y.data_ptr(), n, eb, seed, rounds, stream.cuda_stream),
             "bs_shuffle_noalloc")


def _reference(x, seed, rounds, stream):
    n = x.shape[0]
    eb = x.element_size() * (x[0].numel() if x.dim() > 1 else 1)
    y = torch.empty_like(x)
    ws = torch.empty(B.bs_workspace_bytes(n, 0, eb), dtype=torch.uint8, device=DEV)
    B._check(B.bs_workspace_init(ws.data_ptr(), ws.numel(), stream.cuda_stream), "bs_workspace_init")
    B._check(B.bs_shuffle(x.data_ptr(), y.data_ptr(), n, eb, seed, rounds, ws.data_ptr(), ws.numel(),
                          stream.cuda_stream), "bs_shuffle")
    return y


@pytest.mark.parametrize("shape,dtype,seeds,rounds", [
    (((1 << 22) + 3, (1 << 17) - 5), torch.int32, (7, 8), 24),
    (((1 << 25) + 1, 100_000), torch.int32, (42, 42), 4),
    ((3_000_001, 5_000), torch.int64, (1, 2), 24),
    ((700_001, 1_025), torch.uint8, (3, 4), 24),
])
def test_noalloc_matches_bs_shuffle_on_two_calls(shape, dtype, seeds, rounds):
    stream = torch.cuda.current_stream(DEV)
    for n, seed in zip(shape, seeds):  # the second call is smaller than the first
        gen = torch.Generator(device=DEV).manual_seed(n)
        x = torch.randint(0, 2**31 - 1, (n,), generator=gen, device=DEV).to(dtype)
        y = torch.full_like(x, -1 if dtype != torch.uint8 else 255)
        _noalloc(x, y, seed, rounds, stream)
        want = _reference(x, seed, rounds, stream)
        torch.cuda.synchronize()
        assert torch.equal(y, want), (n, seed)


def test_noalloc_16_byte_records():
    stream = torch.cuda.current_stream(DEV)
    for n in ((1 << 20) + 7, 33):
        x = torch.from_numpy(W.normal_records_f32(n, 4, seed=11)).to(DEV)
        y = torch.empty_like(x)
        _noalloc(x, y, 11, 24, stream)
        torch.cuda.synchronize()
        assert torch.equal(y, _reference(x, 11, 24, stream))


def test_noalloc_replayed_from_a_graph():
    """Captured calls (the first call of the process already ran outside
    capture in the tests above, or runs here first), replayed several times
    with eager calls of other sizes in between; every replay is exact."""
    stream = torch.cuda.current_stream(DEV)
    n1, n2 = (1 << 21) + 1, 50_000
    x1 = torch.from_numpy(W.uniform_u32(n1, seed=5).view(np.int32)).to(DEV)
    x2 = torch.from_numpy(W.uniform_u32(n2, seed=6).view(np.int32)).to(DEV)
    y1, y2 = torch.empty_like(x1), torch.empty_like(x2)
    _noalloc(x2, y2, 9, 24, stream)  # set-up outside capture
    torch.cuda.synchronize()
    want1, want2 = _reference(x1, 5, 24, stream), _reference(x2, 9, 24, stream)
    side = torch.cuda.Stream(DEV)
    side.wait_stream(stream)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        _noalloc(x1, y1, 5, 24, side)
    torch.cuda.synchronize()
    for rep in range(4):
        y1.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y1, want1), rep
        y2.zero_()
        _noalloc(x2, y2, 9, 24, stream)
        torch.cuda.synchronize()
        assert torch.equal(y2, want2), rep
