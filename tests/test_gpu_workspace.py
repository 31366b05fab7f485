"""GPU regression tests for the workspace protocol: the status words' 24-bit
generation tag wrapping, and batched tables never being read as status words
by a later launch on the same workspace.

Workspace header (first 256 bytes): ticket @0, done @4, generation @8,
error @12, capacity @16, batch_tiles @20, xcd tickets @24, xcd ranges @56,
batch_bad @92, status high-water mark @96; status words from byte 256.
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
TAG_MASK = (1 << 24) - 1


@pytest.fixture(autouse=True)
def _default_config():
    B.bs_set_config(0, 0, 0, 0)
    B.bs_probe_set_batch_small(1)
    yield
    B.bs_set_config(0, 0, 0, 0)
    B.bs_probe_set_batch_small(1)


def header_u32(ws, offset):
    torch.cuda.synchronize()
    return int(ws[offset:offset + 4].cpu().numpy().view(np.uint32)[0])


def set_generation(ws, gen):
    torch.cuda.synchronize()
    ws[8:12] = torch.from_numpy(np.array([gen], dtype=np.uint32).view(np.uint8)).to(ws.device)
    torch.cuda.synchronize()


def batched(x_np, offsets, seeds, rounds, ws):
    x = torch.from_numpy(np.ascontiguousarray(x_np)).to(DEV)
    off = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int64)).to(DEV)
    sd = torch.from_numpy(np.ascontiguousarray(seeds, dtype=np.uint64).view(np.int64)).to(DEV)
    y = bs.shuffle_batched(x, off, sd, rounds, workspace=ws)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def single(x_np, seed, rounds, ws):
    x = torch.from_numpy(np.ascontiguousarray(x_np)).to(DEV)
    y = bs.shuffle(x, seed, rounds, workspace=ws)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def small_batch():
    sizes = np.array([5, 1, 0, 17, 100, 1000, 1024, 3, 64, 513] * 40, dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    seeds = np.arange(1, len(sizes) + 1, dtype=np.uint64)
    return W.uniform_u32(int(offsets[-1]), seed=21), offsets, seeds


def mixed_batch():
    b = W.batch(200, 5, 200_000, seed=23)
    return W.arange_u32(b["total"]), b["offsets"], b["seeds"]


@pytest.mark.parametrize("kind", ["small", "mixed"])
def test_batch_across_the_tag_wrap(kind):
    """The launch that takes the generation from 2^24 - 1 to 2^24 (tag 0)
    clears status words; the batch's own segment tables must survive it, and
    the launches after the wrap must be exact too."""
    x, offsets, seeds = small_batch() if kind == "small" else mixed_batch()
    total, S = int(offsets[-1]), len(seeds)
    ws = bs.make_workspace(bs.workspace_bytes(total, S), device=DEV)
    want = oracle.shuffle_batched(x, offsets, seeds, 24)
    set_generation(ws, TAG_MASK)
    for call in range(3):  # the wrapping launch, then two with tags 0 and 1
        got = batched(x, offsets, seeds, 24, ws)
        assert np.array_equal(got, want), (kind, call)
        assert bs.workspace_error(ws) == B.BS_OK
    assert header_u32(ws, 8) == TAG_MASK + 3


def test_single_then_batch_across_the_tag_wrap():
    """A single call leaves more status words than the batch uses; the
    batched launch that wraps clears all of them (the high-water mark), and a
    later large single call is exact."""
    xs = W.uniform_u32((1 << 22) + 1, seed=31)  # domain 2^23: more status words than the batch below
    xb, offsets, seeds = small_batch()
    need = max(bs.workspace_bytes(len(xs)), bs.workspace_bytes(int(offsets[-1]), len(seeds)))
    ws = bs.make_workspace(need, device=DEV)
    want_s = oracle.shuffle(xs, 5, 4)
    want_b = oracle.shuffle_batched(xb, offsets, seeds, 24)
    assert np.array_equal(single(xs, 5, 4, ws), want_s)
    hwm = header_u32(ws, 96)
    assert hwm >= (1 << 23) // 16384
    set_generation(ws, TAG_MASK)
    assert np.array_equal(batched(xb, offsets, seeds, 24, ws), want_b)
    assert header_u32(ws, 8) == TAG_MASK + 1
    assert header_u32(ws, 96) >= hwm
    for _ in range(2):
        assert np.array_equal(single(xs, 5, 4, ws), want_s)
    assert bs.workspace_error(ws) == B.BS_OK


def test_batch_tables_are_zeroed_after_the_launch():
    """Everything past the status words a launch used is zero once a batched
    launch is done, so the tables can never be read as status words."""
    x, offsets, seeds = mixed_batch()
    total, S = int(offsets[-1]), len(seeds)
    ws = bs.make_workspace(bs.workspace_bytes(total, S), device=DEV)
    batched(x, offsets, seeds, 24, ws)
    hwm = header_u32(ws, 96)
    tail = ws[256 + 8 * hwm:].cpu().numpy()
    assert hwm > 0 and tail.size > 0
    assert not tail.any()


def test_single_after_batch_on_one_workspace():
    """A batch with few status words and large round-key tables, then a
    single call whose status words cover where those tables were: the keys
    of 20-bit segments, read as status words, would carry the next launch's
    tag in about one word of eight."""
    sizes = np.full(8, (1 << 19) + 1, dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    seeds = np.arange(100, 108, dtype=np.uint64)
    xb = W.arange_u32(int(offsets[-1]))
    xs = W.uniform_u32((1 << 26) + 1, seed=41)  # domain 2^27: 8,192 tiles of 16,384 indices
    ws = bs.make_workspace(max(bs.workspace_bytes(len(xs)), bs.workspace_bytes(len(xb), 8)), device=DEV)
    want_b = oracle.shuffle_batched(xb, offsets, seeds, 24)
    want_s = oracle.shuffle(xs, 9, 4)
    for _ in range(2):
        assert np.array_equal(batched(xb, offsets, seeds, 24, ws), want_b)
        assert np.array_equal(single(xs, 9, 4, ws), want_s)
    assert bs.workspace_error(ws) == B.BS_OK
