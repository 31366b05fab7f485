"""Autotuner for the launch shape of the shuffle kernels.

For each call kind (single bs_shuffle, batched bs_shuffle_batched), element
size and size class it times every compiled tile shape (waves per workgroup,
indices per lane, tile schedule: one or two tiles in flight with records in
registers, or kept images compacted through LDS) with each grid choice, on
seeded random data, and keeps the fastest.  The table is stored as JSON next to this file
and handed to the library with bs_set_tuned_config when the library is
loaded.  Launch shapes never change results, only speed.

    python -m paper_2106_06161_amd.autotune            # tune and write the table
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import binding as B

TUNED_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_configs.json")
SHAPES = [(4, 16, 2), (8, 16, 2), (8, 16, 1), (16, 16, 1), (16, 8, 1), (8, 8, 2), (4, 16, 1), (16, 16, 2), (16, 8, 2)]
# LDS-compacted schedules: depth field = B.DEPTH_COMPACT or B.DEPTH_COMPACT_PIPE
COMPACT_SHAPES = [(w, i, d) for d in (B.DEPTH_COMPACT, B.DEPTH_COMPACT_PIPE)
                  for (w, i) in ((16, 16), (8, 16), (16, 8), (8, 8), (4, 16))]
GRIDS = [0, 1, 2, B.GRID_ONE_PER_TILE]
KIND_SINGLE, KIND_BATCHED = 0, 1


def apply(entries) -> int:
    """Installs tuned entries in the library; returns how many were accepted."""
    ok = 0
    for e in entries:
        st = B.bs_set_tuned_config(e["kind"], e["elem_bytes"], e["size_bits"], e["waves"], e["items"], e["depth"],
                                   e["grid_mult"])
        ok += st == B.BS_OK
    return ok


def load(path: str = TUNED_FILE) -> list[dict]:
    try:
        with open(path) as fh:
            table = json.load(fh)
    except (OSError, ValueError):
        return []
    return list(table.get("entries", []))


def _time(torch, fn, iters: int) -> float:
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(iters):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def _dtype(torch, eb):
    return {1: torch.uint8, 2: torch.int16, 4: torch.int32, 8: torch.int64}[eb] if eb != 16 else torch.int32


def _candidates():
    for sh in SHAPES + COMPACT_SHAPES:
        for g in GRIDS:
            yield sh + (g,)


def tune_single(torch, bs, elem_bytes: int, size_bits: int, rounds: int, iters: int, device) -> dict:
    """Shape for one shuffle with a padded domain of 2^size_bits: the summed
    time at both ends of the size class (n = 2^(size_bits-1) + 1, half the
    domain rejected, and n = 2^size_bits, none rejected)."""
    hi = 1 << size_bits
    lo = (hi >> 1) + 1 if size_bits > 4 else hi
    width = 4 if elem_bytes == 16 else 1
    gen = torch.Generator(device=device).manual_seed(size_bits)
    x = torch.randint(0, 120, (hi, width) if width > 1 else (hi,), dtype=_dtype(torch, elem_bytes), device=device,
                      generator=gen)
    y = torch.empty_like(x)
    xl, yl = x[:lo], y[:lo]
    best = None
    for cfg in _candidates():
        if B.bs_set_config(*cfg) != B.BS_OK:
            continue
        ms = _time(torch, lambda: bs.shuffle(x, 7, rounds, out=y), iters)
        ms += _time(torch, lambda: bs.shuffle(xl, 7, rounds, out=yl), iters)
        if best is None or ms < best[0]:
            best = (ms, cfg)
    B.bs_set_config(0, 0, 0, 0)
    ms, (w, i, d, g) = best
    return {"kind": KIND_SINGLE, "elem_bytes": elem_bytes, "size_bits": size_bits, "waves": w, "items": i,
            "depth": d, "grid_mult": g, "ms": ms, "n": [lo, hi]}


def tune_batched(torch, bs, elem_bytes: int, size_bits: int, rounds: int, iters: int, device,
                 total_items: int = 1 << 26) -> dict:
    """Shape for a batch whose mean segment size is about 2^size_bits
    (sizes log-uniform over a factor of 16 around it, seeded)."""
    from .workloads import log_uniform_sizes

    mean = 1 << size_bits
    count = max(16, min(65536, total_items // mean))
    sizes, seeds = log_uniform_sizes(count, max(1, mean // 4), mean * 4, seed=size_bits)
    offsets = np.zeros(count + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    total = int(offsets[-1])
    width = 4 if elem_bytes == 16 else 1
    x = torch.zeros((total, width) if width > 1 else (total,), dtype=_dtype(torch, elem_bytes), device=device)
    y = torch.empty_like(x)
    off = torch.from_numpy(offsets).to(device)
    sd = torch.from_numpy(seeds.view(np.int64)).to(device)
    real_bits = int(np.ceil(np.log2(max(1, -(-total // count)))))
    best = None
    for cfg in _candidates():
        if B.bs_set_config(*cfg) != B.BS_OK:
            continue
        ms = _time(torch, lambda: bs.shuffle_batched(x, off, sd, rounds, out=y), iters)
        if best is None or ms < best[0]:
            best = (ms, cfg)
    B.bs_set_config(0, 0, 0, 0)
    ms, (w, i, d, g) = best
    return {"kind": KIND_BATCHED, "elem_bytes": elem_bytes, "size_bits": real_bits, "waves": w, "items": i,
            "depth": d, "grid_mult": g, "ms": ms, "segments": count, "total_items": total}


def tune(single_bits=range(12, 31), batched_bits=range(8, 21), elem_sizes=(4, 8, 16), rounds: int = 24,
         iters: int = 3, log=print) -> dict:
    import torch

    import paper_2106_06161_amd as bs

    device = torch.device("cuda:0")
    entries = []
    for eb in elem_sizes:
        for bits in single_bits:
            if (1 << bits) * eb * 2 > 40 << 30:
                continue
            e = tune_single(torch, bs, eb, bits, rounds, iters, device)
            log(json.dumps(e))
            entries.append(e)
        for bits in batched_bits:
            e = tune_batched(torch, bs, eb, bits, rounds, iters, device)
            log(json.dumps(e))
            entries.append(e)
    # a size class left untuned (skipped for memory) takes the entry below it
    filled = list(entries)
    have = {(e["kind"], e["elem_bytes"], e["size_bits"]) for e in entries}
    for e in entries:
        k = (e["kind"], e["elem_bytes"], e["size_bits"] + 1)
        if k not in have:
            filled.append(dict(e, size_bits=e["size_bits"] + 1, interpolated=True))
            have.add(k)
    arch = torch.cuda.get_device_properties(device).gcnArchName
    return {"arch": arch, "rounds": rounds, "entries": filled}


def main() -> int:
    import argparse

    p = argparse.ArgumentParser(description="Tune launch shapes and write the table.")
    p.add_argument("--out", default=TUNED_FILE)
    p.add_argument("--iters", type=int, default=3)
    p.add_argument("--rounds", type=int, default=24)
    a = p.parse_args()
    table = tune(rounds=a.rounds, iters=a.iters)
    with open(a.out, "w") as fh:
        json.dump(table, fh, indent=1)
        fh.write("\n")
    print(f"wrote {len(table['entries'])} entries to {a.out}")
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
