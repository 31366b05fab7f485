"""Launch-shape autotuning: a thin wrapper over the library's native tuner.

bs_autotune (csrc/autotune.hip) times every compiled tile shape (waves per
workgroup, indices per lane, tile schedule) with each grid choice, per call
kind, element size and size class, keeps the fastest and writes the table as
text.  The table shipped with the package (tuned_configs.txt, measured on
gfx950) is loaded when the library is loaded.  Shapes never change results.

    python -m paper_2106_06161_amd.autotune            # re-tune and rewrite the shipped table
"""
from __future__ import annotations

import os

from . import binding as B

TUNED_FILE = B.TUNED_FILE
SHAPES = [(4, 16, 2), (8, 16, 2), (8, 16, 1), (16, 16, 1), (16, 8, 1), (8, 8, 2), (4, 16, 1), (16, 16, 2), (16, 8, 2)]
# LDS-compacted schedules: depth field = B.DEPTH_COMPACT or B.DEPTH_COMPACT_PIPE
COMPACT_SHAPES = [(w, i, d) for d in (B.DEPTH_COMPACT, B.DEPTH_COMPACT_PIPE)
                  for (w, i) in ((16, 16), (8, 16), (16, 8), (8, 8), (4, 16))]
GRIDS = [0, 1, 2, B.GRID_ONE_PER_TILE]
KIND_SINGLE, KIND_BATCHED = 0, 1


def read_table(path: str = TUNED_FILE) -> list[dict]:
    """Shape entries of a table file, as dicts (the library reads the same format)."""
    keys = ("kind", "elem_bytes", "size_bits", "waves", "items", "depth", "grid_mult")
    entries = []
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if not line or line[0] in ("arch", "rounds", "staged"):
                continue
            e = dict(zip(keys, map(int, line[:7])))
            if len(line) > 7:
                e["ms"] = float(line[7])
            entries.append(e)
    return entries


def read_staged(path: str = TUNED_FILE) -> list[dict]:
    """The table's "staged" lines: single-shuffle classes where the staged form
    was timed against the fused kernel, and whether bs_shuffle prefers it."""
    out = []
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if not line or line[0] != "staged":
                continue
            e = {"elem_bytes": int(line[1]), "size_bits": int(line[2]), "prefer": int(line[3]) == 1}
            if len(line) > 5:
                e["ms_staged"], e["ms_fused"] = float(line[4]), float(line[5])
            out.append(e)
    return out


def tune(path: str = TUNED_FILE, device: int = 0, max_size_bits: int = 0, verbose: bool = True) -> list[dict]:
    """Tunes on `device` (minutes at the default sizes; a progress line per size
    class on stderr), installs the table and writes it to `path`."""
    if os.path.exists(path):
        os.remove(path)  # otherwise bs_autotune would load it as a cache
    st = B.bs_autotune(device, path, max_size_bits, B.AUTOTUNE_VERBOSE if verbose else 0)
    B._check(st, "bs_autotune")
    return read_table(path)


def main() -> int:
    import argparse

    p = argparse.ArgumentParser(description="Tune launch shapes and write the table.")
    p.add_argument("--out", default=TUNED_FILE)
    p.add_argument("--device", type=int, default=0)
    p.add_argument("--max-size-bits", type=int, default=0, help="largest single-shuffle domain 2^bits (0: 30)")
    a = p.parse_args()
    entries = tune(a.out, a.device, a.max_size_bits)
    for e in entries:
        print(e, flush=True)
    print(f"wrote {len(entries)} entries to {a.out}")
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
