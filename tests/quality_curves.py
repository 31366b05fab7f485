"""Distribution-quality curves of Sec. 5 with permutations generated on the GPU.

For VariablePhilox at several round counts (one batched launch of 100,000
shuffles of arange(n), seeds 1..100,000), for the LCG bijection (one call per
seed) and for std::shuffle (CPU, the control that should pass), this prints:

  - the chi-square statistic over all 120 orderings at n = 5 (119 degrees of
    freedom, critical value 145.46 at alpha = 0.05);
  - the Mallows-kernel MMD^2 estimate (lambda = 5) at n = 5, 100 and 1000 as a
    z-score of its null distribution (|z| > 2.576 rejects at alpha = 0.01).

Not collected by pytest (it takes about a minute on one GPU):
    python tests/quality_curves.py [--out FILE.md] [--perms 100000]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from oracle import stats  # noqa: E402

ROUNDS = [2, 4, 8, 12, 16, 20, 24, 32]
SIZES = [5, 100, 1000]


def philox_perms(torch, bs, n: int, rounds: int, count: int) -> np.ndarray:
    x = torch.arange(n, dtype=torch.int32, device="cuda:0").repeat(count)
    off = torch.arange(count + 1, dtype=torch.int64, device="cuda:0") * n
    sd = torch.arange(1, count + 1, dtype=torch.int64, device="cuda:0")
    y = bs.shuffle_batched(x, off, sd, rounds)
    torch.cuda.synchronize()
    return y.view(count, n).cpu().numpy().astype(np.uint32)


def lcg_perms(torch, bs, n: int, count: int) -> np.ndarray:
    x = torch.arange(n, dtype=torch.int32, device="cuda:0")
    out = torch.empty((count, n), dtype=torch.int32, device="cuda:0")
    for s in range(count):
        bs.shuffle_lcg(x, s + 1, out=out[s])
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.uint32)


def std_perms(n: int, count: int) -> np.ndarray:
    base = np.arange(n, dtype=np.uint32)
    return np.stack([oracle.std_shuffle_u32(base, s + 1) for s in range(count)])


def row(name: str, perms_by_n: dict, count: int) -> str:
    cells = [name]
    if 5 in perms_by_n:
        chi, _ = stats.chi_square(perms_by_n[5])
        cells.append(f"{chi:,.1f}{' (fail)' if chi > stats.chi_square_critical(119, 0.05) else ''}")
    for n in SIZES:
        z = stats.mmd_z(n, stats.mmd2(perms_by_n[n]), count // 2)
        cells.append(f"{z:+.2f}{' (fail)' if abs(z) > 2.576 else ''}")
    return "| " + " | ".join(cells) + " |"


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--perms", type=int, default=100_000)
    a = ap.parse_args()
    import torch

    import paper_2106_06161_amd as bs

    count = a.perms
    lines = [
        f"Permutations per point: {count:,} (seeds 1..{count:,}); MMD pairs ({count // 2:,}) are (2i, 2i+1).",
        "",
        "| generator | chi-square n=5 | MMD z n=5 | MMD z n=100 | MMD z n=1000 |",
        "|---|---|---|---|---|",
    ]
    t0 = time.time()
    for r in ROUNDS:
        lines.append(row(f"VariablePhilox, {r} rounds", {n: philox_perms(torch, bs, n, r, count) for n in SIZES}, count))
        print(lines[-1], flush=True)
    lines.append(row("LCG", {n: lcg_perms(torch, bs, n, count) for n in SIZES}, count))
    print(lines[-1], flush=True)
    lines.append(row("std::shuffle (mt19937_64)", {n: std_perms(n, count) for n in SIZES}, count))
    print(lines[-1], flush=True)
    lines += ["", f"chi-square critical value (119 dof, alpha 0.05): {stats.chi_square_critical(119, 0.05):.2f}; "
              f"|z| > 2.576 rejects at alpha 0.01.  Wall time {time.time() - t0:.0f} s."]
    text = "\n".join(lines) + "\n"
    print(text)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
