"""Sec. 5's distribution-quality curves against the round count, with the
permutations generated on the GPU: for each round count, 100,000 shuffles of
arange(n) (seeds 1..100,000) in one batched launch at n = 5, 100 and 1,000;
the chi-square statistic over all 120 orderings at n = 5 and the
Mallows-kernel MMD^2 estimate as a z-score of its null distribution.

The assertions are the paper's qualitative outcomes: chi-square rejects the
cipher below 20 rounds and accepts it at 24 and 32; MMD rejects 2 and 4
rounds at every n and accepts 24 and 32.  The LCG bijection fails both.  The
whole table is written to the file named by BSHUFFLE_QUALITY_OUT when that
variable is set."""
import os

import numpy as np
import pytest
import torch

import paper_2106_06161_amd as bs
from oracle import stats

pytestmark = pytest.mark.gpu

P = 100_000
ROUNDS = [2, 4, 8, 12, 16, 20, 24, 32]
SIZES = [5, 100, 1000]
Z_01 = 2.5758293035489  # two-sided normal quantile at alpha = 0.01


def philox_perms(n, rounds):
    x = torch.arange(n, dtype=torch.int32, device="cuda:0").repeat(P)
    off = torch.arange(P + 1, dtype=torch.int64, device="cuda:0") * n
    sd = torch.arange(1, P + 1, dtype=torch.int64, device="cuda:0")
    y = bs.shuffle_batched(x, off, sd, rounds)
    torch.cuda.synchronize()
    return y.view(P, n).cpu().numpy().astype(np.uint32)


def lcg_perms(n):
    x = torch.arange(n, dtype=torch.int32, device="cuda:0")
    out = torch.empty((P, n), dtype=torch.int32, device="cuda:0")
    for s in range(P):
        bs.shuffle_lcg(x, s + 1, out=out[s])
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.uint32)


def measure(perms_by_n):
    row = {}
    row["chi2"] = stats.chi_square(perms_by_n[5])[0]
    for n in SIZES:
        row[n] = stats.mmd_z(n, stats.mmd2(perms_by_n[n]), P)
    return row


@pytest.fixture(scope="module")
def table():
    rows = {r: measure({n: philox_perms(n, r) for n in SIZES}) for r in ROUNDS}
    rows["LCG"] = measure({n: lcg_perms(n) for n in SIZES})
    out = os.environ.get("BSHUFFLE_QUALITY_OUT")
    if out:
        crit = stats.chi_square_critical(119, 0.05)
        lines = [f"Permutations per point: {P:,} (seeds 1..{P:,}); MMD over {P // 2:,} pairs (2i, 2i+1); "
                 f"z = MMD^2 / sqrt(2 Var K / |Pi|).", "",
                 "| generator | chi-square n=5 | MMD z n=5 | MMD z n=100 | MMD z n=1000 |", "|---|---|---|---|---|"]
        for key, row in rows.items():
            name = "LCG" if key == "LCG" else f"VariablePhilox, {key} rounds"
            cells = [name, f"{row['chi2']:,.1f}" + (" (fail)" if row["chi2"] > crit else "")]
            cells += [f"{row[n]:+.2f}" + (" (fail)" if abs(row[n]) > Z_01 else "") for n in SIZES]
            lines.append("| " + " | ".join(cells) + " |")
        lines += ["", f"chi-square critical value (119 dof, alpha 0.05): {crit:.2f}; |z| > {Z_01:.3f} "
                  "rejects at alpha 0.01."]
        with open(out, "w") as fh:
            fh.write("\n".join(lines) + "\n")
    return rows


def test_chi_square_against_rounds(table):
    crit = stats.chi_square_critical(119, 0.05)
    for r in (2, 4, 8, 12, 16):
        assert table[r]["chi2"] > crit, (r, table[r]["chi2"])
    for r in (24, 32):
        assert table[r]["chi2"] < crit, (r, table[r]["chi2"])


@pytest.mark.parametrize("n", SIZES)
def test_mmd_against_rounds(table, n):
    for r in (2, 4):
        assert table[r][n] > Z_01, (r, n, table[r][n])
    for r in (24, 32):
        assert abs(table[r][n]) < Z_01, (r, n, table[r][n])


def test_lcg_fails_both(table):
    assert table["LCG"]["chi2"] > 1000 * stats.chi_square_critical(119, 0.05)
    for n in SIZES:
        assert table["LCG"][n] > Z_01, (n, table["LCG"][n])
