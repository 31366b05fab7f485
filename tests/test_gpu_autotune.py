"""The native autotuner on the GPU, on small size classes: it writes a table
of compiled shapes that the library then uses, it restores a forced shape,
and outputs stay bit-exact whatever shape it picks."""
import numpy as np
import pytest
import torch

import oracle
import paper_2106_06161_amd as bs
from paper_2106_06161_amd import autotune
from paper_2106_06161_amd import binding as B
from paper_2106_06161_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _restore_shipped_table():
    yield
    B.bs_set_config(0, 0, 0, 0)
    assert B.bs_load_tuned_configs(B.TUNED_FILE) == B.BS_OK


def test_autotune_small_classes(tmp_path):
    path = tmp_path / "tuned.txt"
    assert B.bs_set_config(8, 16, 2, 1) == B.BS_OK  # a forced shape survives tuning
    assert B.bs_autotune(0, str(path), 14) == B.BS_OK
    assert B.bs_get_config() == (8, 16, 2, 1)
    assert B.bs_set_config(0, 0, 0, 0) == B.BS_OK
    entries = autotune.read_table(str(path))
    singles = {(e["elem_bytes"], e["size_bits"]) for e in entries if e["kind"] == 0}
    assert singles == {(eb, b) for eb in (1, 2, 4, 8, 16) for b in (12, 13, 14)}
    assert sum(e["kind"] == 1 for e in entries) == 5 * 7
    shapes = [tuple(s) for s in autotune.SHAPES + autotune.COMPACT_SHAPES]
    assert all((e["waves"], e["items"], e["depth"]) in shapes for e in entries)
    e = next(e for e in entries if e["kind"] == 0 and e["elem_bytes"] == 4 and e["size_bits"] == 14)
    assert B.bs_query_config(0, 4, 10_000) == (e["waves"], e["items"], e["depth"], e["grid_mult"])
    # the table is now a cache: a second call loads it without tuning
    path.write_text(path.read_text().replace("rounds 24", "rounds 24  # cached"))
    assert B.bs_autotune(0, str(path), 14) == B.BS_OK
    for n in (5_000, 10_000, 16_384):
        x = W.uniform_u32(n, seed=n)
        y = bs.shuffle(torch.from_numpy(x).to("cuda:0"), 3, 24)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), oracle.shuffle(x, 3, 24)), n
