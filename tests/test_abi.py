"""The C ABI on the host: the library loads, exports every declared symbol,
and rejects bad arguments before touching a device (no GPU needed)."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2106_06161_amd import binding as B


@pytest.fixture(scope="module")
def lib():
    return B.lib()


def test_every_declared_symbol_is_exported(lib):
    names = B.declared_functions()
    assert "bs_shuffle" in names and "bs_shuffle_batched" in names
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code in range(9):
        assert B.status_string(code).startswith("BS_")
    assert "unknown" in B.status_string(99)


@pytest.mark.parametrize("n", [0, 1, 2, 5, 16, 17, 100_000, (1 << 27) + 1, 10**9, (1 << 38) - 1])
def test_domain_bits_matches_oracle(n):
    assert B.bs_domain_bits(n) == oracle.domain_bits(n)


@pytest.mark.parametrize("seed", [0, 1, 42, 2**64 - 1])
def test_round_keys_match_oracle(seed):
    assert B.bs_round_keys(seed, 64) == list(oracle.round_keys(seed, 64))


def test_workspace_bytes(lib):
    w1 = B.bs_workspace_bytes(100_000)
    assert w1 >= 256 + 8 * ((1 << 17) // 2048)
    w2 = B.bs_workspace_bytes((1 << 27) + 1)
    assert w2 >= 256 + 8 * ((1 << 28) // 2048)
    wb = B.bs_workspace_bytes(445_000_000, 4096)
    assert wb > w2


FAKE_IN, FAKE_OUT = 1 << 40, 1 << 41  # never dereferenced: validation fails first


@pytest.mark.parametrize("eb", [0, 3, 5, 12, 32])
def test_rejects_bad_elem_bytes(eb):
    assert B.bs_shuffle(FAKE_IN, FAKE_OUT, 10, eb, 1, 24, None, 0, None) == B.BS_EELEM


def test_rejects_misaligned():
    assert B.bs_shuffle(FAKE_IN + 2, FAKE_OUT, 10, 4, 1, 24, None, 0, None) == B.BS_EELEM
    assert B.bs_shuffle(FAKE_IN, FAKE_OUT + 8, 10, 16, 1, 24, None, 0, None) == B.BS_EELEM


def test_rejects_bad_rounds_and_sizes():
    assert B.bs_shuffle(FAKE_IN, FAKE_OUT, 10, 4, 1, 65, None, 0, None) == B.BS_EINVAL
    assert B.bs_shuffle(FAKE_IN, FAKE_OUT, 1 << 38, 4, 1, 24, None, 0, None) == B.BS_EINVAL


def test_rejects_null_and_alias():
    assert B.bs_shuffle(None, FAKE_OUT, 10, 4, 1, 24, None, 0, None) == B.BS_EINVAL
    assert B.bs_shuffle(FAKE_IN, None, 10, 4, 1, 24, None, 0, None) == B.BS_EINVAL
    assert B.bs_shuffle(FAKE_IN, FAKE_IN, 10, 4, 1, 24, None, 0, None) == B.BS_EALIAS
    assert B.bs_shuffle(FAKE_IN, FAKE_IN + 36, 10, 4, 1, 24, None, 0, None) == B.BS_EALIAS
    assert B.bs_shuffle(FAKE_IN + 36, FAKE_IN, 10, 4, 1, 24, None, 0, None) == B.BS_EALIAS


def test_zero_items_is_a_noop():
    assert B.bs_shuffle(None, None, 0, 4, 1, 24, None, 0, None) == B.BS_OK
    assert B.bs_shuffle_batched(None, None, None, None, 0, 0, 4, 24, None, 0, None) == B.BS_OK


def test_batched_rejects_bad_arguments():
    assert B.bs_shuffle_batched(FAKE_IN, FAKE_OUT, None, 1, 3, 10, 4, 24, None, 0, None) == B.BS_EINVAL
    assert B.bs_shuffle_batched(FAKE_IN, FAKE_OUT, 1, 1, 3, 10, 3, 24, None, 0, None) == B.BS_EELEM
    assert B.bs_shuffle_batched(FAKE_IN, FAKE_IN, 8, 8, 3, 10, 4, 24, None, 0, None) == B.BS_EALIAS
    assert B.bs_shuffle_batched(FAKE_IN, FAKE_OUT, 8, 8, 3, 10, 4, 99, None, 0, None) == B.BS_EINVAL


def test_user_workspace_too_small_is_rejected():
    assert B.bs_shuffle(FAKE_IN, FAKE_OUT, 100_000, 4, 1, 24, 1 << 42, 64, None) == B.BS_ENOMEM


def test_config_round_trip():
    before = B.bs_get_config()
    assert B.bs_set_config(8, 8, 2, 2) == B.BS_OK
    assert B.bs_get_config() == (8, 8, 2, 2)
    assert B.bs_set_config(3, 8, 1, 0) == B.BS_EINVAL
    assert B.bs_set_config(8, 8, 1, 0) == B.BS_EINVAL
    assert B.bs_set_config(8, 16, 1, 65) == B.BS_EINVAL
    assert B.bs_set_config(8, 16, 1, B.GRID_ONE_PER_TILE) == B.BS_OK
    assert B.bs_set_config(16, 8, B.DEPTH_COMPACT, 0) == B.BS_OK
    assert B.bs_get_config() == (16, 8, B.DEPTH_COMPACT, 0)
    assert B.bs_set_config(16, 4, B.DEPTH_COMPACT, 0) == B.BS_EINVAL
    assert B.bs_set_config(0, 0, 0, 0) == B.BS_OK
    assert B.bs_get_config() == before


def test_forced_shape_applies_to_both_call_kinds():
    """A forced shape applies to single and batched launches, except that
    domains above 2^32 always run the 64-bit index shape."""
    try:
        assert B.bs_set_config(16, 8, B.DEPTH_COMPACT, 0) == B.BS_OK
        assert B.bs_query_config(0, 4, 1 << 20) == (16, 8, B.DEPTH_COMPACT, 0)
        assert B.bs_query_config(1, 4, 1 << 20, 16) == (16, 8, B.DEPTH_COMPACT, 0)
        assert B.bs_set_config(8, 8, B.DEPTH_COMPACT_PIPE, 1) == B.BS_OK
        assert B.bs_query_config(1, 4, 1 << 20, 16) == (8, 8, B.DEPTH_COMPACT_PIPE, 1)
        assert B.bs_query_config(0, 4, (1 << 32) + 1) == (16, 8, B.DEPTH_COMPACT_PIPE, 1)  # 64-bit index path
    finally:
        B.bs_set_config(0, 0, 0, 0)


def test_probe_argument_checks():
    assert B.bs_probe_copy(FAKE_IN + 4, FAKE_OUT, 64, None) == B.BS_EELEM
    assert B.bs_probe_copy(FAKE_IN, FAKE_IN + 16, 64, None) == B.BS_EALIAS
    assert B.bs_probe_gather(FAKE_IN, 10, FAKE_OUT, None, 10, 4, None) == B.BS_EINVAL
    assert B.bs_probe_cipher_scan(10, 1, 99, None, 0, None) == B.BS_EINVAL


def test_tuned_config_table():
    assert B.bs_set_tuned_config(0, 4, 28, 16, 16, 1, 0) == B.BS_OK
    assert B.bs_set_tuned_config(1, 8, 12, 8, 16, 2, 1) == B.BS_OK
    assert B.bs_set_tuned_config(2, 4, 28, 16, 16, 1, 0) == B.BS_EINVAL  # kind
    assert B.bs_set_tuned_config(0, 3, 28, 16, 16, 1, 0) == B.BS_EINVAL  # element size
    assert B.bs_set_tuned_config(0, 4, 41, 16, 16, 1, 0) == B.BS_EINVAL  # size class
    assert B.bs_set_tuned_config(0, 4, 28, 16, 4, 1, 0) == B.BS_EINVAL   # shape not compiled
    assert B.bs_clear_tuned_configs() == B.BS_OK
    assert B.bs_load_tuned_configs(B.TUNED_FILE) == B.BS_OK


def test_shipped_tuned_table_is_valid():
    from paper_2106_06161_amd import autotune

    entries = autotune.read_table()
    assert len(entries) >= 90
    shapes = [tuple(s) for s in autotune.SHAPES + autotune.COMPACT_SHAPES]
    for e in entries:
        assert (e["waves"], e["items"], e["depth"]) in shapes and e["grid_mult"] in autotune.GRIDS
    assert B.bs_load_tuned_configs(B.TUNED_FILE) == B.BS_OK
    # the table decides the form and launch shape the library reports
    e = next(e for e in entries if e["kind"] == 0 and e["elem_bytes"] == 4 and e["size_bits"] == 28)
    staged = {(t["elem_bytes"], t["size_bits"]): t["prefer"] for t in autotune.read_staged()}
    if staged.get((4, 28)):
        assert B.bs_query_config(0, 4, (1 << 27) + 1) == (0, 0, B.DEPTH_STAGED, 0)
    else:
        assert B.bs_query_config(0, 4, (1 << 27) + 1) == (e["waves"], e["items"], e["depth"], e["grid_mult"])
    # 16-byte records stay with the fused kernel at 2^28
    e16 = next(e for e in entries if e["kind"] == 0 and e["elem_bytes"] == 16 and e["size_bits"] == 28)
    if not staged.get((16, 28)):
        assert B.bs_query_config(0, 16, 250_000_000) == (e16["waves"], e16["items"], e16["depth"], e16["grid_mult"])


def test_tuned_table_files_round_trip(tmp_path):
    """Saving and loading a table keeps every entry; a malformed or
    non-compiled entry is rejected and leaves the table unchanged."""
    from paper_2106_06161_amd import autotune

    assert B.bs_load_tuned_configs(B.TUNED_FILE) == B.BS_OK
    out = tmp_path / "t.txt"
    assert B.bs_save_tuned_configs(str(out)) == B.BS_OK
    key = lambda e: (e["kind"], e["elem_bytes"], e["size_bits"], e["waves"], e["items"], e["depth"], e["grid_mult"])
    assert sorted(map(key, autotune.read_table(str(out)))) == sorted(map(key, autotune.read_table()))
    before = B.bs_query_config(0, 4, (1 << 27) + 1)
    bad = tmp_path / "bad.txt"
    bad.write_text("arch gfx950\n0 4 28 16 4 1 0\n")  # 16 waves x 4 items is not compiled
    assert B.bs_load_tuned_configs(str(bad)) == B.BS_EINVAL
    bad.write_text("0 4 28 16\n")
    assert B.bs_load_tuned_configs(str(bad)) == B.BS_EINVAL
    assert B.bs_load_tuned_configs(str(tmp_path / "missing.txt")) == B.BS_EINVAL
    assert B.bs_query_config(0, 4, (1 << 27) + 1) == before


def test_autotune_without_a_device():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present (the GPU test runs the tuner)")
    assert B.bs_autotune(0, None) == B.BS_ENODEV
    assert B.bs_autotune(0, None, 0, 2) in (B.BS_EINVAL, B.BS_ENODEV)


def test_permutation_and_unshuffle_argument_checks():
    assert B.bs_permutation(FAKE_OUT, 10, 2, 1, 24, None, 0, None) == B.BS_EELEM
    assert B.bs_permutation(FAKE_OUT + 2, 10, 4, 1, 24, None, 0, None) == B.BS_EELEM
    assert B.bs_permutation(FAKE_OUT, (1 << 32) + 1, 4, 1, 24, None, 0, None) == B.BS_EINVAL
    assert B.bs_permutation(None, 10, 4, 1, 24, None, 0, None) == B.BS_EINVAL
    assert B.bs_permutation(None, 0, 4, 1, 24, None, 0, None) == B.BS_OK
    assert B.bs_unshuffle(FAKE_IN, FAKE_IN, 10, 4, 1, 24, None, 0, None) == B.BS_EALIAS
    assert B.bs_unshuffle(FAKE_IN, FAKE_OUT, 10, 3, 1, 24, None, 0, None) == B.BS_EELEM
    assert B.bs_unshuffle(FAKE_IN, FAKE_OUT, 10, 4, 1, 65, None, 0, None) == B.BS_EINVAL
    assert B.bs_probe_shuffle_two_pass(FAKE_IN, FAKE_OUT, (1 << 32) + 1, 4, 1, 24, None, 0, None) == B.BS_EINVAL
    assert B.bs_probe_shuffle_unfused(FAKE_IN, FAKE_OUT, 100, 4, 1, 24, 1 << 42, 16, None, 0, None) == B.BS_ENOMEM
    assert B.bs_probe_unfused_scratch_bytes(100_000) >= 4 * (1 << 17) + 4 * 100_000


@pytest.mark.parametrize("n", [1, 5, 16, 17, 1000, 65_537, 1 << 30, (1 << 32) + 1])
def test_lcg_params_match_oracle(n):
    for seed in (0, 1, 2**63 + 5):
        assert B.bs_lcg_params(n, seed) == oracle.lcg_params(n, seed)


def test_lcg_argument_checks():
    assert B.bs_shuffle_lcg(FAKE_IN, FAKE_IN, 10, 4, 1, None, 0, None) == B.BS_EALIAS
    assert B.bs_shuffle_lcg(FAKE_IN, FAKE_OUT, 10, 3, 1, None, 0, None) == B.BS_EELEM
    assert B.bs_shuffle_lcg(None, FAKE_OUT, 10, 4, 1, None, 0, None) == B.BS_EINVAL
    assert B.bs_shuffle_lcg(None, None, 0, 4, 1, None, 0, None) == B.BS_OK
    assert B.bs_shuffle_lcg(FAKE_IN, FAKE_OUT, B.MAX_ITEMS + 1, 1, 1, None, 0, None) == B.BS_EINVAL


def test_bijection_argument_checks():
    for k, rounds, inv in [(0, 24, 0), (41, 24, 0), (10, 65, 0), (10, 24, 2)]:
        assert B.bs_bijection(FAKE_IN, FAKE_OUT, 8, k, 1, rounds, inv, None) == B.BS_EINVAL
    assert B.bs_bijection(None, FAKE_OUT, 8, 10, 1, 24, 0, None) == B.BS_EINVAL
    assert B.bs_bijection(FAKE_IN + 4, FAKE_OUT, 8, 10, 1, 24, 0, None) == B.BS_EELEM
    assert B.bs_bijection(None, None, 0, 40, 1, 64, 1, None) == B.BS_OK


def test_unshuffle_inverse_argument_checks():
    need = B.bs_unshuffle_inverse_scratch_bytes(1000)
    assert need >= (1024 // 32) * 8 and need % 256 == 0
    assert B.bs_unshuffle_inverse_scratch_bytes(B.MAX_ITEMS + 1) == 0
    # about 2^k / 4 bytes: one 8-byte entry per 32 indices plus per-tile words
    assert B.bs_unshuffle_inverse_scratch_bytes(1 << 28) <= (1 << 26) + (1 << 19)
    S = 1 << 42
    assert B.bs_unshuffle_inverse(FAKE_IN, FAKE_OUT, 1000, 3, 1, 24, S, need, None) == B.BS_EELEM
    assert B.bs_unshuffle_inverse(FAKE_IN, FAKE_OUT, 1000, 4, 1, 65, S, need, None) == B.BS_EINVAL
    assert B.bs_unshuffle_inverse(FAKE_IN, FAKE_OUT, 1000, 4, 1, 24, None, need, None) == B.BS_EINVAL
    assert B.bs_unshuffle_inverse(FAKE_IN, FAKE_OUT, 1000, 4, 1, 24, S + 16, need, None) == B.BS_EINVAL
    assert B.bs_unshuffle_inverse(FAKE_IN, FAKE_OUT, 1000, 4, 1, 24, S, need - 1, None) == B.BS_ENOMEM
    assert B.bs_unshuffle_inverse(FAKE_IN, FAKE_IN, 1000, 4, 1, 24, S, need, None) == B.BS_EALIAS
    assert B.bs_unshuffle_inverse(None, None, 0, 4, 1, 24, None, 0, None) == B.BS_OK


def test_batch_small_argument_check():
    assert B.bs_probe_set_batch_small(2) == B.BS_EINVAL
    for m in (0, 1):
        assert B.bs_probe_set_batch_small(m) == B.BS_OK


def test_random_reads_probe_argument_checks():
    assert B.bs_probe_random_reads(None, 1 << 10, FAKE_OUT, 0, None) == B.BS_EINVAL
    assert B.bs_probe_random_reads(FAKE_IN, 1000, FAKE_OUT, 0, None) == B.BS_EINVAL  # not a power of two
    assert B.bs_probe_random_reads(FAKE_IN, 8, FAKE_OUT, 0, None) == B.BS_EINVAL  # fewer than 16 words
    assert B.bs_probe_random_reads(FAKE_IN, (1 << 32) * 2, FAKE_OUT, 0, None) == B.BS_EINVAL
    assert B.bs_probe_random_reads(FAKE_IN + 2, 1 << 10, FAKE_OUT, 0, None) == B.BS_EELEM


def test_random_reads_region_probe_argument_checks():
    f = B.bs_probe_random_reads_region
    assert f(None, 1 << 20, 4, 1 << 10, FAKE_OUT, 0, None) == B.BS_EINVAL
    assert f(FAKE_IN, 1 << 20, 2, 1 << 10, FAKE_OUT, 0, None) == B.BS_EELEM  # record size
    assert f(FAKE_IN + 8, 1 << 20, 16, 1 << 10, FAKE_OUT, 0, None) == B.BS_EELEM  # misaligned for 16 B
    assert f(FAKE_IN, 3 << 20, 4, 1 << 10, FAKE_OUT, 0, None) == B.BS_EINVAL  # records not a power of two
    assert f(FAKE_IN, (1 << 20) + 4, 8, 1 << 10, FAKE_OUT, 0, None) == B.BS_EINVAL  # not whole records
    assert f(FAKE_IN, 16 << 32, 4, 1 << 10, FAKE_OUT, 0, None) == B.BS_EINVAL  # more than 2^32 records
    assert f(FAKE_IN, 1 << 20, 4, 24, FAKE_OUT, 0, None) == B.BS_EINVAL  # reads not a multiple of 16
    assert f(FAKE_IN, 1 << 20, 4, 1 << 37, FAKE_OUT, 0, None) == B.BS_EINVAL  # more than 2^36 reads


def test_xcd_mode_argument_check():
    assert B.bs_probe_set_xcd_mode(3) == B.BS_EINVAL
    for m in (0, 1, 2):
        assert B.bs_probe_set_xcd_mode(m) == B.BS_OK


def test_tuned_lookup_falls_back_to_nearest_class():
    try:
        assert B.bs_clear_tuned_configs() == B.BS_OK
        assert B.bs_set_tuned_config(0, 4, 20, 8, 8, 2, 1) == B.BS_OK
        assert B.bs_set_tuned_config(0, 4, 24, 16, 8, 9, 1) == B.BS_OK
        assert B.bs_set_tuned_config(0, 8, 30, 16, 16, 1, 2) == B.BS_OK
        assert B.bs_query_config(0, 4, 1 << 24) == (16, 8, 9, 1)
        assert B.bs_query_config(0, 4, 1 << 22) == (8, 8, 2, 1)        # largest class below
        assert B.bs_query_config(0, 4, (1 << 31) + 1) == (16, 8, 9, 1)  # k = 32: still below
        assert B.bs_query_config(0, 4, 100) == (8, 8, 2, 1)            # smallest class above
        assert B.bs_query_config(0, 8, 1 << 20) == (16, 16, 1, 2)      # other element size's own entries
        assert B.bs_query_config(0, 16, 1 << 20) == B.bs_get_config()  # none for this size: default
    finally:
        B.bs_load_tuned_configs(B.TUNED_FILE)


def test_watchdog_argument_check():
    assert B.bs_probe_set_watchdog(100, 2) == B.BS_EINVAL
    assert B.bs_probe_set_watchdog(0, 0) == B.BS_OK


def test_tensor_wrappers_check_out_and_devices(monkeypatch):
    """shuffle / shuffle_batched reject an `out` that does not match x (a
    smaller one would take out-of-bounds device writes) and batch tables on
    another device, before any pointer reaches the library.  Meta tensors
    stand in for device tensors (no GPU here)."""
    import torch

    monkeypatch.setattr(B, "_require_device", lambda t, name: None)
    x = torch.empty(1000, dtype=torch.int32, device="meta")
    off = torch.empty(3, dtype=torch.int64, device="meta")
    sd = torch.empty(2, dtype=torch.int64, device="meta")
    for bad in (torch.empty(999, dtype=torch.int32, device="meta"),
                torch.empty(1000, dtype=torch.int64, device="meta"),
                torch.empty((1000, 2), dtype=torch.int32, device="meta")):
        with pytest.raises(ValueError, match="out must match"):
            B.shuffle_batched(x, off, sd, out=bad)
        with pytest.raises(ValueError, match="out must match"):
            B.shuffle(x, 1, out=bad)
    with pytest.raises(ValueError, match="offsets must be on"):
        B.shuffle_batched(x, torch.zeros(3, dtype=torch.int64), sd)
    with pytest.raises(ValueError, match="seeds must be on"):
        B.shuffle_batched(x, off, torch.zeros(2, dtype=torch.int64))


def test_noalloc_argument_checks():
    """bs_shuffle_noalloc rejects what bs_shuffle rejects, and n above its
    static array's limit (2^30 records) with BS_ENOMEM, before any device work."""
    assert B.bs_shuffle_noalloc(None, None, 0, 4, 1, 24, None) == B.BS_OK
    assert B.bs_shuffle_noalloc(FAKE_IN, FAKE_OUT, 10, 3, 1, 24, None) == B.BS_EELEM
    assert B.bs_shuffle_noalloc(FAKE_IN, FAKE_OUT, 10, 4, 1, 65, None) == B.BS_EINVAL
    assert B.bs_shuffle_noalloc(None, FAKE_OUT, 10, 4, 1, 24, None) == B.BS_EINVAL
    assert B.bs_shuffle_noalloc(FAKE_IN, FAKE_IN, 10, 4, 1, 24, None) == B.BS_EALIAS
    assert B.bs_shuffle_noalloc(FAKE_IN, FAKE_OUT, B.NOALLOC_MAX_ITEMS + 1, 4, 1, 24, None) == B.BS_ENOMEM



def test_staged_scratch_sizes_and_argument_checks():
    # n = 2^27 + 1 uint32: k = 28, windows of 2^14, passes of 8 and 6 digit
    # bits (2^8 bucket counts); bucket arrays of 2^28 entries: 4-byte indices
    # and records, then 2-byte window indices and records
    want = 4 * (1 << 8) + 2 * 4 * (1 << 14) + (1 << 28) * (4 + 4 + 2 + 4)
    assert B.bs_staged_scratch_bytes((1 << 27) + 1, 4) == want
    assert B.bs_staged_scratch_bytes(0, 4) == 0
    assert B.bs_staged_scratch_bytes(1000, 3) == 0
    assert B.bs_staged_scratch_bytes((1 << 32) + 1, 4) == 0  # domain above 2^32
    assert B.bs_staged_scratch_bytes(1 << 31, 8) > 0 and B.bs_staged_scratch_bytes((1 << 31) + 1, 8) == 0
    n = 1 << 20
    need = B.bs_staged_scratch_bytes(n, 4)
    f = B.bs_shuffle_staged
    assert f(FAKE_IN, FAKE_OUT, n, 4, 1, 24, None, need, None) == B.BS_EINVAL
    assert f(FAKE_IN, FAKE_OUT, n, 4, 1, 24, 1 << 42, need - 1, None) == B.BS_ENOMEM
    assert f(FAKE_IN, FAKE_OUT, n, 4, 1, 24, (1 << 42) + 64, need, None) == B.BS_EINVAL
    assert f(FAKE_IN, FAKE_OUT, n, 4, 1, 24, FAKE_IN - 256, need, None) == B.BS_EALIAS
    assert f(FAKE_IN, FAKE_OUT, n, 3, 1, 24, 1 << 42, need, None) == B.BS_EELEM
    assert f(FAKE_IN, FAKE_OUT, n, 4, 1, 65, 1 << 42, need, None) == B.BS_EINVAL
    assert f(FAKE_IN, FAKE_OUT, (1 << 32) + 1, 4, 1, 24, 1 << 42, 1 << 40, None) == B.BS_EINVAL
    assert f(FAKE_IN, FAKE_OUT, 0, 4, 1, 24, None, 0, None) == B.BS_OK


def test_unshuffle_staged_scratch_sizes_and_argument_checks():
    # the staged form's scratch, then one key word per padded index (2^28)
    # and two words per tile of 8,192 padded indices (2^15 tiles)
    n = (1 << 27) + 1
    assert B.bs_unshuffle_staged_scratch_bytes(n, 4) == B.bs_staged_scratch_bytes(n, 4) + 4 * (1 << 28) + 8 * (1 << 15)
    # 8- and 16-byte records: tiles of 8,192 and 4,096 padded indices
    assert B.bs_unshuffle_staged_scratch_bytes(n, 8) == (B.bs_staged_scratch_bytes(n, 8) + 4 * (1 << 28)
                                                          + 8 * (1 << 15))
    assert B.bs_unshuffle_staged_scratch_bytes(n, 16) == (B.bs_staged_scratch_bytes(n, 16) + 4 * (1 << 28)
                                                           + 8 * (1 << 16))
    # a domain smaller than one tile: one tile's key words, one count and prefix
    assert B.bs_unshuffle_staged_scratch_bytes(1000, 4) == B.bs_staged_scratch_bytes(1000, 4) + 4 * 8192 + 2 * 256
    assert B.bs_unshuffle_staged_scratch_bytes(0, 4) == 0
    assert B.bs_unshuffle_staged_scratch_bytes(1000, 3) == 0
    assert B.bs_unshuffle_staged_scratch_bytes((1 << 32) + 1, 4) == 0
    n = 1 << 20
    need = B.bs_unshuffle_staged_scratch_bytes(n, 4)
    f = B.bs_unshuffle_staged
    assert f(FAKE_IN, FAKE_OUT, n, 4, 1, 24, None, need, None) == B.BS_EINVAL
    assert f(FAKE_IN, FAKE_OUT, n, 4, 1, 24, 1 << 42, need - 1, None) == B.BS_ENOMEM
    assert f(FAKE_IN, FAKE_OUT, n, 4, 1, 24, (1 << 42) + 64, need, None) == B.BS_EINVAL
    assert f(FAKE_IN, FAKE_OUT, n, 4, 1, 24, FAKE_IN - 256, need, None) == B.BS_EALIAS
    assert f(FAKE_IN, FAKE_OUT, n, 3, 1, 24, 1 << 42, need, None) == B.BS_EELEM
    assert f(FAKE_IN, FAKE_OUT, n, 4, 1, 65, 1 << 42, need, None) == B.BS_EINVAL
    assert f(FAKE_IN, FAKE_OUT, (1 << 32) + 1, 4, 1, 24, 1 << 42, 1 << 40, None) == B.BS_EINVAL
    assert f(FAKE_IN, FAKE_OUT, 0, 4, 1, 24, None, 0, None) == B.BS_OK


def test_staged_workspace_bytes_and_policy():
    n = (1 << 27) + 1
    fused = B.bs_workspace_bytes(n, 0, 4)
    assert B.bs_workspace_bytes_staged(n, 4) == ((fused + 255) // 256) * 256 + B.bs_staged_scratch_bytes(n, 4)
    # sizes the staged form does not cover: just the fused workspace
    assert B.bs_workspace_bytes_staged((1 << 32) + 1, 4) == B.bs_workspace_bytes((1 << 32) + 1, 0, 4)
    assert B.bs_workspace_bytes_staged(n, 3) == 0
    assert B.bs_probe_set_staged_policy(3) == B.BS_EINVAL
    for mode in (0, 1, 2):
        assert B.bs_probe_set_staged_policy(mode) == B.BS_OK


def test_staged_table_lines(tmp_path):
    """A "staged" line makes bs_query_config report the staged form for that
    class; saving keeps it; a malformed staged line is rejected."""
    from paper_2106_06161_amd import autotune

    t = tmp_path / "t.txt"
    t.write_text("arch gfx950\nrounds 24\n0 4 28 16 16 9 1\nstaged 4 28 1 1.7 2.4\nstaged 8 28 0\n")
    try:
        assert B.bs_load_tuned_configs(str(t)) == B.BS_OK
        assert B.bs_query_config(0, 4, (1 << 27) + 1) == (0, 0, B.DEPTH_STAGED, 0)
        assert B.bs_query_config(0, 8, (1 << 27) + 1)[2] != B.DEPTH_STAGED
        # classes without a line take the nearest listed class below them
        assert B.bs_query_config(0, 4, (1 << 30) + 1) == (0, 0, B.DEPTH_STAGED, 0)
        assert B.bs_query_config(0, 4, (1 << 26) + 1)[2] != B.DEPTH_STAGED
        assert B.bs_query_config(0, 8, (1 << 30) + 1)[2] != B.DEPTH_STAGED
        assert B.bs_query_config(0, 2, (1 << 30) + 1)[2] != B.DEPTH_STAGED
        out = tmp_path / "out.txt"
        assert B.bs_save_tuned_configs(str(out)) == B.BS_OK
        assert [(e["elem_bytes"], e["size_bits"], e["prefer"]) for e in autotune.read_staged(str(out))] == [
            (4, 28, True), (8, 28, False)]
        assert B.bs_probe_set_staged_policy(0) == B.BS_OK
        assert B.bs_query_config(0, 4, (1 << 27) + 1)[2] != B.DEPTH_STAGED
        bad = tmp_path / "bad.txt"
        bad.write_text("staged 4 28 2\n")
        assert B.bs_load_tuned_configs(str(bad)) == B.BS_EINVAL
    finally:
        B.bs_probe_set_staged_policy(2)
        assert B.bs_load_tuned_configs(B.TUNED_FILE) == B.BS_OK


def test_int_rate_probe_argument_checks():
    f = B.bs_probe_int_rate
    assert f(0, 16, None, 8, None) == B.BS_EINVAL
    assert f(6, 16, FAKE_OUT, 8, None) == B.BS_EINVAL
    assert f(0, 0, FAKE_OUT, 8, None) == B.BS_EINVAL
    assert f(0, (1 << 20) + 1, FAKE_OUT, 8, None) == B.BS_EINVAL
    assert f(0, 16, FAKE_OUT, 0, None) == B.BS_EINVAL
    assert f(0, 16, FAKE_OUT, 65537, None) == B.BS_EINVAL
    assert f(0, 16, FAKE_OUT + 2, 8, None) == B.BS_EELEM


def test_round_trip_probe_argument_checks():
    f = B.bs_probe_round_trips
    assert f(None, 32, 4, None) == B.BS_EINVAL
    assert f(FAKE_OUT, 0, 4, None) == B.BS_EINVAL
    assert f(FAKE_OUT, 65537, 4, None) == B.BS_EINVAL
    assert f(FAKE_OUT, 32, 1025, None) == B.BS_EINVAL
    assert f(FAKE_OUT + 2, 32, 4, None) == B.BS_EELEM
