"""MI355X-native bijective shuffle (arXiv 2106.06161), HIP kernels for gfx950.

    import paper_2106_06161_amd as bs
    y = bs.shuffle(x, seed=7, rounds=24)           # x: GPU tensor, permuted along dim 0
    y = bs.shuffle_batched(x, offsets, seeds)      # many independent shuffles, one launch

The work runs in libbshuffle.so (C ABI in include/bshuffle.h); this package
only marshals arguments.  Importing it does not load the library; the first
call does, and raises if the library has not been built.
"""
from .binding import (  # noqa: F401
    DEFAULT_ROUNDS,
    MAX_ITEMS,
    MAX_ROUNDS,
    BShuffleError,
    bijection,
    bs_bijection,
    bs_domain_bits,
    bs_get_config,
    bs_lcg_params,
    bs_round_keys,
    bs_set_config,
    bs_shuffle,
    bs_shuffle_batched,
    bs_workspace_bytes,
    bs_workspace_error,
    bs_workspace_init,
    make_workspace,
    permutation,
    shuffle,
    shuffle_batched,
    shuffle_lcg,
    shuffle_staged,
    staged_scratch_bytes,
    unshuffle,
    unshuffle_inverse,
    unshuffle_staged,
    unshuffle_staged_scratch_bytes,
    workspace_bytes,
    workspace_error,
    workspace_error_async,
)

__version__ = "0.1.0"
