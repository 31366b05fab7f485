"""ctypes binding of libbshuffle.so (argument marshalling only).

The raw entry points keep the C names (``bs_shuffle``, ``bs_shuffle_batched``,
...) and take integers for pointers and streams.  ``shuffle`` and
``shuffle_batched`` wrap them for torch tensors: the tensors' device memory
is passed straight to the library, and the work is enqueued on the tensor's
current torch (HIP) stream.  Every step of the shuffle runs in the library's
HIP kernels; there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os
import re

_PKG = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_PKG)
LIB_PATH = os.path.join(_PKG, "libbshuffle.so")
TUNED_FILE = os.path.join(_PKG, "tuned_configs.txt")  # shipped table (bs_autotune format)
HEADERS = [os.path.join(_ROOT, "include", h) for h in ("bshuffle.h", "bshuffle_probe.h")]

BS_OK, BS_EINVAL, BS_EALIAS, BS_EELEM, BS_ENOMEM, BS_EHIP, BS_ETIMEOUT, BS_ENODEV, BS_EDEVICE = range(9)
MAX_ROUNDS = 64
MAX_ITEMS = (1 << 38) - 1
DEFAULT_ROUNDS = 24  # the round count the paper recommends (Sec. 5)


class BShuffleError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} (status {status})")


_lib = None

_u32, _u64, _i32, _sz, _vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_size_t, ctypes.c_void_p

_SIGNATURES = {
    "bs_status_string": (ctypes.c_char_p, [_i32]),
    "bs_last_hip_error": (_i32, []),
    "bs_version": (_u32, []),
    "bs_domain_bits": (_u32, [_u64]),
    "bs_round_keys": (_i32, [_u64, _u32, _vp]),
    "bs_workspace_bytes": (_sz, [_u64, _u32, _u32]),
    "bs_workspace_init": (_i32, [_vp, _sz, _vp]),
    "bs_workspace_error": (_i32, [_vp, _vp]),
    "bs_workspace_error_async": (_i32, [_vp, _vp, _vp]),
    "bs_shuffle": (_i32, [_vp, _vp, _u64, _u32, _u64, _u32, _vp, _sz, _vp]),
    "bs_shuffle_batched": (_i32, [_vp, _vp, _vp, _vp, _u32, _u64, _u32, _u32, _vp, _sz, _vp]),
    "bs_shuffle_noalloc": (_i32, [_vp, _vp, _u64, _u32, _u64, _u32, _vp]),
    "bs_set_config": (_i32, [_u32, _u32, _u32, _u32]),
    "bs_get_config": (_i32, [_vp, _vp, _vp, _vp]),
    "bs_set_tuned_config": (_i32, [_u32, _u32, _u32, _u32, _u32, _u32, _u32]),
    "bs_clear_tuned_configs": (_i32, []),
    "bs_query_config": (_i32, [_u32, _u32, _u64, _u32, _vp, _vp, _vp, _vp]),
    "bs_permutation": (_i32, [_vp, _u64, _u32, _u64, _u32, _vp, _sz, _vp]),
    "bs_unshuffle": (_i32, [_vp, _vp, _u64, _u32, _u64, _u32, _vp, _sz, _vp]),
    "bs_lcg_params": (_i32, [_u64, _u64, _vp, _vp]),
    "bs_shuffle_lcg": (_i32, [_vp, _vp, _u64, _u32, _u64, _vp, _sz, _vp]),
    "bs_bijection": (_i32, [_vp, _vp, _u64, _u32, _u64, _u32, _u32, _vp]),
    "bs_unshuffle_inverse_scratch_bytes": (_sz, [_u64]),
    "bs_unshuffle_inverse": (_i32, [_vp, _vp, _u64, _u32, _u64, _u32, _vp, _sz, _vp]),
    "bs_staged_scratch_bytes": (_sz, [_u64, _u32]),
    "bs_workspace_bytes_staged": (_sz, [_u64, _u32]),
    "bs_probe_set_staged_policy": (_i32, [_u32]),
    "bs_shuffle_staged": (_i32, [_vp, _vp, _u64, _u32, _u64, _u32, _vp, _sz, _vp]),
    "bs_unshuffle_staged_scratch_bytes": (_sz, [_u64, _u32]),
    "bs_unshuffle_staged": (_i32, [_vp, _vp, _u64, _u32, _u64, _u32, _vp, _sz, _vp]),
    "bs_autotune": (_i32, [ctypes.c_int, ctypes.c_char_p, _u32, _u32]),
    "bs_load_tuned_configs": (_i32, [ctypes.c_char_p]),
    "bs_save_tuned_configs": (_i32, [ctypes.c_char_p]),
    "bs_probe_shuffle_two_pass": (_i32, [_vp, _vp, _u64, _u32, _u64, _u32, _vp, _sz, _vp]),
    "bs_probe_unfused_scratch_bytes": (_sz, [_u64]),
    "bs_probe_shuffle_unfused": (_i32, [_vp, _vp, _u64, _u32, _u64, _u32, _vp, _sz, _vp, _sz, _vp]),
    "bs_probe_copy": (_i32, [_vp, _vp, _u64, _vp]),
    "bs_probe_gather": (_i32, [_vp, _u64, _vp, _vp, _u64, _u32, _vp]),
    "bs_probe_random_reads": (_i32, [_vp, _u64, _vp, _u32, _vp]),
    "bs_probe_random_reads_region": (_i32, [_vp, _u64, _u32, _u64, _vp, _u32, _vp]),
    "bs_probe_round_trips": (_i32, [_vp, _u32, _u32, _vp]),
    "bs_probe_int_rate": (_i32, [_u32, _u32, _vp, _u32, _vp]),
    "bs_probe_cipher_scan": (_i32, [_u64, _u64, _u32, _vp, _sz, _vp]),
    "bs_probe_set_store_mode": (_i32, [_u32]),
    "bs_probe_set_xcd_mode": (_i32, [_u32]),
    "bs_probe_set_batch_small": (_i32, [_u32]),
    "bs_probe_set_watchdog": (_i32, [_u32, _u32]),
}


def lib() -> ctypes.CDLL:
    """Loads libbshuffle.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -m paper_2106_06161_amd.build or __graft_entry__.build())"
            )
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _lib = l
        # launch shapes picked by the autotuner (speed only; results never depend on them)
        if os.path.exists(TUNED_FILE):
            l.bs_load_tuned_configs(TUNED_FILE.encode())
    return _lib


def declared_functions() -> list[str]:
    """Names of every function declared in include/*.h."""
    names = []
    for h in HEADERS:
        with open(h) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(bs_\w+)\s*\(", text)
    return sorted(set(names))


def status_string(status: int) -> str:
    return lib().bs_status_string(status).decode()


def _check(status: int, where: str) -> None:
    if status != BS_OK:
        raise BShuffleError(status, where)


# ------------------------------------------------------------- raw ABI --
def bs_domain_bits(n: int) -> int:
    return int(lib().bs_domain_bits(n))


def bs_round_keys(seed: int, rounds: int) -> list[int]:
    buf = (ctypes.c_uint32 * max(rounds, 1))()
    _check(lib().bs_round_keys(seed & (2**64 - 1), rounds, buf), "bs_round_keys")
    return list(buf)[:rounds]


def bs_workspace_bytes(items: int, num_segments: int = 0, elem_bytes: int = 4) -> int:
    return int(lib().bs_workspace_bytes(items, num_segments, elem_bytes))


def bs_shuffle(in_ptr, out_ptr, n, elem_bytes, seed, rounds, workspace, workspace_bytes, stream) -> int:
    return int(lib().bs_shuffle(in_ptr, out_ptr, n, elem_bytes, seed & (2**64 - 1), rounds, workspace,
                                workspace_bytes, stream))


NOALLOC_MAX_ITEMS = 1 << 30


def bs_shuffle_noalloc(in_ptr, out_ptr, n, elem_bytes, seed, rounds, stream) -> int:
    return int(lib().bs_shuffle_noalloc(in_ptr, out_ptr, n, elem_bytes, seed & (2**64 - 1), rounds, stream))


def bs_shuffle_batched(in_ptr, out_ptr, offsets_ptr, seeds_ptr, num_segments, total_items, elem_bytes, rounds,
                       workspace, workspace_bytes, stream) -> int:
    return int(lib().bs_shuffle_batched(in_ptr, out_ptr, offsets_ptr, seeds_ptr, num_segments, total_items,
                                        elem_bytes, rounds, workspace, workspace_bytes, stream))


def bs_workspace_init(workspace, workspace_bytes, stream) -> int:
    return int(lib().bs_workspace_init(workspace, workspace_bytes, stream))


def bs_workspace_error(workspace, stream) -> int:
    return int(lib().bs_workspace_error(workspace, stream))


GRID_ONE_PER_TILE = 1000
DEPTH_COMPACT = 8  # tile schedule: kept images compacted through LDS
DEPTH_COMPACT_PIPE = 9  # same, with the next tile's cipher overlapping the current tile's gathers
DEPTH_STAGED = 16  # bs_query_config: bs_shuffle takes the staged form (streaming passes)


def bs_set_config(waves: int, items: int, depth: int, grid_mult: int) -> int:
    return int(lib().bs_set_config(waves, items, depth, grid_mult))


def bs_get_config() -> tuple[int, int, int, int]:
    w, i, d, g = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().bs_get_config(ctypes.byref(w), ctypes.byref(i), ctypes.byref(d), ctypes.byref(g)), "bs_get_config")
    return w.value, i.value, d.value, g.value


def bs_set_tuned_config(kind: int, elem_bytes: int, size_bits: int, waves: int, items: int, depth: int,
                        grid_mult: int) -> int:
    return int(lib().bs_set_tuned_config(kind, elem_bytes, size_bits, waves, items, depth, grid_mult))


def bs_query_config(kind: int, elem_bytes: int, items: int, num_segments: int = 0) -> tuple[int, int, int, int]:
    w, i, d, g = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().bs_query_config(kind, elem_bytes, items, num_segments, ctypes.byref(w), ctypes.byref(i),
                                 ctypes.byref(d), ctypes.byref(g)), "bs_query_config")
    return w.value, i.value, d.value, g.value


def bs_clear_tuned_configs() -> int:
    return int(lib().bs_clear_tuned_configs())


def bs_permutation(out_ptr, n, index_bytes, seed, rounds, workspace, workspace_bytes, stream) -> int:
    return int(lib().bs_permutation(out_ptr, n, index_bytes, seed & (2**64 - 1), rounds, workspace,
                                    workspace_bytes, stream))


def bs_unshuffle(in_ptr, out_ptr, n, elem_bytes, seed, rounds, workspace, workspace_bytes, stream) -> int:
    return int(lib().bs_unshuffle(in_ptr, out_ptr, n, elem_bytes, seed & (2**64 - 1), rounds, workspace,
                                  workspace_bytes, stream))


AUTOTUNE_VERBOSE = 1


def bs_autotune(device: int, cache_path: str | None, max_size_bits: int = 0, flags: int = 0) -> int:
    return int(lib().bs_autotune(device, cache_path.encode() if cache_path else None, max_size_bits, flags))


def bs_load_tuned_configs(path: str) -> int:
    return int(lib().bs_load_tuned_configs(path.encode()))


def bs_save_tuned_configs(path: str) -> int:
    return int(lib().bs_save_tuned_configs(path.encode()))


def bs_lcg_params(n: int, seed: int) -> tuple[int, int]:
    a, c = ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().bs_lcg_params(n, seed & (2**64 - 1), ctypes.byref(a), ctypes.byref(c)), "bs_lcg_params")
    return a.value, c.value


def bs_shuffle_lcg(in_ptr, out_ptr, n, elem_bytes, seed, workspace, workspace_bytes, stream) -> int:
    return int(lib().bs_shuffle_lcg(in_ptr, out_ptr, n, elem_bytes, seed & (2**64 - 1), workspace, workspace_bytes,
                                    stream))


def bs_bijection(in_ptr, out_ptr, count, domain_bits, seed, rounds, inverse, stream) -> int:
    return int(lib().bs_bijection(in_ptr, out_ptr, count, domain_bits, seed & (2**64 - 1), rounds, inverse, stream))


def bs_unshuffle_inverse_scratch_bytes(n) -> int:
    return int(lib().bs_unshuffle_inverse_scratch_bytes(n))


def bs_unshuffle_inverse(in_ptr, out_ptr, n, elem_bytes, seed, rounds, scratch, scratch_bytes, stream) -> int:
    return int(lib().bs_unshuffle_inverse(in_ptr, out_ptr, n, elem_bytes, seed & (2**64 - 1), rounds, scratch,
                                          scratch_bytes, stream))


def bs_probe_shuffle_two_pass(in_ptr, out_ptr, n, elem_bytes, seed, rounds, workspace, workspace_bytes,
                              stream) -> int:
    return int(lib().bs_probe_shuffle_two_pass(in_ptr, out_ptr, n, elem_bytes, seed & (2**64 - 1), rounds,
                                               workspace, workspace_bytes, stream))


def bs_probe_unfused_scratch_bytes(n: int) -> int:
    return int(lib().bs_probe_unfused_scratch_bytes(n))


def bs_probe_shuffle_unfused(in_ptr, out_ptr, n, elem_bytes, seed, rounds, scratch, scratch_bytes, workspace,
                             workspace_bytes, stream) -> int:
    return int(lib().bs_probe_shuffle_unfused(in_ptr, out_ptr, n, elem_bytes, seed & (2**64 - 1), rounds, scratch,
                                              scratch_bytes, workspace, workspace_bytes, stream))


def bs_probe_copy(in_ptr, out_ptr, nbytes, stream) -> int:
    return int(lib().bs_probe_copy(in_ptr, out_ptr, nbytes, stream))


def bs_probe_gather(in_ptr, n_in, out_ptr, idx_ptr, n, elem_bytes, stream) -> int:
    return int(lib().bs_probe_gather(in_ptr, n_in, out_ptr, idx_ptr, n, elem_bytes, stream))


def bs_probe_cipher_scan(n, seed, rounds, workspace, workspace_bytes, stream) -> int:
    return int(lib().bs_probe_cipher_scan(n, seed & (2**64 - 1), rounds, workspace, workspace_bytes, stream))


def bs_probe_set_watchdog(spin_limit: int, stall_first_tile: int) -> int:
    return int(lib().bs_probe_set_watchdog(spin_limit, stall_first_tile))


def bs_probe_random_reads(in_ptr, words, out_ptr, salt, stream) -> int:
    return int(lib().bs_probe_random_reads(in_ptr, words, out_ptr, salt, stream))


def bs_probe_random_reads_region(in_ptr, region_bytes, elem_bytes, reads, out_ptr, salt, stream) -> int:
    return int(lib().bs_probe_random_reads_region(in_ptr, region_bytes, elem_bytes, reads, out_ptr, salt, stream))


def bs_probe_set_batch_small(enable: int) -> int:
    return int(lib().bs_probe_set_batch_small(enable))


def bs_probe_set_xcd_mode(mode: int) -> int:
    return int(lib().bs_probe_set_xcd_mode(mode))


def bs_probe_set_store_mode(nontemporal: int) -> int:
    return int(lib().bs_probe_set_store_mode(nontemporal))


# ---------------------------------------------------- torch-level API --
def _records(x) -> tuple[int, int]:
    """(n, elem_bytes) of a tensor permuted along dim 0."""
    n = x.shape[0] if x.dim() else 1
    trailing = 1
    for d in x.shape[1:]:
        trailing *= d
    return n, x.element_size() * trailing


def _stream_ptr(x, stream) -> int:
    import torch

    if stream is None:
        stream = torch.cuda.current_stream(x.device)
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _require_device(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (the shuffle runs only in HIP kernels)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def workspace_bytes(items: int, num_segments: int = 0, elem_bytes: int = 4, staged: bool = False) -> int:
    """Workspace bytes for a call; staged=True (single shuffles): room for the
    staged form as well, which bs_shuffle then takes where the tuned table
    prefers it."""
    if staged and num_segments == 0:
        return bs_workspace_bytes_staged(items, elem_bytes)
    return bs_workspace_bytes(items, num_segments, elem_bytes)


def make_workspace(nbytes: int, device=None, stream=None):
    """Allocates and initialises a caller-owned workspace tensor."""
    import torch

    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device or "cuda")
    _check(bs_workspace_init(ws.data_ptr(), ws.numel(), _stream_ptr(ws, stream)), "bs_workspace_init")
    return ws


def shuffle(x, seed: int, rounds: int = DEFAULT_ROUNDS, out=None, workspace=None, stream=None):
    """Bijective shuffle of x along dim 0 (one record = x[i], raw bytes)."""
    import torch

    _require_device(x, "x")
    if out is None:
        out = torch.empty_like(x)
    _require_device(out, "out")
    if out.shape != x.shape or out.dtype != x.dtype or out.device != x.device:
        raise ValueError("out must match x in shape, dtype and device")
    n, eb = _records(x)
    ws_ptr, ws_bytes = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) if workspace is not None else (None, 0)
    with torch.cuda.device(x.device):
        st = bs_shuffle(x.data_ptr(), out.data_ptr(), n, eb, seed, rounds, ws_ptr, ws_bytes, _stream_ptr(x, stream))
    _check(st, "bs_shuffle")
    return out


def shuffle_batched(x, offsets, seeds, rounds: int = DEFAULT_ROUNDS, out=None, total_items=None, workspace=None,
                    stream=None):
    """Independent shuffles of the segments x[offsets[s]:offsets[s+1]] with seeds[s].

    offsets: int64 GPU tensor of S+1 entries; seeds: int64 (bit pattern of the
    uint64 seed) GPU tensor of S entries.  total_items defaults to x.shape[0]."""
    import torch

    _require_device(x, "x")
    _require_device(offsets, "offsets")
    _require_device(seeds, "seeds")
    if offsets.dtype != torch.int64 or seeds.dtype not in (torch.int64, torch.uint64):
        raise ValueError("offsets must be int64 and seeds int64/uint64")
    s = seeds.numel()
    if offsets.numel() != s + 1:
        raise ValueError("offsets needs num_segments + 1 entries")
    for t, name in ((offsets, "offsets"), (seeds, "seeds")):
        if t.device != x.device:
            raise ValueError(f"{name} must be on x's device ({x.device}), not {t.device}")
    if out is None:
        out = torch.empty_like(x)
    _require_device(out, "out")
    if out.shape != x.shape or out.dtype != x.dtype or out.device != x.device:
        raise ValueError("out must match x in shape, dtype and device")
    n, eb = _records(x)
    total = n if total_items is None else int(total_items)
    if total > n:
        raise ValueError("total_items exceeds x")
    ws_ptr, ws_bytes = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) if workspace is not None else (None, 0)
    with torch.cuda.device(x.device):
        st = bs_shuffle_batched(x.data_ptr(), out.data_ptr(), offsets.data_ptr(), seeds.data_ptr(), s, total, eb,
                                rounds, ws_ptr, ws_bytes, _stream_ptr(x, stream))
    _check(st, "bs_shuffle_batched")
    return out


def permutation(n: int, seed: int, rounds: int = DEFAULT_ROUNDS, index_dtype=None, device="cuda", out=None,
                workspace=None, stream=None):
    """The shuffle's gather map: out[j] = input position of output j (int32 or int64)."""
    import torch

    index_dtype = index_dtype or (torch.int32 if n <= (1 << 31) else torch.int64)
    if out is None:
        out = torch.empty(n, dtype=index_dtype, device=device)
    _require_device(out, "out")
    ws_ptr, ws_bytes = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) if workspace is not None else (None, 0)
    with torch.cuda.device(out.device):
        st = bs_permutation(out.data_ptr(), n, out.element_size(), seed, rounds, ws_ptr, ws_bytes,
                            _stream_ptr(out, stream))
    _check(st, "bs_permutation")
    return out


def unshuffle(y, seed: int, rounds: int = DEFAULT_ROUNDS, out=None, workspace=None, stream=None):
    """Inverse of shuffle(x, seed, rounds) along dim 0."""
    import torch

    _require_device(y, "y")
    if out is None:
        out = torch.empty_like(y)
    _require_device(out, "out")
    n, eb = _records(y)
    ws_ptr, ws_bytes = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) if workspace is not None else (None, 0)
    with torch.cuda.device(y.device):
        st = bs_unshuffle(y.data_ptr(), out.data_ptr(), n, eb, seed, rounds, ws_ptr, ws_bytes, _stream_ptr(y, stream))
    _check(st, "bs_unshuffle")
    return out


def unshuffle_inverse(y, seed: int, rounds: int = DEFAULT_ROUNDS, out=None, scratch=None, stream=None):
    """Inverse of shuffle(x, seed, rounds) along dim 0, in gather form through f^-1."""
    import torch

    _require_device(y, "y")
    if out is None:
        out = torch.empty_like(y)
    _require_device(out, "out")
    n, eb = _records(y)
    need = bs_unshuffle_inverse_scratch_bytes(n)
    if scratch is None:
        scratch = torch.empty(max(need, 1), dtype=torch.uint8, device=y.device)
    _require_device(scratch, "scratch")
    with torch.cuda.device(y.device):
        st = bs_unshuffle_inverse(y.data_ptr(), out.data_ptr(), n, eb, seed, rounds, scratch.data_ptr(),
                                  scratch.numel() * scratch.element_size(), _stream_ptr(y, stream))
    _check(st, "bs_unshuffle_inverse")
    return out


def shuffle_lcg(x, seed: int, out=None, workspace=None, stream=None):
    """Shuffle of x along dim 0 with the LCG bijection (Sec. 3.1) in place of VariablePhilox."""
    import torch

    _require_device(x, "x")
    if out is None:
        out = torch.empty_like(x)
    _require_device(out, "out")
    if out.shape != x.shape or out.dtype != x.dtype:
        raise ValueError("out must match x in shape and dtype")
    n, eb = _records(x)
    ws_ptr, ws_bytes = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) if workspace is not None else (None, 0)
    with torch.cuda.device(x.device):
        st = bs_shuffle_lcg(x.data_ptr(), out.data_ptr(), n, eb, seed, ws_ptr, ws_bytes, _stream_ptr(x, stream))
    _check(st, "bs_shuffle_lcg")
    return out


def bijection(x, domain_bits: int, seed: int, rounds: int = DEFAULT_ROUNDS, inverse: bool = False, out=None,
              stream=None):
    """f(x) (or f^-1(x)) elementwise for a device int64/uint64 tensor of values in [0, 2^domain_bits)."""
    import torch

    _require_device(x, "x")
    if x.dtype not in (torch.int64, torch.uint64) or not x.is_contiguous():
        raise ValueError("x must be a contiguous int64 or uint64 tensor")
    if out is None:
        out = torch.empty_like(x)
    _require_device(out, "out")
    if out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous():
        raise ValueError("out must match x in shape and dtype")
    with torch.cuda.device(x.device):
        st = bs_bijection(x.data_ptr(), out.data_ptr(), x.numel(), domain_bits, seed, rounds, int(inverse),
                          _stream_ptr(x, stream))
    _check(st, "bs_bijection")
    return out


def workspace_error(workspace=None, stream=None, device=None) -> int:
    """Drains the stream and returns (and clears) the workspace's device-side error status."""
    import torch

    dev = workspace.device if workspace is not None else torch.device(device or "cuda")
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    with torch.cuda.device(dev):
        return bs_workspace_error(workspace.data_ptr() if workspace is not None else None, sp)


def workspace_error_async(workspace, status, stream=None) -> None:
    """Enqueues on the stream a read-and-clear of the workspace's error word
    into status[0] (a 4-byte int32 tensor on the device or in pinned host
    memory); status[0] holds BS_OK / BS_ETIMEOUT / BS_EDEVICE once the stream
    has passed this point."""
    import torch

    if status.dtype != torch.int32 or status.numel() < 1:
        raise ValueError("status must be an int32 tensor with at least one element")
    if not (status.is_cuda or status.is_pinned()):
        raise ValueError("status must be device memory or pinned host memory")
    sp = _stream_ptr(workspace, stream)
    with torch.cuda.device(workspace.device):
        _check(lib().bs_workspace_error_async(workspace.data_ptr(), status.data_ptr(), sp),
               "bs_workspace_error_async")


def bs_staged_scratch_bytes(n: int, elem_bytes: int) -> int:
    return int(lib().bs_staged_scratch_bytes(n, elem_bytes))


def bs_shuffle_staged(in_ptr, out_ptr, n, elem_bytes, seed, rounds, scratch, scratch_bytes, stream) -> int:
    return int(lib().bs_shuffle_staged(in_ptr, out_ptr, n, elem_bytes, seed & (2**64 - 1), rounds, scratch,
                                       scratch_bytes, stream))


def staged_scratch_bytes(n: int, elem_bytes: int) -> int:
    """Scratch bytes bs_shuffle_staged needs (0: the staged form does not cover this size)."""
    return bs_staged_scratch_bytes(n, elem_bytes)


def shuffle_staged(x, seed: int, rounds: int = DEFAULT_ROUNDS, out=None, scratch=None, stream=None):
    """bs_shuffle's result through the staged (streaming) passes; scratch is a
    uint8 GPU tensor of at least staged_scratch_bytes(n, elem_bytes) bytes
    (allocated here when None)."""
    import torch

    _require_device(x, "x")
    if out is None:
        out = torch.empty_like(x)
    _require_device(out, "out")
    if out.shape != x.shape or out.dtype != x.dtype or out.device != x.device:
        raise ValueError("out must match x in shape, dtype and device")
    n, eb = _records(x)
    if n == 0:
        return out
    need = bs_staged_scratch_bytes(n, eb)
    if need == 0:
        raise BShuffleError(BS_EINVAL, "bs_shuffle_staged: size outside the staged form")
    if scratch is None:
        scratch = torch.empty(need, dtype=torch.uint8, device=x.device)
    _require_device(scratch, "scratch")
    with torch.cuda.device(x.device):
        st = bs_shuffle_staged(x.data_ptr(), out.data_ptr(), n, eb, seed, rounds, scratch.data_ptr(),
                               scratch.numel() * scratch.element_size(), _stream_ptr(x, stream))
    _check(st, "bs_shuffle_staged")
    return out


def bs_unshuffle_staged_scratch_bytes(n: int, elem_bytes: int) -> int:
    return int(lib().bs_unshuffle_staged_scratch_bytes(n, elem_bytes))


def bs_unshuffle_staged(in_ptr, out_ptr, n, elem_bytes, seed, rounds, scratch, scratch_bytes, stream) -> int:
    return int(lib().bs_unshuffle_staged(in_ptr, out_ptr, n, elem_bytes, seed & (2**64 - 1), rounds, scratch,
                                         scratch_bytes, stream))


def unshuffle_staged_scratch_bytes(n: int, elem_bytes: int) -> int:
    """Scratch bytes bs_unshuffle_staged needs (0: the staged form does not cover this size)."""
    return bs_unshuffle_staged_scratch_bytes(n, elem_bytes)


def unshuffle_staged(y, seed: int, rounds: int = DEFAULT_ROUNDS, out=None, scratch=None, stream=None):
    """bs_unshuffle's result (the inverse of shuffle with the same seed and
    rounds) through the staged passes; scratch is a uint8 GPU tensor of at
    least unshuffle_staged_scratch_bytes(n, elem_bytes) bytes (allocated here
    when None)."""
    import torch

    _require_device(y, "y")
    if out is None:
        out = torch.empty_like(y)
    _require_device(out, "out")
    if out.shape != y.shape or out.dtype != y.dtype or out.device != y.device:
        raise ValueError("out must match y in shape, dtype and device")
    n, eb = _records(y)
    if n == 0:
        return out
    need = bs_unshuffle_staged_scratch_bytes(n, eb)
    if need == 0:
        raise BShuffleError(BS_EINVAL, "bs_unshuffle_staged: size outside the staged form")
    if scratch is None:
        scratch = torch.empty(need, dtype=torch.uint8, device=y.device)
    _require_device(scratch, "scratch")
    with torch.cuda.device(y.device):
        st = bs_unshuffle_staged(y.data_ptr(), out.data_ptr(), n, eb, seed, rounds, scratch.data_ptr(),
                                 scratch.numel() * scratch.element_size(), _stream_ptr(y, stream))
    _check(st, "bs_unshuffle_staged")
    return out


def bs_workspace_bytes_staged(n: int, elem_bytes: int) -> int:
    return int(lib().bs_workspace_bytes_staged(n, elem_bytes))


def bs_probe_set_staged_policy(mode: int) -> int:
    return int(lib().bs_probe_set_staged_policy(mode))


def bs_probe_round_trips(words_ptr, groups, chain, stream) -> int:
    return int(lib().bs_probe_round_trips(words_ptr, groups, chain, stream))


def bs_probe_int_rate(op, iters, out_ptr, groups, stream) -> int:
    return int(lib().bs_probe_int_rate(op, iters, out_ptr, groups, stream))
