"""Sequential CPU oracle for the bijective shuffle (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does; the
oracle and the HIP path share no code.  The arithmetic lives in
``vphilox_oracle.c`` (plain C, built with gcc); this module only marshals
numpy arrays through ctypes.  Statistics (chi-square, Mallows MMD) are in
``oracle.stats``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vphilox_oracle.c")
# ORACLE_SANITIZE=1 builds and loads a copy instrumented with AddressSanitizer
# and UndefinedBehaviorSanitizer (any report aborts); the process must preload
# the ASan runtime (LD_PRELOAD=$(gcc -print-file-name=libasan.so)).
SANITIZE = os.environ.get("ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "liboracle_san.so" if SANITIZE else "liboracle.so")
_SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=all"]
_STD_SRC = os.path.join(_HERE, "std_shuffle.cpp")
_STD_LIB = os.path.join(_HERE, "libstdshuffle.so")

MAX_ROUNDS = 64
MIN_DOMAIN_BITS = 4
MAX_DOMAIN_BITS = 40
M0 = 0xD2B74407B1CE6E93


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        opt = _SAN_FLAGS if SANITIZE else ["-O2"]
        subprocess.check_call(
            ["gcc", *opt, "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB)
    if force or not os.path.exists(_STD_LIB) or os.path.getmtime(_STD_LIB) < os.path.getmtime(_STD_SRC):
        tmp = _STD_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", _STD_SRC, "-o", tmp])
        os.replace(tmp, _STD_LIB)
    return _LIB


class _Cipher(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_uint32),
        ("w", ctypes.c_uint32),
        ("odd", ctypes.c_uint32),
        ("rounds", ctypes.c_uint32),
        ("key", ctypes.c_uint32 * MAX_ROUNDS),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        u32, u64, i64, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p
        cp = ctypes.POINTER(_Cipher)
        lib.orc_splitmix64_next.argtypes = [ctypes.POINTER(u64)]
        lib.orc_splitmix64_next.restype = u64
        lib.orc_round_keys.argtypes = [u64, u32, vp]
        lib.orc_round_keys.restype = None
        lib.orc_domain_bits.argtypes = [u64]
        lib.orc_domain_bits.restype = u32
        lib.orc_cipher_init.argtypes = [cp, u32, u64, u32]
        lib.orc_cipher_init.restype = ctypes.c_int
        lib.orc_encrypt.argtypes = [cp, u64]
        lib.orc_encrypt.restype = u64
        lib.orc_decrypt.argtypes = [cp, u64]
        lib.orc_decrypt.restype = u64
        lib.orc_encrypt_all.argtypes = [cp, vp]
        lib.orc_encrypt_all.restype = ctypes.c_int
        lib.orc_shuffle.argtypes = [vp, vp, u64, u32, u64, u32]
        lib.orc_shuffle.restype = i64
        lib.orc_shuffle_sources.argtypes = [u64, u64, u32, vp]
        lib.orc_shuffle_sources.restype = i64
        lib.orc_count_kept.argtypes = [u64, u64, u32, u64, u64]
        lib.orc_count_kept.restype = i64
        lib.orc_shuffle_window.argtypes = [vp, u64, u32, u64, u32, u64, u64, vp]
        lib.orc_shuffle_window.restype = i64
        lib.orc_shuffle_batched.argtypes = [vp, vp, vp, vp, u32, u32, u32]
        lib.orc_shuffle_batched.restype = ctypes.c_int
        lib.orc_discordant_pairs_brute.argtypes = [vp, vp, u32]
        lib.orc_discordant_pairs_brute.restype = u64
        lib.orc_discordant_pairs.argtypes = [vp, vp, u32]
        lib.orc_discordant_pairs.restype = i64
        lib.orc_pair_discordances.argtypes = [vp, u64, u32, vp]
        lib.orc_pair_discordances.restype = ctypes.c_int
        lib.orc_lcg_params.argtypes = [u64, u64, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        lib.orc_lcg_params.restype = None
        lib.orc_lcg_shuffle.argtypes = [vp, vp, u64, u32, u64]
        lib.orc_lcg_shuffle.restype = i64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _as_bytes(x: np.ndarray) -> tuple[np.ndarray, int]:
    """View an (n, ...) array as n records of elem_bytes bytes."""
    x = np.ascontiguousarray(x)
    n = x.shape[0] if x.ndim else 1
    eb = x.itemsize * (int(np.prod(x.shape[1:])) if x.ndim > 1 else 1)
    return x, eb if n else x.itemsize


# ----------------------------------------------------------------- keys --
def splitmix64(seed: int, count: int) -> list[int]:
    st = ctypes.c_uint64(seed & (2**64 - 1))
    lib = _load()
    return [int(lib.orc_splitmix64_next(ctypes.byref(st))) for _ in range(count)]


def round_keys(seed: int, rounds: int) -> np.ndarray:
    keys = np.zeros(max(rounds, 1), dtype=np.uint32)
    _load().orc_round_keys(seed & (2**64 - 1), rounds, _ptr(keys))
    return keys[:rounds]


def domain_bits(n: int) -> int:
    return int(_load().orc_domain_bits(n))


# --------------------------------------------------------------- cipher --
class Cipher:
    """VariablePhilox on [0, 2^k) with the given seed and round count."""

    def __init__(self, k: int, seed: int, rounds: int):
        self._c = _Cipher()
        rc = _load().orc_cipher_init(ctypes.byref(self._c), k, seed & (2**64 - 1), rounds)
        if rc != 0:
            raise ValueError(f"bad cipher parameters k={k} rounds={rounds}")
        self.k, self.rounds = k, rounds

    @property
    def keys(self) -> list[int]:
        return list(self._c.key[: self.rounds])

    def encrypt(self, x: int) -> int:
        return int(_load().orc_encrypt(ctypes.byref(self._c), x))

    def decrypt(self, y: int) -> int:
        return int(_load().orc_decrypt(ctypes.byref(self._c), y))

    def table(self) -> np.ndarray:
        """f(x) for every x in the domain (k <= 32)."""
        t = np.empty(1 << self.k, dtype=np.uint32)
        if _load().orc_encrypt_all(ctypes.byref(self._c), _ptr(t)) != 0:
            raise ValueError("domain too large for a table")
        return t


# -------------------------------------------------------------- shuffle --
def shuffle(x: np.ndarray, seed: int, rounds: int = 24) -> np.ndarray:
    """Algorithm 1 along axis 0: out[rank(i)] = x[f(i)]."""
    x, eb = _as_bytes(x)
    out = np.empty_like(x)
    n = x.shape[0]
    got = _load().orc_shuffle(_ptr(x), _ptr(out), n, eb, seed & (2**64 - 1), rounds)
    if got != n:
        raise ValueError(f"oracle shuffle failed ({got})")
    return out


def shuffle_sources(n: int, seed: int, rounds: int = 24) -> np.ndarray:
    """perm[j] = index of the input element that lands at output j."""
    perm = np.empty(max(n, 1), dtype=np.uint64)
    got = _load().orc_shuffle_sources(n, seed & (2**64 - 1), rounds, _ptr(perm))
    if got != n:
        raise ValueError(f"oracle failed ({got})")
    return perm[:n]


def count_kept(n: int, seed: int, rounds: int, i_begin: int, i_end: int) -> int:
    got = _load().orc_count_kept(n, seed & (2**64 - 1), rounds, i_begin, i_end)
    if got < 0:
        raise ValueError("bad arguments")
    return int(got)


def shuffle_window(x: np.ndarray, seed: int, rounds: int, i_begin: int, i_end: int) -> np.ndarray:
    """Outputs produced by the padded indices in [i_begin, i_end), in order."""
    x, eb = _as_bytes(x)
    n = x.shape[0]
    k = domain_bits(n)
    i_end = min(i_end, 1 << k)
    cap = max(i_end - i_begin, 1)
    win = np.empty((cap,) + x.shape[1:], dtype=x.dtype)
    got = _load().orc_shuffle_window(
        _ptr(x), n, eb, seed & (2**64 - 1), rounds, i_begin, i_end, _ptr(win)
    )
    if got < 0:
        raise ValueError("bad arguments")
    return win[:got]


def shuffle_batched(x: np.ndarray, offsets: np.ndarray, seeds: np.ndarray, rounds: int = 24) -> np.ndarray:
    x, eb = _as_bytes(x)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
    out = np.empty_like(x)
    s = len(seeds)
    assert len(offsets) == s + 1
    rc = _load().orc_shuffle_batched(_ptr(x), _ptr(out), _ptr(offsets), _ptr(seeds), s, eb, rounds)
    if rc != 0:
        raise ValueError("oracle batched shuffle failed")
    return out


def permutations(n: int, seeds, rounds: int) -> np.ndarray:
    """Row p is the shuffle of arange(n) with seeds[p] (one-line notation)."""
    seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
    p = len(seeds)
    x = np.tile(np.arange(n, dtype=np.uint32), p)
    offsets = np.arange(p + 1, dtype=np.int64) * n
    return shuffle_batched(x, offsets, seeds, rounds).reshape(p, n)


def lcg_params(n: int, seed: int) -> tuple[int, int]:
    a, c = ctypes.c_uint64(), ctypes.c_uint64()
    _load().orc_lcg_params(n, seed & (2**64 - 1), ctypes.byref(a), ctypes.byref(c))
    return a.value, c.value


def lcg_shuffle(x: np.ndarray, seed: int) -> np.ndarray:
    """Algorithm 1 with the LCG bijection y = (a*i + c) mod 2^k (Sec. 3.1)."""
    x, eb = _as_bytes(x)
    out = np.empty_like(x)
    n = x.shape[0]
    got = _load().orc_lcg_shuffle(_ptr(x), _ptr(out), n, eb, seed & (2**64 - 1))
    if got != n:
        raise ValueError(f"oracle LCG shuffle failed ({got})")
    return out


def lcg_permutations(n: int, seeds) -> np.ndarray:
    return np.stack([lcg_shuffle(np.arange(n, dtype=np.uint32), int(s)) for s in seeds])


# ------------------------------------------------------ Mallows helpers --
def discordant_pairs(a: np.ndarray, b: np.ndarray, brute: bool = False) -> int:
    a = np.ascontiguousarray(a, dtype=np.uint32)
    b = np.ascontiguousarray(b, dtype=np.uint32)
    lib = _load()
    if brute:
        return int(lib.orc_discordant_pairs_brute(_ptr(a), _ptr(b), len(a)))
    d = lib.orc_discordant_pairs(_ptr(a), _ptr(b), len(a))
    if d < 0:
        raise ValueError("a must be a permutation of 0..n-1")
    return int(d)


def pair_discordances(perms: np.ndarray) -> np.ndarray:
    """n_dis of rows (2i, 2i+1) for each i."""
    perms = np.ascontiguousarray(perms, dtype=np.uint32)
    p, n = perms.shape
    out = np.empty(max(p // 2, 1), dtype=np.uint64)
    if _load().orc_pair_discordances(_ptr(perms), p, n, _ptr(out)) != 0:
        raise ValueError("rows must be permutations")
    return out[: p // 2]


# ------------------------------------------------------- CPU timing reference --
def std_shuffle_u32(x: np.ndarray, seed: int) -> np.ndarray:
    """std::shuffle with std::mt19937_64(seed) on a copy of x (uint32), single thread.
    A timing reference for the benchmark, not a reference for the method."""
    build()
    lib = ctypes.CDLL(_STD_LIB)
    lib.cpu_std_shuffle_u32.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64]
    lib.cpu_std_shuffle_u32.restype = None
    y = np.array(x, dtype=np.uint32, copy=True)
    lib.cpu_std_shuffle_u32(_ptr(y), len(y), seed & (2**64 - 1))
    return y


def std_permutations(n: int, count: int, first_seed: int = 1) -> np.ndarray:
    """Row p is arange(n) shuffled by std::shuffle with std::mt19937_64(first_seed + p):
    the control generator of the statistical tests (Sec. 5 compares against it)."""
    build()
    lib = ctypes.CDLL(_STD_LIB)
    lib.cpu_std_permutations_u32.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    lib.cpu_std_permutations_u32.restype = None
    out = np.empty((count, n), dtype=np.uint32)
    lib.cpu_std_permutations_u32(_ptr(out), n, count, first_seed & (2**64 - 1))
    return out
