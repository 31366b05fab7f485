"""Pins for the oracle's keyed bijection (VariablePhilox, Sec. 3.2).

Nothing here re-types the oracle's formulas.  Each test checks a fact fixed
by the paper's description or by mathematics: the cipher is a bijection, the
paper's inversion steps undo it, the round has the stated Feistel structure,
rounds compose, zero rounds is the identity, permutations of a power-of-two
domain are even, and domains below 2^4 collapse to a handful of
permutations.  The key schedule is pinned to SplitMix64's published output.
"""
import numpy as np
import pytest

import oracle


# --------------------------------------------------------------- keys ----
def test_splitmix64_published_outputs():
    # The first three outputs of SplitMix64 from state 0, as printed with the
    # generator's reference implementation (Steele, Lea, Flood 2014; Vigna).
    assert oracle.splitmix64(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_round_keys_are_low_words_of_the_stream():
    stream = oracle.splitmix64(12345, 8)
    assert list(oracle.round_keys(12345, 8)) == [v & 0xFFFFFFFF for v in stream]


def test_round_keys_prefix_stable():
    # More rounds only append keys (the r-th key does not depend on R).
    assert list(oracle.round_keys(9, 24)[:4]) == list(oracle.round_keys(9, 4))


# ------------------------------------------------------------- domain ----
@pytest.mark.parametrize(
    "n,k",
    [(0, 4), (1, 4), (2, 4), (5, 4), (8, 4), (16, 4), (17, 5), (100, 7), (100_000, 17),
     (1 << 27, 27), ((1 << 27) + 1, 28), (10**9, 30), (250_000_000, 28)],
)
def test_domain_bits(n, k):
    # Pad to the next power of two (Sec. 4), never below 2^4.
    assert oracle.domain_bits(n) == k


# -------------------------------------------------------- bijectivity ----
@pytest.mark.parametrize("k", list(range(4, 21)))
@pytest.mark.parametrize("rounds", [0, 1, 2, 3, 4, 24])
def test_bijective_exhaustive(k, rounds):
    for seed in (0, 1, 0xDEADBEEFCAFEF00D):
        t = oracle.Cipher(k, seed, rounds).table()
        assert np.unique(t).size == (1 << k)
        assert int(t.max()) == (1 << k) - 1


@pytest.mark.parametrize("k", [23, 24])
def test_bijective_exhaustive_large(k):
    t = oracle.Cipher(k, 7, 24).table()
    seen = np.zeros(1 << k, dtype=np.bool_)
    seen[t] = True
    assert seen.all()


# --------------------------------------------------------- inverse ----
@pytest.mark.parametrize("k", [4, 5, 9, 10, 13, 16, 17])
def test_inverse_undoes_cipher_exhaustive(k):
    # The paper's inversion steps G^-1, B^-1, R = F(L) xor L' recover x.
    c = oracle.Cipher(k, 2024 + k, 24)
    t = c.table()
    xs = np.arange(1 << k)
    for x in xs[:: max(1, (1 << k) // 4096)]:
        assert c.decrypt(int(t[x])) == int(x)


@pytest.mark.parametrize("k", [28, 29, 30, 31, 38, 40])
def test_inverse_undoes_cipher_sampled(k):
    rng = np.random.default_rng(k)
    c = oracle.Cipher(k, 99, 24)
    for x in rng.integers(0, 1 << k, size=2000, dtype=np.uint64):
        y = c.encrypt(int(x))
        assert 0 <= y < (1 << k)
        assert c.decrypt(y) == int(x)


# ------------------------------------------------- Feistel structure ----
def _split(x, k):
    w, odd = k // 2, k & 1
    return x >> (w + odd), (x >> w) & 1 if odd else 0, x & ((1 << w) - 1)


@pytest.mark.parametrize("k", [8, 9, 16, 17])
def test_one_round_structure(k):
    """One round is L' = F(L) xor R and (R', b') = G(B(L), b) (Sec. 3.2)."""
    w, odd = k // 2, k & 1
    c = oracle.Cipher(k, 31337, 1)
    rng = np.random.default_rng(k)
    for x in rng.integers(0, 1 << k, size=300):
        x = int(x)
        L, b, R = _split(x, k)
        y = c.encrypt(x)
        Ly, by, Ry = _split(y, k)
        # Changing R by d changes only L', and by exactly d.
        d = int(rng.integers(1, 1 << w))
        L2, b2, R2 = _split(c.encrypt(x ^ d), k)
        assert (L2 ^ Ly, b2, R2) == (d, by, Ry)
        if odd:
            # b is inserted below B(L): flipping it flips only the low bit of R'.
            L3, b3, R3 = _split(c.encrypt(x ^ (1 << w)), k)
            assert (L3, b3, R3 ^ Ry) == (Ly, by, 1)
    # For fixed (b, R), L -> (R', b') is a bijection (B is one, G is one).
    outs = {(_split(c.encrypt((L << (w + odd))), k)[1:]) for L in range(1 << w)}
    assert len(outs) == (1 << w)


@pytest.mark.parametrize("k", [10, 11])
def test_rounds_compose(k):
    """g = f_r o ... o f_1: the cipher with R+1 rounds is one more round, keyed
    with the (R+1)-th key, applied to the R-round output (Sec. 3.2)."""
    seed = 777
    full = oracle.Cipher(k, seed, 24)
    head = oracle.Cipher(k, seed, 23)
    last = oracle.Cipher(k, 0, 1)
    last._c.key[0] = full.keys[23]
    for x in range(0, 1 << k, 7):
        assert full.encrypt(x) == last.encrypt(head.encrypt(x))


def test_only_low_key_bits_matter():
    # Only the half-width low bits of a round key reach the state.
    k = 12
    a = oracle.Cipher(k, 5, 3)
    b = oracle.Cipher(k, 5, 3)
    for r in range(3):
        b._c.key[r] ^= 0xFFFFFFFF ^ ((1 << (k // 2)) - 1)
    assert all(a.encrypt(x) == b.encrypt(x) for x in range(1 << k))


def test_zero_rounds_is_identity():
    for k in (4, 7, 20):
        t = oracle.Cipher(k, 1, 0).table()
        assert np.array_equal(t, np.arange(1 << k, dtype=np.uint32))


def test_seeds_give_different_permutations():
    tabs = {oracle.Cipher(12, s, 24).table().tobytes() for s in range(50)}
    assert len(tabs) == 50


# ------------------------------------------------ derived invariants ----
def _parity(p):
    p = list(p)
    seen = [False] * len(p)
    swaps = 0
    for i in range(len(p)):
        if not seen[i]:
            j, length = i, 0
            while not seen[j]:
                seen[j] = True
                j = p[j]
                length += 1
            swaps += length - 1
    return swaps & 1


@pytest.mark.parametrize("k", [4, 5, 6, 7])
@pytest.mark.parametrize("rounds", [1, 23, 24])
def test_power_of_two_domain_permutations_are_even(k, rounds):
    """Every round is a composition of even permutations when the half width
    is >= 2 (a key-dependent xor on R, B applied for every R, the half swap),
    so the cipher on a full 2^k domain never reaches an odd permutation."""
    for seed in range(40):
        assert _parity(oracle.Cipher(k, seed, rounds).table()) == 0


@pytest.mark.parametrize("k,bound", [(1, 2), (2, 4), (3, 8)])
def test_below_four_bits_the_family_is_tiny(k, bound):
    """With a half width of at most one bit every round is affine over GF(2)
    and the key only translates, so at most 2^k permutations appear for any
    round count.  This is why the domain never goes below 2^4."""
    for rounds in (4, 24):
        tabs = {oracle.Cipher(k, s, rounds).table().tobytes() for s in range(2000)}
        assert len(tabs) <= bound
    tabs4 = {oracle.Cipher(4, s, 24).table().tobytes() for s in range(2000)}
    assert len(tabs4) > 1000


@pytest.mark.parametrize("k", [8, 9, 16, 17, 24, 25, 33])
@pytest.mark.parametrize("rounds", [1, 2, 24])
def test_round_key_enters_only_the_new_left_half(k, rounds):
    """Where the key enters a round (reading C4).  The text calls both F_k and
    B_k key-dependent; the listing keys only the round function: the key is
    xored into F's output, which lands in L', and B(L) carries no key.  So in
    the last round, changing that round's key by d (d below the half width)
    changes L' by exactly d and leaves R' and b' alone.  A key folded into B,
    or into R', or combined with F by addition, fails this."""
    w = k // 2
    rng = np.random.default_rng(1000 * k + rounds)
    base = oracle.Cipher(k, 4242 + k, rounds)
    xs = [int(v) for v in rng.integers(0, 1 << k, size=64, dtype=np.uint64)]
    ys = [base.encrypt(x) for x in xs]
    for d in [1, (1 << w) - 1] + [int(v) for v in rng.integers(1, 1 << w, size=6)]:
        alt = oracle.Cipher(k, 4242 + k, rounds)
        alt._c.key[rounds - 1] ^= d
        for x, y in zip(xs, ys):
            Ly, by, Ry = _split(y, k)
            La, ba, Ra = _split(alt.encrypt(x), k)
            assert (La ^ Ly, ba, Ra) == (d, by, Ry), (k, rounds, d, x)
