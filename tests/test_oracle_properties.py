"""Property tests of the oracle (hypothesis): for any domain size, seed and
round count the cipher is a bijection that its inverse undoes, and the
shuffle of n items is the domain permutation with the images >= n deleted."""
import numpy as np
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle

seeds = st.integers(min_value=0, max_value=2**64 - 1)


@settings(max_examples=40, deadline=None)
@given(k=st.integers(min_value=1, max_value=14), seed=seeds, rounds=st.integers(min_value=0, max_value=40))
def test_cipher_is_a_bijection_undone_by_its_inverse(k, seed, rounds):
    c = oracle.Cipher(k, seed, rounds)
    table = c.table()
    assert np.array_equal(np.sort(table), np.arange(1 << k, dtype=table.dtype))
    xs = np.arange(1 << k, dtype=np.uint64)
    assert all(c.decrypt(int(c.encrypt(int(v)))) == int(v) for v in xs[:: max(1, len(xs) // 64)])


@settings(max_examples=40, deadline=None)
@given(n=st.integers(min_value=1, max_value=5000), seed=seeds, rounds=st.integers(min_value=0, max_value=32))
def test_shuffle_is_the_filtered_domain_permutation(n, seed, rounds):
    k = oracle.domain_bits(n)
    table = oracle.Cipher(k, seed, rounds).table()
    got = oracle.shuffle(np.arange(n, dtype=np.uint32), seed, rounds)
    assert np.array_equal(got.astype(table.dtype), table[table < n])
