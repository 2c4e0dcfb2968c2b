"""Pins of the oracle for the paper's own secEval (one-hot RSS attributes,
replicated FSS keys, Eq. predEval): the XOR of the three servers' shares is
the plaintext predicate for every attribute value, and no single server's
share is."""
import numpy as np
import pytest

import synth
from oracle import rss


@pytest.mark.parametrize("npos", [16, 64, 200])
def test_equality_every_value(npos):
    values = np.arange(npos, dtype=np.uint32)
    shares = synth.onehot_rss(3, values, npos)
    np.testing.assert_array_equal(np.bitwise_xor.reduce(shares, axis=0).argmax(axis=1), values)
    for a in (0, npos // 3, npos - 1):
        keys, nb = rss.token("eq", npos, 11, 1, a, a=a)
        x = rss.server_shares("eq", npos, keys, nb, shares)
        np.testing.assert_array_equal(x[0] ^ x[1] ^ x[2], (values == a).astype(np.uint8))


@pytest.mark.parametrize("npos", [16, 64])
def test_range_every_value(npos):
    values = np.arange(npos, dtype=np.uint32)
    shares = synth.onehot_rss(4, values, npos)
    for lo, hi in ((0, npos - 1), (3, 9), (5, 5), (1, npos - 1)):
        keys, nb = rss.token("range", npos, 12, 1, lo, lo=lo, hi=hi)
        x = rss.server_shares("range", npos, keys, nb, shares)
        np.testing.assert_array_equal(x[0] ^ x[1] ^ x[2], ((values >= lo) & (values < hi)).astype(np.uint8))


def test_one_server_alone_is_not_the_predicate():
    npos = 64
    values = np.random.default_rng(1).integers(0, npos, 4000).astype(np.uint32)
    shares = synth.onehot_rss(5, values, npos)
    keys, nb = rss.token("eq", npos, 13, 1, 0, a=7)
    x = rss.server_shares("eq", npos, keys, nb, shares)
    truth = (values == 7).astype(np.uint8)
    for i in range(3):
        assert 0.4 < x[i].mean() < 0.6
        assert 0.4 < (x[i] ^ x[(i + 1) % 3]).mean() < 0.6     # two servers together learn nothing either
    np.testing.assert_array_equal(x[0] ^ x[1] ^ x[2], truth)


def test_word_major_packing():
    bits = np.zeros((3, 40), np.uint8)
    bits[1, 0] = bits[1, 33] = bits[2, 39] = 1
    w = synth.pack_word_major(bits)
    assert w.shape == (2, 3)
    assert w[0, 1] == 1 and w[1, 1] == 2 and w[1, 2] == 1 << 7 and w[0, 0] == 0
