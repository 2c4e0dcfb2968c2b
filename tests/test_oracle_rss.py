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


def _rand_words(seed, n):
    return np.random.default_rng(seed).integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)


def test_zero_shares_xor_to_zero_and_look_random():
    a = rss.zero_shares([11, 22, 33], 7, 64)
    assert not (a[0] ^ a[1] ^ a[2]).any()
    for i in range(3):
        bits = np.unpackbits(a[i].view(np.uint8))
        assert 0.4 < bits.mean() < 0.6


def test_rss_and_truth_table():
    """Every assignment of the three shares of x and y (packed 64 ways into
    words) reconstructs to x AND y."""
    n = 64 * 32
    rng = np.random.default_rng(3)
    for trial in range(4):
        x = [_rand_words(10 * trial + i, n // 32) for i in range(3)]
        y = [_rand_words(10 * trial + 5 + i, n // 32) for i in range(3)]
        z = rss.rss_and(x, y, [1, 2, 3 + trial], trial, n)
        np.testing.assert_array_equal(z[0] ^ z[1] ^ z[2], (x[0] ^ x[1] ^ x[2]) & (y[0] ^ y[1] ^ y[2]))
    # a dropped cross term is caught
    x = [_rand_words(100 + i, 8) for i in range(3)]
    y = [_rand_words(200 + i, 8) for i in range(3)]
    bad = [(x[i] & y[i]) ^ (x[i] & y[(i + 1) % 3]) for i in range(3)]
    assert ((bad[0] ^ bad[1] ^ bad[2]) != ((x[0] ^ x[1] ^ x[2]) & (y[0] ^ y[1] ^ y[2]))).any()


def test_reshare_keeps_the_value_and_clears_pad():
    x3 = [_rand_words(7 + i, 5) for i in range(3)]
    vm = rss.fss.valid_mask(150)
    z = rss.reshare(x3, [4, 5, 6], 1, 150)
    np.testing.assert_array_equal(z[0] ^ z[1] ^ z[2], (x3[0] ^ x3[1] ^ x3[2]) & vm)
    assert (z[0][-1] >> (150 % 32)) == 0


def test_sec_eval_then_rss_and_is_the_conjunction():
    """Two predicates by secEval, re-shared into RSS, ANDed: the reconstruction
    is the conjunction of the plaintext predicates (multi-predicate
    aggregation of Sec. V-D in the paper's own three-party form)."""
    npos = 64
    values = np.random.default_rng(8).integers(0, npos, 1000).astype(np.uint32)
    shares = synth.onehot_rss(21, values, npos)
    k1, nb = rss.token("range", npos, 5, 1, 0, lo=10, hi=40)
    k2, _ = rss.token("range", npos, 5, 1, 1, lo=30, hi=60)
    x1 = rss.server_shares("range", npos, k1, nb, shares)
    x2 = rss.server_shares("range", npos, k2, nb, shares)
    from oracle import fss as ofss
    p1 = rss.reshare([ofss.pack_bits(x1[i]) for i in range(3)], [7, 8, 9], 0, values.size)
    p2 = rss.reshare([ofss.pack_bits(x2[i]) for i in range(3)], [7, 8, 9], 1, values.size)
    z = rss.rss_and(p1, p2, [7, 8, 9], 2, values.size)
    got = ofss.unpack_bits(z[0] ^ z[1] ^ z[2], values.size)
    np.testing.assert_array_equal(got, ((values >= 30) & (values < 40)).astype(np.uint8))


def test_prf_words_follow_their_definition():
    """F(k, j), built batched, against one ChaCha12 block per word: word w is
    slice word w mod 16 (slice word 4c + k = state word 4k + c) of block
    (w div 16, j, 0, 0) under the key (k mod 2^32, k div 2^32, 5, 0, ...)."""
    from oracle import chacha
    k, j = 0xFEDC_BA98_7654_3210, 11
    got = rss.prf_words(k, j, 37)
    assert got.shape == (37,)
    for w in range(37):
        blk = chacha.blocks([0x76543210, 0xFEDCBA98, 5, 0, 0, 0, 0, 0], w // 16, j, 0, 0, 12)[0]
        s = w % 16
        assert int(got[w]) == int(blk[4 * (s % 4) + s // 4])


def test_prf_words_at_equals_the_stream():
    """The sampled accessor gives the stream's own words, in any order and
    with repeats, across block boundaries."""
    k, j = 0x0123_4567_89AB_CDEF, 4
    full = rss.prf_words(k, j, 1000)
    idx = np.array([999, 0, 15, 16, 17, 500, 15, 31, 32, 733])
    np.testing.assert_array_equal(rss.prf_words_at(k, j, idx), full[idx])


def test_two_party_fss_bits_to_rss_then_and():
    """The masked-input path's two-party predicate shares, converted to RSS
    and ANDed in RSS, reconstruct to the conjunction of the plaintext
    predicates; each converted share alone, and any two servers' shares
    together short of all three, look random (Sec. III-B re-share)."""
    from oracle import fss as ofss
    n, seed = 3000, 77
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 1 << 12, n).astype(np.uint32)
    r1 = ofss.masks(seed, 1, 0, n)
    r2 = ofss.masks(seed, 1, 1, n)
    xh1 = (x + r1).astype(np.uint32)
    xh2 = (x + r2).astype(np.uint32)
    k1 = ofss.keygen_range(32, seed, 1, 0, 100, 2500, r1)
    k2b = ofss.keygen_range(32, seed, 1, 1, 2000, 4000, r2)
    y1 = [ofss.pack_bits(ofss.eval_range(32, b, k1[b], xh1)) for b in range(2)]
    y2 = [ofss.pack_bits(ofss.eval_range(32, b, k2b[b], xh2)) for b in range(2)]
    keys = [91, 92, 93]
    p1 = rss.from_two_party(y1[0], y1[1], keys, 0, n)
    p2 = rss.from_two_party(y2[0], y2[1], keys, 1, n)
    want1 = ((x >= 100) & (x < 2500)).astype(np.uint8)
    want2 = ((x >= 2000) & (x < 4000)).astype(np.uint8)
    np.testing.assert_array_equal(ofss.unpack_bits(p1[0] ^ p1[1] ^ p1[2], n), want1)
    np.testing.assert_array_equal(ofss.unpack_bits(p2[0] ^ p2[1] ^ p2[2], n), want2)
    z = rss.rss_and(p1, p2, keys, 2, n)
    np.testing.assert_array_equal(ofss.unpack_bits(z[0] ^ z[1] ^ z[2], n), want1 & want2)
    for i in range(3):
        bits = ofss.unpack_bits(p1[i], n)
        assert 0.4 < bits.mean() < 0.6
        pair = ofss.unpack_bits(p1[i] ^ p1[(i + 1) % 3], n)
        assert 0.4 < pair.mean() < 0.6
    # a conversion that forgets the zero share of P_3 (z_3 = 0) is caught:
    # the third share would then be constant
    bad = [y1[0], y1[1], np.zeros_like(y1[0])]
    assert not ofss.unpack_bits(bad[2], n).any()
    assert ofss.unpack_bits(p1[2], n).any()
