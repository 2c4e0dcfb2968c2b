"""Pins of the shuffle / fetch oracle (Alg. 4, Alg. 5): the three output shares
reconstruct to the input table under the composition of the three
permutations (and so to a permutation of its rows), no output share equals
an input share, Case I returns the unique matching record, Case II returns
exactly the matching records."""
import numpy as np

from oracle import shuffle as osh


def _rss_table(seed, n, w):
    rng = np.random.default_rng(seed)
    d = rng.integers(0, 2**32, (n, w), dtype=np.uint64).astype(np.uint32)
    s1 = rng.integers(0, 2**32, (n, w), dtype=np.uint64).astype(np.uint32)
    s2 = rng.integers(0, 2**32, (n, w), dtype=np.uint64).astype(np.uint32)
    return d, [s1, s2, d ^ s1 ^ s2]


def test_shuffle_reconstructs_to_composed_permutation():
    for n, w in ((1, 1), (17, 3), (200, 5)):
        d, sh = _rss_table(n * w, n, w)
        r = osh.sec_shuffle(sh, 11, 22, 33)
        out = r[0] ^ r[1] ^ r[2]
        perm = osh.composed_permutation(11, 22, 33, n)
        np.testing.assert_array_equal(out, d[perm])
        assert sorted(map(tuple, out.tolist())) == sorted(map(tuple, d.tolist()))
        if n > 1:
            assert not np.array_equal(perm, np.arange(n))
            for i in range(3):
                assert not np.array_equal(r[i], sh[i])


def test_literal_x2_reading_fails():
    """Feeding CS2's second step anything but X1 breaks reconstruction: the
    printed X_2 must be the message X1."""
    n, w = 32, 2
    d, (d1, d2, d3) = _rss_table(5, n, w)
    p12, p23, p31 = (osh.permutation(s, p, n) for s, p in ((11, osh.P12), (22, osh.P23), (33, osh.P31)))
    t12, r2 = osh.mask_table(11, osh.T12, n, w), osh.mask_table(11, osh.R2, n, w)
    t23 = osh.mask_table(22, osh.T23, n, w)
    t31, r1 = osh.mask_table(33, osh.T31, n, w), osh.mask_table(33, osh.R1, n, w)
    y1 = osh.apply(p12, d3 ^ t12)
    wrong = np.zeros_like(d1)                       # no such message exists
    c1 = osh.apply(p23, wrong ^ t23) ^ r2
    c2 = osh.apply(p23, osh.apply(p31, y1 ^ t31) ^ t23) ^ r1
    assert not np.array_equal(r1 ^ r2 ^ c1 ^ c2, d[osh.composed_permutation(11, 22, 33, n)])


def test_fetch_case1_unique_match():
    n, w = 50, 4
    rng = np.random.default_rng(2)
    d, rows = _rss_table(9, n, w)
    x = np.zeros(n, np.uint8)
    x[31] = 1
    xs1 = rng.integers(0, 2, n, dtype=np.uint8)
    xs2 = rng.integers(0, 2, n, dtype=np.uint8)
    xsh = [xs1, xs2, x ^ xs1 ^ xs2]
    out = osh.fetch_case1(xsh, rows)
    np.testing.assert_array_equal(out[0] ^ out[1] ^ out[2], d[31])


def test_fetch_case2_all_matches():
    n, w = 120, 3
    rng = np.random.default_rng(4)
    d, rows = _rss_table(13, n, w)
    x = (rng.random(n) < 0.2).astype(np.uint8)
    xs1 = rng.integers(0, 2, n, dtype=np.uint8)
    xs2 = rng.integers(0, 2, n, dtype=np.uint8)
    keep, fetched = osh.fetch_case2([xs1, xs2, x ^ xs1 ^ xs2], rows, 7, 8, 9)
    got = fetched[0] ^ fetched[1] ^ fetched[2]
    assert keep.size == x.sum()
    assert sorted(map(tuple, got.tolist())) == sorted(map(tuple, d[x == 1].tolist()))


def test_batched_blocks_are_the_single_blocks():
    """The batched AES generator returns rng_block's blocks for consecutive
    counters."""
    from oracle import fss as ofss
    got = ofss.rng_blocks(77, 6, 4, 9, 0, 2**32 - 3, 6)
    for i in range(6):
        assert got[i].tobytes() == ofss.rng_block(77, 6, 4, 9, 0, (2**32 - 3 + i) % 2**32)


def test_tables_and_keys_follow_their_definitions():
    """Mask tables and sort keys, built batched, against one ChaCha12 block per
    word or row: word w of record r is slice word w mod 16 of block (r, w div
    16, table, W), slice word 4c + k being state word 4k + c; the key of row r
    is slice words 2e, 2e + 1 (e = r mod 8) of block (r div 8, 0, 16 + p, 0);
    the permutation sorts by (key, row)."""
    from oracle import chacha
    seed = 0x1234_5678_9ABC_DEF0
    key = [0x9ABCDEF0, 0x12345678, 6, 0, 0, 0, 0, 0]

    def slice_word(blk, s):
        return int(blk[4 * (s % 4) + s // 4])

    for n, w in ((7, 3), (3, 37)):
        t = osh.mask_table(seed, osh.T31, n, w)
        assert t.shape == (n, w)
        for r in range(n):
            for c in range(w):
                blk = chacha.blocks(key, r, c // 16, osh.T31, w, 12)[0]
                assert int(t[r, c]) == slice_word(blk, c % 16)
    keys = []
    for r in range(50):
        blk = chacha.blocks(key, r // 8, 0, 16 + osh.P23, 0, 12)[0]
        e = r % 8
        keys.append(slice_word(blk, 2 * e) | (slice_word(blk, 2 * e + 1) << 32))
    np.testing.assert_array_equal(osh.permutation(seed, osh.P23, 50),
                                  sorted(range(50), key=lambda r: (keys[r], r)))
