"""Pins of the oracle's ChaCha block function (the generator of the shuffle's
pairwise tables and permutation keys): RFC 8439's quarter-round and block
vectors, the published reduced-round vectors, and an independent
implementation (the openssl command-line tool) on random keys and counters."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import chacha

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _key_words(hexkey):
    b = bytes.fromhex(hexkey)
    return [int.from_bytes(b[4 * i:4 * i + 4], "little") for i in range(8)]


def test_rfc8439_quarter_round():
    """RFC 8439 section 2.1.1."""
    a, b, c, d = chacha.quarter_round(*[np.array([v], dtype=np.uint32)
                                        for v in (0x11111111, 0x01020304, 0x9B8D6F43, 0x01234567)])
    assert [int(a[0]), int(b[0]), int(c[0]), int(d[0])] == [0xEA2A92F4, 0xCB1CF8CE, 0x4581472E, 0x5881C4BB]


def test_known_answer_vectors():
    with open(os.path.join(GOLDEN, "chacha_vectors.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 4
    for rounds, key, tail, out in rows:
        w = [int(x, 16) for x in tail.split(",")]
        assert chacha.keystream_bytes(_key_words(key), *w, rounds=int(rounds)).hex() == out


def test_vectorised_blocks_are_the_single_blocks():
    key = list(range(100, 108))
    many = chacha.blocks(key, np.arange(5, dtype=np.uint64), 7, np.array([1, 2, 3, 4, 5]), 9, 12)
    for i in range(5):
        one = chacha.blocks(key, i, 7, i + 1, 9, 12)
        np.testing.assert_array_equal(many[i], one[0])


@pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl not installed")
def test_against_openssl_chacha20():
    """openssl's chacha20 takes a 16-byte IV = state words 12-15, little-endian."""
    rng = np.random.default_rng(8439)
    for _ in range(4):
        key = rng.integers(0, 256, 32, dtype=np.uint8).tobytes()
        tail = [int(x) for x in rng.integers(0, 2**32, 4, dtype=np.uint64)]
        iv = b"".join(t.to_bytes(4, "little") for t in tail)
        res = subprocess.run(["openssl", "enc", "-chacha20", "-K", key.hex(), "-iv", iv.hex()],
                             input=bytes(128), stdout=subprocess.PIPE, check=True)
        kw = _key_words(key.hex())
        want = chacha.keystream_bytes(kw, *tail, rounds=20)
        nxt = chacha.keystream_bytes(kw, (tail[0] + 1) % 2**32, *tail[1:], rounds=20)
        assert res.stdout == want + nxt
