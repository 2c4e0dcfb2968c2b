"""Pins of the oracle's AES-128 against FIPS-197 known answers and against an
independent implementation (the openssl command-line tool)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import fss

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_fips197_known_answers():
    rows = _rows("fips197_kat.txt")
    assert len(rows) == 2
    for key, pt, ct in rows:
        assert fss.aes128_encrypt(bytes.fromhex(key), bytes.fromhex(pt)).hex() == ct


def test_fips197_key_expansion():
    for key, i, word in _rows("fips197_keyexp.txt"):
        rk = fss.aes128_round_keys(bytes.fromhex(key))
        i = int(i)
        assert rk[4 * i:4 * i + 4].hex() == word


def test_fips197_sbox_examples():
    for x, y in _rows("fips197_sbox.txt"):
        assert fss.sbox(int(x, 16)) == int(y, 16)


def test_sbox_is_a_permutation_without_fixed_points():
    s = [fss.sbox(x) for x in range(256)]
    assert sorted(s) == list(range(256))
    assert all(s[x] != x and s[x] != x ^ 0xFF for x in range(256))


def _openssl_ecb(key: bytes, data: bytes) -> bytes:
    return subprocess.run(["openssl", "enc", "-aes-128-ecb", "-nopad", "-K", key.hex()],
                          input=data, stdout=subprocess.PIPE, check=True).stdout


@pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl CLI not present")
def test_random_blocks_match_openssl():
    rng = np.random.default_rng(7)
    for _ in range(4):
        key = rng.bytes(16)
        blocks = rng.bytes(16 * 64)
        ref = _openssl_ecb(key, blocks)
        ours = b"".join(fss.aes128_encrypt(key, blocks[16 * i:16 * i + 16]) for i in range(64))
        assert ours == ref


@pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl CLI not present")
def test_dealer_rng_is_aes_counter_mode():
    """block = AES_{LE64(seed) || 'OBLIVGM1'}(LE16 dom || LE16 j || LE32 q || LE32 p || LE32 e)."""
    for seed, dom, j, q, p, e in [(0, 1, 0, 0, 0, 0), (0x0123456789ABCDEF, 3, 4, 77, 5, 123456),
                                  (2**64 - 1, 4, 0, 2**32 - 1, 9, 2**32 - 1)]:
        key = seed.to_bytes(8, "little") + b"OBLIVGM1"
        blk = (dom.to_bytes(2, "little") + j.to_bytes(2, "little") + q.to_bytes(4, "little") +
               p.to_bytes(4, "little") + e.to_bytes(4, "little"))
        assert fss.rng_block(seed, dom, j, q, p, e) == _openssl_ecb(key, blk)


@pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl CLI not present")
def test_dealer_masks_are_domain_2_words():
    r = fss.masks(0xABCDEF, 9, 4, 6, row_offset=100)
    key = (0xABCDEF).to_bytes(8, "little") + b"OBLIVGM1"
    for i in range(6):
        blk = (2).to_bytes(2, "little") + (0).to_bytes(2, "little") + (9).to_bytes(4, "little") + \
              (4).to_bytes(4, "little") + (100 + i).to_bytes(4, "little")
        assert int(r[i]) == int.from_bytes(_openssl_ecb(key, blk)[:4], "little")
