"""Oracle for the three-party secret-shared shuffle (Alg. 5) and secure
matched-vertex fetching (Alg. 4, Cases I and II).

TEST INFRASTRUCTURE ONLY (see ``oracle/fss.py``).

A table D of C records of W 32-bit words is held in binary RSS: three share
tables D_1, D_2, D_3 with XOR D; CS_i holds (D_i, D_{i+1}).  Pairwise seeds
s12, s23, s31 give each pair of servers common pseudo-random permutations and
masks (Alg. 5):
  from s12: pi12, T12, R2;  from s23: pi23, T23;  from s31: pi31, T31, R1.
  CS1: X1 = pi31[pi12(D1 ^ D2 ^ T12) ^ T31]                  -> CS2
  CS2: Y1 = pi12(D3 ^ T12); C1 = pi23(X1 ^ T23) ^ R2          -> CS3
  CS3: C2 = pi23[pi31(Y1 ^ T31) ^ T23] ^ R1; R3 = C1 ^ C2      -> CS2
  result shares (R1, R2, R3), an RSS of pi23(pi31(pi12(D))).
(The algorithm's text names X_2 in CS2's step; the message CS2 holds is X1,
and only that reading makes the shares reconstruct -- see the tests.)

Readings where the paper is silent: a permutation pi applied to a table is
the row gather pi(D)[i] = D[perm[i]]; perm is the stable argsort of 64-bit
keys drawn per row from the pair's seed.  Masks and keys are ChaCha12 output
(``oracle/chacha.py``) under the key (seed mod 2^32, seed div 2^32, 6, 0, 0,
0, 0, 0), with state words 12-15 naming the block.  A block's 16 output words
are read column by column: its slice word 4c + k is state word 4k + c.
  mask word w of record r of table t (W words a record) = slice word (w mod 16)
  of block (r, w div 16, t, W);  sort key of row r for permutation p = slice
  words 2e (low) and 2e + 1 (high), e = r mod 8, of block (r div 8, 0, 16 + p, 0).
Table ids: T12 = 1, R2 = 2, T23 = 3, T31 = 4, R1 = 5; permutation ids:
pi12 = 0, pi23 = 1, pi31 = 2.
"""
from __future__ import annotations

import numpy as np

from . import chacha

T12, R2, T23, T31, R1 = 1, 2, 3, 4, 5
P12, P23, P31 = 0, 1, 2
ROUNDS = 12


def pair_key(seed: int):
    """The eight ChaCha key words of a pair seed (the 6 separates this use)."""
    seed &= (1 << 64) - 1
    return [seed & 0xFFFFFFFF, seed >> 32, 6, 0, 0, 0, 0, 0]


def _slices(words: np.ndarray) -> np.ndarray:
    """Blocks (N, 16) in state order -> (N, 16) in slice order: slice word
    4c + k is state word 4k + c."""
    return words.reshape(-1, 4, 4).transpose(0, 2, 1).reshape(-1, 16)


def mask_table(seed: int, table: int, nrows: int, nwords: int) -> np.ndarray:
    """Record r, word w = slice word (w mod 16) of block (r, w div 16, table, W)."""
    nb = (nwords + 15) // 16
    r = np.repeat(np.arange(nrows, dtype=np.uint64), nb)
    b = np.tile(np.arange(nb, dtype=np.uint64), nrows)
    words = _slices(chacha.blocks(pair_key(seed), r, b, table, nwords, ROUNDS))      # (nrows * nb, 16)
    return words.reshape(nrows, nb * 16)[:, :nwords].copy()


def permutation(seed: int, perm_id: int, nrows: int) -> np.ndarray:
    """Stable argsort of the rows' keys: key of row r = slice words 2e (low)
    and 2e + 1 (high), e = r mod 8, of block (r div 8, 0, 16 + p, 0)."""
    nblk = (nrows + 7) // 8
    words = _slices(chacha.blocks(pair_key(seed), np.arange(nblk, dtype=np.uint64), 0, 16 + perm_id, 0, ROUNDS))
    keys = words.reshape(-1, 2).astype(np.uint64)
    keys = (keys[:, 0] | (keys[:, 1] << np.uint64(32)))[:nrows]
    return np.argsort(keys, kind="stable")


def apply(perm: np.ndarray, table: np.ndarray) -> np.ndarray:
    return table[perm]


def sec_shuffle(D, s12: int, s23: int, s31: int):
    """Alg. 5 step by step: returns (R1, R2, R3)."""
    d1, d2, d3 = D
    n, w = d1.shape
    p12, p23, p31 = permutation(s12, P12, n), permutation(s23, P23, n), permutation(s31, P31, n)
    t12, r2 = mask_table(s12, T12, n, w), mask_table(s12, R2, n, w)
    t23 = mask_table(s23, T23, n, w)
    t31, r1 = mask_table(s31, T31, n, w), mask_table(s31, R1, n, w)
    x1 = apply(p31, apply(p12, d1 ^ d2 ^ t12) ^ t31)           # CS1
    y1 = apply(p12, d3 ^ t12)                                   # CS2
    c1 = apply(p23, x1 ^ t23) ^ r2
    c2 = apply(p23, apply(p31, y1 ^ t31) ^ t23) ^ r1            # CS3
    r3 = c1 ^ c2
    return r1, r2, r3


def composed_permutation(s12: int, s23: int, s31: int, nrows: int) -> np.ndarray:
    """The row order of pi23(pi31(pi12(D))): D[p12][p31][p23] = D[p12[p31[p23]]]."""
    p12, p23, p31 = permutation(s12, P12, nrows), permutation(s23, P23, nrows), permutation(s31, P31, nrows)
    return p12[p31[p23]]


def fetch_case1(x, rows):
    """Case I (exactly one candidate matches): XOR over candidates of
    record_c AND x_c on RSS shares.  x: three (C,) 0/1 share vectors of the
    predicate bits; rows: three (C, W) share tables.  The 3-out-of-3 products
    x_i*r_i ^ x_i*r_{i+1} ^ x_{i+1}*r_i are summed over candidates; returns the
    three additive shares of the fetched record (re-sharing is rss.reshare)."""
    out = []
    for i in range(3):
        j = (i + 1) % 3
        mi = (0 - x[i].astype(np.uint32))[:, None]
        mj = (0 - x[j].astype(np.uint32))[:, None]
        prod = (rows[i] & mi) ^ (rows[j] & mi) ^ (rows[i] & mj)
        out.append(np.bitwise_xor.reduce(prod, axis=0))
    return out


def fetch_case2(x, rows, s12, s23, s31):
    """Case II: shuffle the table {x || record}, open the shuffled x, keep the
    records whose opened bit is 1.  Returns (positions in the shuffled order,
    three share tables of the kept records)."""
    table = [np.concatenate([x[i].astype(np.uint32)[:, None], rows[i]], axis=1) for i in range(3)]
    r = sec_shuffle(table, s12, s23, s31)
    opened = (r[0][:, 0] ^ r[1][:, 0] ^ r[2][:, 0]) & 1
    keep = np.flatnonzero(opened)
    return keep, [r[i][keep, 1:] for i in range(3)]
