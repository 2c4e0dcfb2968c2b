"""ChaCha block function (Bernstein 2008; the 20-round form is RFC 8439,
section 2.3), written from its definition in numpy, vectorised over blocks.

TEST INFRASTRUCTURE ONLY (see ``oracle/fss.py``).

The state is 16 little-endian 32-bit words: the four constants of
"expand 32-byte k", eight key words, and words 12-15 (RFC 8439: the block
counter and the three nonce words).  A column round applies the quarter round
to (0, 4, 8, 12), (1, 5, 9, 13), (2, 6, 10, 14), (3, 7, 11, 15); a diagonal
round to (0, 5, 10, 15), (1, 6, 11, 12), (2, 7, 8, 13), (3, 4, 9, 14).  An
r-round block is r/2 column-and-diagonal pairs, and its output is the final
state plus the initial state, word by word mod 2^32.

The shuffle's pairwise tables and permutation keys use 12 rounds (the paper
asks only for a pseudo-random generator under each pair's seed; it fixes
none).
"""
from __future__ import annotations

import numpy as np

SIGMA = (0x61707865, 0x3320646E, 0x79622D32, 0x6B206574)     # "expand 32-byte k", little-endian words


def _rotl(x: np.ndarray, n: int) -> np.ndarray:
    return (x << np.uint32(n)) | (x >> np.uint32(32 - n))


def quarter_round(a, b, c, d):
    """One quarter round on four uint32 arrays; returns the new (a, b, c, d)."""
    a = a + b; d = _rotl(d ^ a, 16)
    c = c + d; b = _rotl(b ^ c, 12)
    a = a + b; d = _rotl(d ^ a, 8)
    c = c + d; b = _rotl(b ^ c, 7)
    return a, b, c, d


_COLUMNS = ((0, 4, 8, 12), (1, 5, 9, 13), (2, 6, 10, 14), (3, 7, 11, 15))
_DIAGONALS = ((0, 5, 10, 15), (1, 6, 11, 12), (2, 7, 8, 13), (3, 4, 9, 14))


def blocks(key, w12, w13, w14, w15, rounds: int = 12) -> np.ndarray:
    """ChaCha output blocks, shape (N, 16) uint32, for the 8 key words ``key``
    and state words 12-15 given as scalars or arrays of one length N."""
    if rounds % 2:
        raise ValueError("rounds must be even")
    key = [np.uint32(k) for k in key]
    if len(key) != 8:
        raise ValueError("eight key words")
    tail = [np.atleast_1d(np.asarray(w, dtype=np.uint64)).astype(np.uint32) for w in (w12, w13, w14, w15)]
    n = max(len(t) for t in tail)
    tail = [np.broadcast_to(t, (n,)).copy() for t in tail]
    init = [np.full(n, np.uint32(s), dtype=np.uint32) for s in SIGMA]
    init += [np.full(n, k, dtype=np.uint32) for k in key]
    init += tail
    x = [w.copy() for w in init]
    with np.errstate(over="ignore"):
        for _ in range(rounds // 2):
            for group in (_COLUMNS, _DIAGONALS):
                for (i, j, k, l) in group:
                    x[i], x[j], x[k], x[l] = quarter_round(x[i], x[j], x[k], x[l])
        out = np.stack([x[i] + init[i] for i in range(16)], axis=1)
    return out.astype(np.uint32)


def keystream_bytes(key, w12, w13, w14, w15, rounds: int = 20) -> bytes:
    """The serialised block (words little-endian), as a stream cipher emits it."""
    return blocks(key, w12, w13, w14, w15, rounds).astype("<u4").tobytes()
