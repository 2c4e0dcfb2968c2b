"""Oracle for the paper's own secure predicate evaluation over one-hot,
replicated-secret-shared attributes (Sec. V-B, Sec. V-C token generation,
Eq. predEval and Alg. 3 of Sec. V-D).

TEST INFRASTRUCTURE ONLY (see ``oracle/fss.py``).

* An attribute value d in [0, n) is the one-hot vector e_d in {0,1}^n; it is
  split into three binary shares <e>_1, <e>_2, <e>_3 with XOR e_d, and server
  CS_i holds (<e>_i, <e>_{i+1}) (Sec. III-B, Sec. V-B).
* A predicate's token is three independent FSS key pairs (k_1^j, k_2^j),
  j = 1, 2, 3, for the same function with beta = 1 in Z_2 (Sec. V-C);
  CS_1 receives (k_1^1, k_1^2), CS_2 (k_2^2, k_1^3), CS_3 (k_2^3, k_2^1).
* Each server evaluates each of its keys at every public position l and takes
  the XOR over l of Eval(k, l) AND <e[l]>_j for the matching share j; its two
  terms XORed are its additive (3-out-of-3) share x_i of the predicate bit, and
  x_1 ^ x_2 ^ x_3 = f(d) (the six-term identity after Eq. predEval).

Keys here are the two-party DPF / range keys of ``oracle/fss.py`` with mask
r = 0, replica j taken from key row j - 1 (the dealer's randomness is addressed
by row, so the three pairs are independent).  Shares are passed in.
"""
from __future__ import annotations

import numpy as np

from . import chacha, fss

# (party of the key, replica j - 1, share index - 1) for the two terms of CS_1, CS_2, CS_3
SERVER_TERMS = [
    ((0, 0, 0), (0, 1, 1)),    # CS_1: k_1^1 on <.>_1, k_1^2 on <.>_2
    ((1, 1, 1), (0, 2, 2)),    # CS_2: k_2^2 on <.>_2, k_1^3 on <.>_3
    ((1, 2, 2), (1, 0, 0)),    # CS_3: k_2^3 on <.>_3, k_2^1 on <.>_1
]


def domain_bits(npos: int) -> int:
    return max(8, int(np.ceil(np.log2(max(npos, 2)))))


def token(kind: str, npos: int, seed: int, query: int, pred: int, a: int = 0, lo: int = 0, hi: int = 0):
    """Three replicated key pairs for f(l) = [l == a] or [lo <= l < hi] over
    positions l in [0, npos): returns (keys party 0, keys party 1), rows 0..2."""
    nb = domain_bits(npos)
    zero = np.zeros(3, np.uint32)
    if kind == "eq":
        return fss.keygen_eq(nb, seed, query, pred, a, zero), nb
    return fss.keygen_range(nb, seed, query, pred, lo, hi, zero), nb


def eval_all(kind: str, nbits: int, party: int, keys, replica: int, npos: int) -> np.ndarray:
    """Eval(k, l) for l = 0 .. npos-1 (one key, every public position)."""
    pts = np.arange(npos, dtype=np.uint32)
    k = keys[replica:replica + 1]
    if kind == "eq":
        return fss.dpf_eval_points(party, k, nbits, pts)
    out = np.zeros(npos, np.uint8)
    for i, x in enumerate(pts):
        out[i] = fss.eval_range(nbits, party, k, np.array([x], np.uint32))[0]
    return out


def server_shares(kind: str, npos: int, keys_pair, nbits: int, shares) -> np.ndarray:
    """x_i for i = 1..3 and every candidate: shape (3, C), 0/1.
    shares: array (3, C, npos) of 0/1 (the three RSS shares of each one-hot row)."""
    ev = {}
    out = np.zeros((3, shares.shape[1]), np.uint8)
    for i, terms in enumerate(SERVER_TERMS):
        for party, replica, j in terms:
            key = (party, replica)
            if key not in ev:
                ev[key] = eval_all(kind, nbits, party, keys_pair[party], replica, npos)
            # XOR over positions of Eval(k, l) AND <e[l]>_j
            out[i] ^= (np.bitwise_and(shares[j], ev[key][None, :]).sum(axis=1) & 1).astype(np.uint8)
    return out


# --------------------------------------------------------------------------- three-party RSS arithmetic

def prf_words(key_seed: int, counter: int, nwords: int) -> np.ndarray:
    """F(k, j) on packed words: ChaCha12 (``oracle/chacha.py``) under the key
    (k mod 2^32, k div 2^32, 5, 0, 0, 0, 0, 0); word w is slice word (w mod 16)
    of block (w div 16, j, 0, 0), a block's words read column by column (slice
    word 4c + k = state word 4k + c)."""
    k = key_seed & ((1 << 64) - 1)
    nblk = (nwords + 15) // 16
    words = chacha.blocks([k & 0xFFFFFFFF, k >> 32, 5, 0, 0, 0, 0, 0], np.arange(nblk, dtype=np.uint64), counter, 0,
                          0, 12)
    words = words.reshape(-1, 4, 4).transpose(0, 2, 1).reshape(-1)
    return words[:nwords].astype(np.uint32)


def prf_words_at(key_seed: int, counter: int, idx) -> np.ndarray:
    """Words idx (any indices) of F(k, j) as ``prf_words`` defines them, making
    only the blocks that hold them (for samples of very long streams)."""
    k = key_seed & ((1 << 64) - 1)
    idx = np.asarray(idx, dtype=np.int64)
    blk = np.unique(idx // 16)
    words = chacha.blocks([k & 0xFFFFFFFF, k >> 32, 5, 0, 0, 0, 0, 0], blk.astype(np.uint64), counter, 0, 0, 12)
    words = words.reshape(-1, 4, 4).transpose(0, 2, 1).reshape(-1, 16)
    return words[np.searchsorted(blk, idx // 16), idx % 16].astype(np.uint32)


def zero_shares(prf_keys, counter: int, nwords: int):
    """<alpha>_i = F(k_i, j) ^ F(k_{i-1}, j): three shares of 0 (Sec. III-B)."""
    f = [prf_words(k, counter, nwords) for k in prf_keys]
    return [f[i] ^ f[(i - 1) % 3] for i in range(3)]


def reshare(x3, prf_keys, counter: int, nrows: int):
    """Three-out-of-three XOR shares x_1, x_2, x_3 (packed words) -> RSS shares:
    z_i = x_i ^ <alpha>_i.  Party P_i keeps z_i and receives z_{i+1} from P_{i+1}
    so that it holds (z_i, z_{i+1}).  Pad bits beyond nrows cleared."""
    nwords = x3[0].size
    a = zero_shares(prf_keys, counter, nwords)
    vm = fss.valid_mask(nrows)
    return [(x3[i] ^ a[i]) & vm for i in range(3)]


def from_two_party(y0, y1, prf_keys, counter: int, nrows: int):
    """Two-party XOR shares of the masked-input path (party 0 held by server
    P_1, party 1 by P_2) -> three-party RSS shares: (y0, y1, 0) is a
    three-out-of-three XOR sharing of the same bits, which the re-share of
    Sec. III-B turns into RSS (P_3 contributes only its zero share)."""
    return reshare([y0, y1, np.zeros_like(y0)], prf_keys, counter, nrows)


def rss_and(x, y, prf_keys, counter: int, nrows: int):
    """AND of two RSS-shared packed bit vectors (Sec. III-B): P_i forms
    z_i = x_i y_i ^ x_i y_{i+1} ^ x_{i+1} y_i from the shares it holds, then
    the result is re-shared."""
    z3 = [(x[i] & y[i]) ^ (x[i] & y[(i + 1) % 3]) ^ (x[(i + 1) % 3] & y[i]) for i in range(3)]
    return reshare(z3, prf_keys, counter, nrows)
