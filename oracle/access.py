"""Oracle for secure neighbouring-vertex access (Alg. 6) over a graph encoded
as in Sec. V-B / Alg. 1: one-hot IDs in binary RSS, posting lists padded with
0-vectors (dummy IDs) -- per group of k same-type vertices of similar list
length (Alg. 1), or to one common length (the dense special case).

TEST INFRASTRUCTURE ONLY (see ``oracle/fss.py``).

Encoding (client side, Alg. 1): the X vertices of the neighbour type carry
IDs 0..X-1; a candidate's posting list is its neighbours' one-hot IDs, padded
with all-zero IDs.  The paper pads each group of k same-type vertices of
similar degree to one length; a table of records needs one length, so every
list is padded to the maximum L_max -- a special case that keeps each group
equal.  Pads are placed at random positions within the list (seeded).

Access for a matched vertex with one-hot ID id_m over the C candidates:
  1. P_m[l] = XOR_c id_m[c] AND id_{c,l}  (a selection product; the
     three-out-of-three products are re-shared into RSS)
  2. shuffle the L_max fetched records, open y = XOR of the bits of each,
     keep the records with y = 1 (valid IDs)
  3. d_ne = XOR_x id_ne[x] AND d_x for each kept ID  (selection product,
     re-shared)
"""
from __future__ import annotations

import numpy as np

from . import rss, shuffle


def words(bits: int) -> int:
    return (bits + 31) // 32


def pack_rows(bits: np.ndarray) -> np.ndarray:
    """(R, nbits) 0/1 -> (R, words) uint32, bit p of a row in word p // 32."""
    r, nb = bits.shape
    w = words(nb)
    padded = np.zeros((r, w * 32), np.uint8)
    padded[:, :nb] = bits
    return np.packbits(padded.reshape(r, w, 32), axis=2, bitorder="little").view("<u4").reshape(r, w).astype(np.uint32)


def encode_posting_lists(adj, x_count: int, seed: int):
    """adj: list over candidates of neighbour-ID lists.  Returns the plaintext
    table (C, L_max, words(X)) of one-hot IDs with 0-vector pads."""
    rng = np.random.default_rng(seed)
    lmax = max(1, max(len(a) for a in adj))
    table = np.zeros((len(adj), lmax, x_count), np.uint8)
    for c, nbrs in enumerate(adj):
        slots = rng.permutation(lmax)[:len(nbrs)]
        for s, v in zip(slots, nbrs):
            table[c, s, v] = 1
    packed = pack_rows(table.reshape(len(adj) * lmax, x_count)).reshape(len(adj), lmax, words(x_count))
    return packed, lmax


def rss_split(table: np.ndarray, seed: int):
    rng = np.random.default_rng(seed)
    s1 = rng.integers(0, 2**32, table.shape, dtype=np.uint64).astype(np.uint32)
    s2 = rng.integers(0, 2**32, table.shape, dtype=np.uint64).astype(np.uint32)
    return [s1, s2, table ^ s1 ^ s2]


def selection(x_bits, rows, prf_keys, counter: int):
    """XOR over c of x[c] AND rows[c] on RSS shares, re-shared into RSS.
    x_bits: three (C,) 0/1 share vectors; rows: three (C, W) tables."""
    add = shuffle.fetch_case1(x_bits, rows)
    w = rows[0].shape[1]
    return rss.reshare(add, prf_keys, counter, 32 * w)


def compact_valid(table, seeds):
    """Shuffle records, open the XOR of each record's bits, keep y = 1."""
    r = shuffle.sec_shuffle(table, *seeds)
    full = r[0] ^ r[1] ^ r[2]
    parity = np.zeros(full.shape[0], np.uint32)
    for w in range(full.shape[1]):
        parity ^= full[:, w]
    y = np.array([bin(int(v)).count("1") & 1 for v in parity], np.uint8)
    keep = np.flatnonzero(y)
    return keep, [r[i][keep] for i in range(3)]


def unpack_onehot(record_bits: np.ndarray, nbits: int):
    """(W,) uint32 -> position list of set bits among the first nbits."""
    bits = np.unpackbits(record_bits.astype("<u4").view(np.uint8), bitorder="little")[:nbits]
    return np.flatnonzero(bits)


def sec_access(idm_shares, posting_shares, attr_shares, x_count: int, prf_keys, seeds, counter0: int = 0):
    """Alg. 6 for one matched vertex.  idm_shares: three (C,) 0/1 vectors;
    posting_shares: three (C, L_max, Wx) tables; attr_shares: three (X, Wd)
    tables.  Returns (ID record shares, attribute record shares), both lists
    of three arrays (one row per kept neighbour).
      1. P_m[l] = XOR_c id_m[c] AND id_{c,l}, re-shared (counter counter0);
      2. shuffle, open the XOR of each record's bits, keep y = 1;
      3. per kept ID, d = XOR_x id[x] AND d_x; the kept IDs' attribute
         records re-shared together (counter counter0 + 1)."""
    c, lmax, wx = posting_shares[0].shape
    rows = [p.reshape(c, lmax * wx) for p in posting_shares]
    pm = selection(idm_shares, rows, prf_keys, counter0)
    table = [p.reshape(lmax, wx) for p in pm]
    keep, ids = compact_valid(table, seeds)
    wd = attr_shares[0].shape[1]
    if keep.size == 0:
        return ids, [np.zeros((0, wd), np.uint32) for _ in range(3)]
    add = [np.zeros((keep.size, wd), np.uint32) for _ in range(3)]
    for k in range(keep.size):
        xb = [np.unpackbits(ids[i][k].astype("<u4").view(np.uint8), bitorder="little")[:x_count]
              for i in range(3)]
        d = shuffle.fetch_case1(xb, attr_shares)
        for i in range(3):
            add[i][k] = d[i]
    attrs = rss.reshare([a.reshape(-1) for a in add], prf_keys, counter0 + 1, 32 * keep.size * wd)
    return ids, [a.reshape(keep.size, wd) for a in attrs]


# --------------------------------------------------------------------------- Alg. 1 with k-groups

def group_k(lengths, types, k: int):
    """Alg. 1's degree protection: the vertices of each type are taken k at a
    time in order of posting-list length (ties by vertex ID), so that each
    group holds vertices of similar length, and every list of a group is
    padded to the group's longest.  A type whose vertex count is not a
    multiple of k puts the remainder into its last group (a group of at least
    k whenever the type has k vertices).

    With several posting-list types per vertex (``lengths`` of shape (L, n),
    row l the lengths of list type l), Alg. 1 picks ONE group for a vertex
    and pads each of its list types within that group, so that every vertex
    shares its whole vector of padded lengths with at least k - 1 others: the
    order is then by the length vector, list type 0 first, ties by vertex ID.
    Returns (padded lengths, of the shape of ``lengths``; group of each
    vertex)."""
    lengths = np.asarray(lengths, np.int64)
    one = lengths.ndim == 1
    lv = lengths[None, :] if one else lengths
    types = np.asarray(types)
    n = lv.shape[1]
    padded = np.zeros(lv.shape, np.int64)
    group = np.full(n, -1, np.int64)
    gid = 0
    for t in np.unique(types):
        members = np.flatnonzero(types == t)
        # np.lexsort sorts by its last key first: list type 0, then 1, ..., then the ID
        order = members[np.lexsort((members,) + tuple(lv[l][members] for l in reversed(range(lv.shape[0]))))]
        ngroups = max(1, order.size // k)
        for g in range(ngroups):
            sel = order[g * k:(g + 1) * k] if g < ngroups - 1 else order[g * k:]
            for l in range(lv.shape[0]):
                padded[l, sel] = lv[l, sel].max()
            group[sel] = gid
            gid += 1
    return (padded[0] if one else padded), group


def csr_offsets(padded) -> np.ndarray:
    return np.concatenate([[0], np.cumsum(np.asarray(padded, np.int64))]).astype(np.int64)


def encode_posting_lists_k(adj, x_count: int, padded, slots):
    """The padded posting lists as one-hot records in CSR order: vertex v's
    padded[v] records start at offset off[v]; its i-th true neighbour adj[v][i]
    is the one-hot record at slot slots[v][i] (flat, CSR-aligned), every other
    record of its list an all-zero dummy ID.  Returns (records (nrec, Wx), off)."""
    off = csr_offsets(padded)
    table = np.zeros((int(off[-1]), x_count), np.uint8)
    at = 0
    for v, nbrs in enumerate(adj):
        for i, x in enumerate(nbrs):
            table[off[v] + int(slots[at + i]), int(x)] = 1
        at += len(nbrs)
    return pack_rows(table), off


def rss_split_prf(table: np.ndarray, key_a: int, key_b: int, counter: int):
    """Binary RSS of a table of words (row-major): share 1 = F(key_a, counter)
    and share 2 = F(key_b, counter) over the table's words (the ChaCha12 PRF of
    the re-share), share 3 = table ^ share 1 ^ share 2."""
    n = table.size
    s1 = rss.prf_words(key_a, counter, n).reshape(table.shape)
    s2 = rss.prf_words(key_b, counter, n).reshape(table.shape)
    return [s1, s2, table ^ s1 ^ s2]


def sec_access_csr(idm_shares, post_shares, off, attr_shares, x_count: int, prf_keys, seeds, counter0: int = 0):
    """Alg. 6 over the Alg. 1 encoding (CSR lists of per-group lengths): the
    selection of step 1 runs over slots l < L_max, where L_max is the longest
    padded list; a candidate whose list is shorter contributes nothing to the
    slots beyond it -- the same as padding it with zero records to L_max."""
    c = off.size - 1
    lens = np.diff(off)
    lmax = max(1, int(lens.max()) if c else 1)
    wx = post_shares[0].shape[1]
    dense = []
    for sh in post_shares:
        d = np.zeros((c, lmax, wx), np.uint32)
        for v in range(c):
            d[v, :lens[v]] = sh[off[v]:off[v + 1]]
        dense.append(d)
    return sec_access(idm_shares, dense, attr_shares, x_count, prf_keys, seeds, counter0)
