"""Alg. 1 encoding and Alg. 6 secAccess on the GPU over 12,000 candidates,
with ID records of 63 words (4-byte loads) and of 64 words (16-byte loads):
the encoder's three RSS shares equal the oracle's share for share; for matched
vertices with short, long and empty posting lists, the kept ID records, their
shuffled positions, their count and the attribute records equal the oracle's
share for share, and they reconstruct to the vertex's true neighbours and
their attributes."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import DEV, T, U
from oracle import access

pytestmark = pytest.mark.gpu

NC, KGROUP = 12000, 4


@pytest.fixture(scope="module")
def fss():
    from paper_2209_03526_amd import fss as f
    return f


@pytest.fixture(scope="module", params=[2000, 2048])
def enc(fss, request):
    X = request.param
    WX = (X + 31) // 32
    types, adj, attr = synth.posting_graph(21, NC, X, 24, n_types=2)
    lengths = np.array([len(a) for a in adj], np.uint32)
    padded, _ = fss.rss_group_k(lengths, types, KGROUP)
    slots = synth.posting_slots(22, lengths, padded)
    rec, off = access.encode_posting_lists_k(adj, X, padded, slots)
    want = access.rss_split_prf(rec, 1001, 1002, 4)
    adj_off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.uint32)
    flat = np.concatenate(adj).astype(np.uint32)
    nrec = int(off[-1])
    out = [torch.full((nrec * WX,), -1, dtype=torch.int32, device=DEV) for _ in range(3)]
    d_off = T(off.astype(np.uint32))
    fss.rss_enc_posting_lists(NC, X, T(adj_off), T(flat), T(slots), d_off, nrec, (1001, 1002), 4, out)
    torch.cuda.synchronize()
    return dict(types=types, adj=adj, attr=attr, padded=padded, off=off, d_off=d_off, nrec=nrec, want=want, out=out,
                X=X, WX=WX)


def test_encoding_shares_equal_oracle(fss, enc):
    WX = enc["WX"]
    for i in range(3):
        np.testing.assert_array_equal(U(enc["out"][i]).reshape(enc["nrec"], WX), enc["want"][i],
                                      err_msg=f"share {i + 1}")
    for t in np.unique(enc["types"]):                   # k-anonymity of the padded lengths
        _, counts = np.unique(enc["padded"][enc["types"] == t], return_counts=True)
        assert counts.min() >= KGROUP


def _split_bits(rng, bits):
    s1 = rng.integers(0, 2, bits.size, dtype=np.uint8)
    s2 = rng.integers(0, 2, bits.size, dtype=np.uint8)
    return [s1, s2, bits ^ s1 ^ s2]


def _pack(bits):
    from oracle import fss as ofss
    return ofss.pack_bits(bits)


@pytest.mark.parametrize("pick", ["long", "short", "empty", "middle"])
def test_sec_access_equals_oracle(fss, enc, pick):
    X, WX = enc["X"], enc["WX"]
    lens = np.array([len(a) for a in enc["adj"]])
    m = {"long": int(np.argmax(lens)), "short": int(np.flatnonzero(lens == 1)[0]),
         "empty": int(np.flatnonzero(lens == 0)[0]), "middle": int(np.flatnonzero(lens == 5)[0])}[pick]
    rng = np.random.default_rng(m)
    idm = np.zeros(NC, np.uint8)
    idm[m] = 1
    idm_sh = _split_bits(rng, idm)
    attr_sh = access.rss_split(enc["attr"], 31 + m)
    keys, seeds, counter = [51, 52, 53], (61 + m, 62, 63), 9
    lmax = int(enc["padded"].max())
    want_ids, want_attrs = access.sec_access_csr(idm_sh, enc["want"], enc["off"], attr_sh, X, keys, seeds, counter)
    kept = want_ids[0].shape[0]
    ids = [torch.full((lmax * WX,), -1, dtype=torch.int32, device=DEV) for _ in range(3)]
    attrs = [torch.full((lmax * 2,), -1, dtype=torch.int32, device=DEV) for _ in range(3)]
    rows = torch.full((lmax,), -1, dtype=torch.int32, device=DEV)
    count = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    post = [t for t in enc["out"]]
    fss.rss_sec_access(NC, X, [T(_pack(b)) for b in idm_sh], enc["d_off"], lmax, post, 2, [T(a) for a in attr_sh],
                       keys, counter, seeds, ids, attrs, rows, count)
    torch.cuda.synchronize()
    assert int(U(count)[0]) == kept == lens[m]
    got_ids = [U(t).reshape(lmax, WX)[:kept] for t in ids]
    got_attrs = [U(t).reshape(lmax, 2)[:kept] for t in attrs]
    for i in range(3):
        np.testing.assert_array_equal(got_ids[i], want_ids[i], err_msg=f"ID share {i + 1}")
        np.testing.assert_array_equal(got_attrs[i], want_attrs[i], err_msg=f"attribute share {i + 1}")
    rec = got_ids[0] ^ got_ids[1] ^ got_ids[2]
    nb = sorted(int(access.unpack_onehot(r, X)[0]) for r in rec)
    assert nb == enc["adj"][m].tolist()
    at = got_attrs[0] ^ got_attrs[1] ^ got_attrs[2]
    for r, a in zip(rec, at):
        np.testing.assert_array_equal(a, enc["attr"][int(access.unpack_onehot(r, X)[0])])


def test_sec_access_batch_equals_oracle_per_call(fss, enc):
    """rss_sec_access_batch over four matched vertices (long, short, empty and
    middle lists), each call with its own counter and seeds: call c's slots
    of the outputs equal the oracle's single secAccess with those arguments,
    share for share."""
    X, WX = enc["X"], enc["WX"]
    lens = np.array([len(a) for a in enc["adj"]])
    picks = [int(np.argmax(lens)), int(np.flatnonzero(lens == 1)[0]), int(np.flatnonzero(lens == 0)[0]),
             int(np.flatnonzero(lens == 5)[0])]
    rng = np.random.default_rng(77)
    attr_sh = access.rss_split(enc["attr"], 88)
    keys, lmax = [51, 52, 53], int(enc["padded"].max())
    idm_t, idm_ptrs, counters, seeds, wants = [], [], [], [], []
    for c, m in enumerate(picks):
        idm = np.zeros(NC, np.uint8)
        idm[m] = 1
        sh = _split_bits(rng, idm)
        ts = [T(_pack(b)) for b in sh]
        idm_t.append(ts)
        idm_ptrs += [t.data_ptr() for t in ts]
        counters.append(20 + 2 * c)
        sd = (300 + 3 * c, 301 + 3 * c, 302 + 3 * c)
        seeds += list(sd)
        wants.append(access.sec_access_csr(sh, enc["want"], enc["off"], attr_sh, X, keys, sd, 20 + 2 * c))
    n = len(picks)
    ids = [torch.full((n * lmax * WX,), -1, dtype=torch.int32, device=DEV) for _ in range(3)]
    attrs = [torch.full((n * lmax * 2,), -1, dtype=torch.int32, device=DEV) for _ in range(3)]
    rows = torch.full((n * lmax,), -1, dtype=torch.int32, device=DEV)
    count = torch.full((n,), -1, dtype=torch.int32, device=DEV)
    fss.rss_sec_access_batch(NC, X, idm_ptrs, enc["d_off"], lmax, list(enc["out"]), 2, [T(a) for a in attr_sh],
                             keys, counters, seeds, ids, attrs, rows, count)
    torch.cuda.synchronize()
    got_count = U(count)
    for c, m in enumerate(picks):
        want_ids, want_attrs = wants[c]
        kept = want_ids[0].shape[0]
        assert int(got_count[c]) == kept == lens[m]
        for i in range(3):
            gi = U(ids[i]).reshape(n, lmax, WX)[c, :kept]
            ga = U(attrs[i]).reshape(n, lmax, 2)[c, :kept]
            np.testing.assert_array_equal(gi, want_ids[i], err_msg=f"call {c} ID share {i + 1}")
            np.testing.assert_array_equal(ga, want_attrs[i], err_msg=f"call {c} attribute share {i + 1}")


def test_sec_access_measured_size(fss):
    """secAccess at the measured size (65,536 candidates, 16,384 neighbour IDs:
    2 KB one-hot records, lists of 0..24 IDs, k = 4): for the vertex with the
    longest list, the opened count is its true length, the kept ID records
    reconstruct to its neighbours and the attribute records to theirs; and the
    encoder's first two shares equal the oracle's PRF words at 64 sampled
    records (the third is the records XOR both)."""
    from oracle import rss as orss
    nc, xbits = 1 << 16, 1 << 14
    wx = xbits // 32
    types, adj, attr = synth.posting_graph(33, nc, xbits, 24, n_types=2)
    lengths = np.array([len(a) for a in adj], np.uint32)
    padded, _ = fss.rss_group_k(lengths, types, 4)
    slots = synth.posting_slots(34, lengths, padded)
    off = np.concatenate([[0], np.cumsum(padded)]).astype(np.uint32)
    nrec, lmax = int(off[-1]), int(padded.max())
    adj_off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.uint32)
    d_off = T(off)
    post = [torch.empty(nrec * wx, dtype=torch.int32, device=DEV) for _ in range(3)]
    fss.rss_enc_posting_lists(nc, xbits, T(adj_off), T(np.concatenate(adj).astype(np.uint32)), T(slots), d_off, nrec,
                              (91, 92), 7, post)
    torch.cuda.synchronize()
    rng = np.random.default_rng(35)
    recs = np.sort(rng.choice(nrec, 64, replace=False))
    for j, key in enumerate((91, 92)):
        words = (recs[:, None] * wx + np.arange(wx)[None, :]).ravel()
        want = orss.prf_words_at(key, 7, words).reshape(len(recs), wx)
        got = U(post[j]).reshape(nrec, wx)[recs]
        np.testing.assert_array_equal(got, want, err_msg=f"share {j + 1}")
    m = int(np.argmax(lengths))
    idm = np.zeros(nc, np.uint8)
    idm[m] = 1
    idm_sh = _split_bits(rng, idm)
    attr_sh = access.rss_split(attr, 36)
    ids = [torch.empty(lmax * wx, dtype=torch.int32, device=DEV) for _ in range(3)]
    attrs = [torch.empty(lmax * 2, dtype=torch.int32, device=DEV) for _ in range(3)]
    rows = torch.empty(lmax, dtype=torch.int32, device=DEV)
    count = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    fss.rss_sec_access(nc, xbits, [T(_pack(b)) for b in idm_sh], d_off, lmax, post, 2, [T(a) for a in attr_sh],
                       [51, 52, 53], 9, (61, 62, 63), ids, attrs, rows, count)
    torch.cuda.synchronize()
    kept = int(U(count)[0])
    assert kept == lengths[m]
    rec = U(ids[0]).reshape(lmax, wx)[:kept] ^ U(ids[1]).reshape(lmax, wx)[:kept] ^ U(ids[2]).reshape(lmax, wx)[:kept]
    nb = [int(access.unpack_onehot(r, xbits)[0]) for r in rec]
    assert sorted(nb) == adj[m].tolist()
    at = U(attrs[0]).reshape(lmax, 2)[:kept] ^ U(attrs[1]).reshape(lmax, 2)[:kept] ^ U(attrs[2]).reshape(lmax, 2)[:kept]
    for v, a in zip(nb, at):
        np.testing.assert_array_equal(a, attr[v])
