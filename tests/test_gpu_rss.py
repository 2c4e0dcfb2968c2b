"""Parity of the paper's own secEval on the GPU (one-hot RSS attributes,
replicated FSS keys, Eq. predEval): full-domain evaluations and each server's
share bits equal the oracle's bit for bit; the three shares XOR to the
plaintext predicate."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import DEV, T, T_off, U, empty_off
from oracle import fss as ofss
from oracle import rss as orss

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_03526_amd import fss as lib
    torch.cuda.set_device(0)
    return lib


def _gpu_token(fss, kind, npos, seed, query, pred, a=0, lo=0, hi=0):
    nb = orss.domain_bits(npos)
    kb = fss.KeyBatch(fss.EQ if kind == "eq" else fss.RANGE, nb, 3)
    fss.fss_keygen(seed, query, pred, a if kind == "eq" else lo, hi, torch.zeros(3, dtype=torch.int32, device=DEV), kb)
    return kb, nb


@pytest.mark.parametrize("kind,npos,ncand", [("eq", 64, 100003), ("eq", 256, 4099), ("range", 200, 70001),
                                             ("range", 16, 1), ("eq", 33, 640)])
def test_sec_eval_parity(fss, kind, npos, ncand):
    rng = np.random.default_rng(npos + ncand)
    values = rng.integers(0, npos, ncand).astype(np.uint32)
    shares = synth.onehot_rss(npos + 7, values, npos)
    a, lo, hi = int(values[0]), npos // 5, npos - npos // 4
    seed, q, p = 77, 5, 3
    okeys, nb = orss.token(kind, npos, seed, q, p, a=a, lo=lo, hi=hi)
    kb, nb2 = _gpu_token(fss, kind, npos, seed, q, p, a=a, lo=lo, hi=hi)
    assert nb == nb2
    nw = (npos + 31) // 32
    ev = {}
    for party in (0, 1):
        for rep in range(3):
            o = torch.zeros(nw, dtype=torch.int32, device=DEV)
            fss.fss_eval_all(party, kb, rep, npos, o)
            got = ofss.unpack_bits(U(o), npos)
            want = orss.eval_all(kind, nb, party, okeys[party], rep, npos)
            np.testing.assert_array_equal(got, want)
            ev[(party, rep)] = o
    dev_sh = [T(synth.pack_word_major(shares[j])) for j in range(3)]
    want = orss.server_shares(kind, npos, okeys, nb, shares)
    xs = []
    for i, ((pa, ra, ja), (pb, rb, jb)) in enumerate(orss.SERVER_TERMS):
        out = torch.full(((ncand + 31) // 32,), -1, dtype=torch.int32, device=DEV)
        fss.rss_sec_eval(ncand, npos, ev[(pa, ra)], ev[(pb, rb)], dev_sh[ja], dev_sh[jb], out)
        xi = ofss.unpack_bits(U(out), ncand)
        np.testing.assert_array_equal(xi, want[i])
        xs.append(U(out))
    truth = (values == a) if kind == "eq" else ((values >= lo) & (values < hi))
    np.testing.assert_array_equal(ofss.unpack_bits(xs[0] ^ xs[1] ^ xs[2], ncand), truth.astype(np.uint8))
    assert (xs[0][-1] >> (ncand % 32 or 32) if ncand % 32 else 0) == 0


@pytest.mark.parametrize("nrows", [1, 33, 4096, 100001, (1 << 25) + 77])
def test_rss_reshare_and_and(fss, nrows):
    nw = (nrows + 31) // 32
    rng = np.random.default_rng(nrows)
    vm = ofss.valid_mask(nrows)
    x = [rng.integers(0, 2**32, nw, dtype=np.uint64).astype(np.uint32) & vm for _ in range(3)]
    y = [rng.integers(0, 2**32, nw, dtype=np.uint64).astype(np.uint32) & vm for _ in range(3)]
    keys = [101, 202, 303]
    z = [torch.empty(nw, dtype=torch.int32, device=DEV) for _ in range(3)]
    fss.rss_reshare(nrows, [T(a) for a in x], keys, 9, z)
    want = orss.reshare(x, keys, 9, nrows)
    for i in range(3):
        np.testing.assert_array_equal(U(z[i]), want[i])
    fss.rss_and(nrows, [T(a) for a in x], [T(b) for b in y], keys, 10, z)
    want = orss.rss_and(x, y, keys, 10, nrows)
    got = [U(t) for t in z]
    for i in range(3):
        np.testing.assert_array_equal(got[i], want[i])
    np.testing.assert_array_equal(got[0] ^ got[1] ^ got[2], (x[0] ^ x[1] ^ x[2]) & (y[0] ^ y[1] ^ y[2]))


@pytest.mark.parametrize("nrows", [4096 * 32 + 5, 1000])
def test_rss_and_unaligned_buffers(fss, nrows):
    """Share buffers that are not 16-byte aligned take the word-by-word path
    and give the same shares."""
    nw = (nrows + 31) // 32
    rng = np.random.default_rng(nrows + 1)
    vm = ofss.valid_mask(nrows)
    x = [rng.integers(0, 2**32, nw, dtype=np.uint64).astype(np.uint32) & vm for _ in range(3)]
    y = [rng.integers(0, 2**32, nw, dtype=np.uint64).astype(np.uint32) & vm for _ in range(3)]
    keys = [7, 8, 9]
    z = [empty_off(nw) for _ in range(3)]
    assert all(t.data_ptr() % 16 == 4 for t in z)
    fss.rss_and(nrows, [T_off(a) for a in x], [T(b) for b in y], keys, 3, z)
    want = orss.rss_and(x, y, keys, 3, nrows)
    for i in range(3):
        np.testing.assert_array_equal(U(z[i]), want[i])


def test_eval_all_batch_matches_oracle(fss):
    """Ten full-domain evaluations in one call (two launches of at most eight):
    equality and range keys, both parties, several point counts -- each equals
    the oracle's evaluation at every position."""
    seed, q = 31, 9
    tok = {"eq": _gpu_token(fss, "eq", 200, seed, q, 0, a=77), "range": _gpu_token(fss, "range", 3000, seed, q, 1,
                                                                                  lo=100, hi=2500)}
    otok = {"eq": orss.token("eq", 200, seed, q, 0, a=77), "range": orss.token("range", 3000, seed, q, 1, lo=100,
                                                                                hi=2500)}
    reqs, want = [], []
    for i in range(10):
        kind = "eq" if i % 3 == 0 else "range"
        party, rep = i % 2, i % 3
        npos = {"eq": [200, 64, 1][i % 3], "range": [3000, 1025, 33][i % 3]}[kind]
        kb, nb = tok[kind]
        okeys, onb = otok[kind]
        out = torch.full(((npos + 31) // 32,), -1, dtype=torch.int32, device=DEV)
        reqs.append((party, kb, rep, npos, out))
        want.append(orss.eval_all(kind, onb, party, okeys[party], rep, npos))
    fss.fss_eval_all_batch(reqs)
    torch.cuda.synchronize()
    for (party, kb, rep, npos, out), w in zip(reqs, want):
        got = U(out)
        np.testing.assert_array_equal(ofss.unpack_bits(got, npos), w)
        assert npos % 32 == 0 or (got[-1] >> (npos % 32)) == 0


@pytest.mark.parametrize("n", [1, 3000, 70001, (1 << 20) + 13])
def test_fss_to_rss_then_and_chain(fss, n):
    """The masked-input path on the GPU (dealer keygen, open, both parties'
    evaluation of two range predicates), its two-party bits converted to RSS
    (rss_from_fss) and ANDed in RSS (rss_and): every server's share equals the
    oracle's at each step, and the reconstruction is the plaintext conjunction."""
    seed, q = 55, 3
    rng = np.random.default_rng(n)
    x = rng.integers(0, 1 << 20, n).astype(np.uint32)
    x0 = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    x1 = (x - x0).astype(np.uint32)
    bounds = [(1000, 700000), (500000, 1 << 20)]
    keys = [41, 42, 43]
    nw = (n + 31) // 32
    conv, oconv = [], []
    for k, (lo, hi) in enumerate(bounds):
        r = ofss.masks(seed, q, k, n)
        xhat = torch.empty(n, dtype=torch.int32, device=DEV)
        fss.fss_mask_open(T(x0), T(x1), T(r), xhat)
        kb = fss.KeyBatch(fss.RANGE, 32, n)
        fss.fss_keygen(seed, q, k, lo, hi, T(r), kb)
        y = [torch.empty(nw, dtype=torch.int32, device=DEV) for _ in range(2)]
        for b in range(2):
            fss.fss_eval_lt(b, kb, xhat, y[b])
        z = [torch.full((nw,), -1, dtype=torch.int32, device=DEV) for _ in range(3)]
        fss.rss_from_fss(n, y, keys, k, z)
        ok = ofss.keygen_range(32, seed, q, k, lo, hi, r)
        xh = (x + r).astype(np.uint32)
        oy = [ofss.pack_bits(ofss.eval_range(32, b, ok[b], xh)) for b in range(2)]
        for b in range(2):
            np.testing.assert_array_equal(U(y[b]), oy[b], err_msg=f"predicate {k} party {b}")
        want = orss.from_two_party(oy[0], oy[1], keys, k, n)
        for i in range(3):
            np.testing.assert_array_equal(U(z[i]), want[i], err_msg=f"predicate {k} server {i}")
        conv.append(z)
        oconv.append(want)
    out = [torch.full((nw,), -1, dtype=torch.int32, device=DEV) for _ in range(3)]
    fss.rss_and(n, conv[0], conv[1], keys, 7, out)
    want = orss.rss_and(oconv[0], oconv[1], keys, 7, n)
    got = [U(t) for t in out]
    for i in range(3):
        np.testing.assert_array_equal(got[i], want[i], err_msg=f"AND server {i}")
    truth = ((x >= bounds[0][0]) & (x < bounds[0][1]) & (x >= bounds[1][0]) & (x < bounds[1][1])).astype(np.uint8)
    np.testing.assert_array_equal(ofss.unpack_bits(got[0] ^ got[1] ^ got[2], n), truth)


def test_sec_eval_reshare_and_chain(fss):
    """The paper's own chain on the GPU: two predicates by secEval (Eq.
    predEval, three-out-of-three shares), each re-shared into RSS, then ANDed:
    share for share equal to the oracle's chain; reconstruction = conjunction."""
    npos, ncand = 64, 50001
    values = np.random.default_rng(12).integers(0, npos, ncand).astype(np.uint32)
    shares = synth.onehot_rss(12, values, npos)
    dev_sh = [T(synth.pack_word_major(shares[j])) for j in range(3)]
    nw = (ncand + 31) // 32
    keys = [5, 6, 7]
    rss_dev, rss_or = [], []
    for p, (lo, hi) in enumerate([(10, 40), (30, 60)]):
        okeys, nb = orss.token("range", npos, 19, 2, p, lo=lo, hi=hi)
        kb, _ = _gpu_token(fss, "range", npos, 19, 2, p, lo=lo, hi=hi)
        ev = {}
        for party in (0, 1):
            for rep in range(3):
                o = torch.zeros((npos + 31) // 32, dtype=torch.int32, device=DEV)
                fss.fss_eval_all(party, kb, rep, npos, o)
                ev[(party, rep)] = o
        xs = []
        for (pa, ra, ja), (pb, rb, jb) in orss.SERVER_TERMS:
            o = torch.empty(nw, dtype=torch.int32, device=DEV)
            fss.rss_sec_eval(ncand, npos, ev[(pa, ra)], ev[(pb, rb)], dev_sh[ja], dev_sh[jb], o)
            xs.append(o)
        z = [torch.empty(nw, dtype=torch.int32, device=DEV) for _ in range(3)]
        fss.rss_reshare(ncand, xs, keys, p, z)
        ox = orss.server_shares("range", npos, okeys, nb, shares)
        want = orss.reshare([ofss.pack_bits(ox[i]) for i in range(3)], keys, p, ncand)
        for i in range(3):
            np.testing.assert_array_equal(U(z[i]), want[i], err_msg=f"predicate {p} server {i}")
        rss_dev.append(z)
        rss_or.append(want)
    out = [torch.empty(nw, dtype=torch.int32, device=DEV) for _ in range(3)]
    fss.rss_and(ncand, rss_dev[0], rss_dev[1], keys, 9, out)
    want = orss.rss_and(rss_or[0], rss_or[1], keys, 9, ncand)
    got = [U(t) for t in out]
    for i in range(3):
        np.testing.assert_array_equal(got[i], want[i])
    truth = ((values >= 30) & (values < 40)).astype(np.uint8)
    np.testing.assert_array_equal(ofss.unpack_bits(got[0] ^ got[1] ^ got[2], ncand), truth)


@pytest.mark.parametrize("kind,npos,ncand", [("eq", 64, 5003), ("range", 100, 777), ("eq", 8, 1), ("range", 33, 64)])
def test_sec_eval_records_parity(fss, kind, npos, ncand):
    """secEval on candidate-major one-hot records (the layout secFetch and
    secAccess return) equals the oracle's server shares."""
    rng = np.random.default_rng(npos * 7 + ncand)
    values = rng.integers(0, npos, ncand).astype(np.uint32)
    shares = synth.onehot_rss(npos + 11, values, npos)
    a, lo, hi = int(values[-1]), npos // 4, npos - npos // 3
    okeys, nb = orss.token(kind, npos, 91, 6, 2, a=a, lo=lo, hi=hi)
    kb, _ = _gpu_token(fss, kind, npos, 91, 6, 2, a=a, lo=lo, hi=hi)
    nw = (npos + 31) // 32
    ev = {}
    for party in (0, 1):
        for rep in range(3):
            ev[(party, rep)] = torch.zeros(nw, dtype=torch.int32, device=DEV)
            fss.fss_eval_all(party, kb, rep, npos, ev[(party, rep)])
    rec = [T(synth.pack_records(shares[j]).ravel()) for j in range(3)]
    want = orss.server_shares(kind, npos, okeys, nb, shares)
    xs = []
    for i, ((pa, ra, ja), (pb, rb, jb)) in enumerate(orss.SERVER_TERMS):
        out = torch.full(((ncand + 31) // 32,), -1, dtype=torch.int32, device=DEV)
        fss.rss_sec_eval_records(ncand, npos, ev[(pa, ra)], ev[(pb, rb)], rec[ja], rec[jb], out)
        np.testing.assert_array_equal(ofss.unpack_bits(U(out), ncand), want[i])
        xs.append(U(out))
    truth = (values == a) if kind == "eq" else ((values >= lo) & (values < hi))
    np.testing.assert_array_equal(ofss.unpack_bits(xs[0] ^ xs[1] ^ xs[2], ncand), truth.astype(np.uint8))


def test_sec_eval_full_size(fss):
    """secEval at the measured size (2^20 candidates, 4096 positions, a range
    predicate): the three servers' bits XOR to the plaintext predicate for
    every candidate, and at 256 sampled candidates each server's bit equals
    the oracle's Eq. predEval on those candidates' shares."""
    ncand, npos, kind = 1 << 20, 4096, "range"
    nw = npos // 32
    rng = np.random.default_rng(12)
    values = rng.integers(0, npos, ncand).astype(np.int64)
    lo, hi = 1000, 3100
    seed, q, p = 78, 6, 2
    g = torch.Generator(device=DEV).manual_seed(8)
    s1 = torch.randint(-2**31, 2**31, (nw, ncand), dtype=torch.int32, device=DEV, generator=g)
    s2 = torch.randint(-2**31, 2**31, (nw, ncand), dtype=torch.int32, device=DEV, generator=g)
    s3 = s1 ^ s2
    v = torch.from_numpy(values).to(DEV)
    flat = s3.view(-1)
    idx = (v >> 5) * ncand + torch.arange(ncand, device=DEV)
    bit = torch.bitwise_left_shift(torch.ones_like(v), v & 31).to(torch.int64)
    bit = (bit - (bit >= 2**31).to(torch.int64) * 2**32).to(torch.int32)
    flat[idx] = flat[idx] ^ bit                         # one-hot word-major, candidate c at column c
    dev_sh = [s1.ravel(), s2.ravel(), s3.ravel()]
    kb, nb = _gpu_token(fss, kind, npos, seed, q, p, lo=lo, hi=hi)
    ev = {}
    for party in (0, 1):
        for rep in range(3):
            ev[(party, rep)] = torch.zeros(nw, dtype=torch.int32, device=DEV)
            fss.fss_eval_all(party, kb, rep, npos, ev[(party, rep)])
    xs = []
    for i, ((pa, ra, ja), (pb, rb, jb)) in enumerate(orss.SERVER_TERMS):
        out = torch.full((ncand // 32,), -1, dtype=torch.int32, device=DEV)
        fss.rss_sec_eval(ncand, npos, ev[(pa, ra)], ev[(pb, rb)], dev_sh[ja], dev_sh[jb], out)
        xs.append(U(out))
    truth = ((values >= lo) & (values < hi)).astype(np.uint8)
    np.testing.assert_array_equal(ofss.unpack_bits(xs[0] ^ xs[1] ^ xs[2], ncand), truth)
    # sampled candidates against the oracle
    okeys, nb_o = orss.token(kind, npos, seed, q, p, lo=lo, hi=hi)
    assert nb_o == nb
    cs = np.sort(rng.choice(ncand, 256, replace=False))
    cidx = torch.from_numpy(cs).to(DEV)
    sub = []
    for sj in (s1, s2, s3):
        words = U(sj[:, cidx].contiguous()).reshape(nw, len(cs)).T.copy()      # (256, nw)
        sub.append(np.unpackbits(words.view(np.uint8).reshape(len(cs), nw * 4), axis=1, bitorder="little"))
    want = orss.server_shares(kind, npos, okeys, nb, np.stack(sub))
    for i in range(3):
        np.testing.assert_array_equal(ofss.unpack_bits(xs[i], ncand)[cs], want[i], err_msg=f"server {i + 1}")
