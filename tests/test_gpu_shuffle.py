"""Parity of the shuffle (Alg. 5) and fetch (Alg. 4) kernels with the oracle:
each of the three output share tables bit for bit, the reconstruction a
permutation of the input, Case I the unique record, Case II exactly the
matching records in shuffled order."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, T, T_off, U, empty_off
from oracle import fss as ofss
from oracle import shuffle as osh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_03526_amd import fss as lib
    torch.cuda.set_device(0)
    return lib


def _rss_table(seed, n, w):
    rng = np.random.default_rng(seed)
    d = rng.integers(0, 2**32, (n, w), dtype=np.uint64).astype(np.uint32)
    s1 = rng.integers(0, 2**32, (n, w), dtype=np.uint64).astype(np.uint32)
    s2 = rng.integers(0, 2**32, (n, w), dtype=np.uint64).astype(np.uint32)
    return d, [s1, s2, d ^ s1 ^ s2]


# sizes: one run of rows (n <= 64); a few runs; runs longer than one wavefront;
# 2^12 rows exactly; the word path with thousands of runs; the 16-byte path
# with 2^11 runs over a ragged 2^16 + 37 rows.  The radix pass takes its
# single-block path up to 1024 rows, its merge path up to 2^20 and its
# one-sweep path above: 2^20 + 100 rows cover the last.  Widths of 48, 33 and
# 17 words take three, three and two 16-word slices per record (ChaCha blocks),
# the last ones partial.
@pytest.mark.parametrize("n,w", [(1, 1), (17, 3), (64, 4), (1000, 8), (1024, 2), (1025, 2), (3000, 2), (4096, 4),
                                 (5000, 3), (65573, 4), ((1 << 20) + 100, 4), (2, 48), (777, 33), (4099, 17)])
def test_shuffle_parity(fss, n, w):
    d, sh = _rss_table(n + w, n, w)
    seeds = (101, 202, 303)
    out = [torch.empty(n * w, dtype=torch.int32, device=DEV) for _ in range(3)]
    fss.rss_shuffle(n, w, [T(s.ravel()) for s in sh], seeds, out)
    torch.cuda.synchronize()
    want = osh.sec_shuffle(sh, *seeds)
    got = [U(o).reshape(n, w) for o in out]
    for i in range(3):
        np.testing.assert_array_equal(got[i], want[i])
    np.testing.assert_array_equal(got[0] ^ got[1] ^ got[2], d[osh.composed_permutation(*seeds, n)])


@pytest.mark.parametrize("n,w", [(1, 1), (1000, 8), (3001, 16), (65573, 4)])
def test_shuffle_in_two_parts(fss, n, w):
    """rss_shuffle_prepare's permutations are the oracle's (pi12 and pi31 as
    their inverses, pi23 as is), and rss_shuffle_prepared with them gives the
    oracle's shares, as the one-call shuffle does; preparing twice gives the
    same permutations (a second prepare overwrites the first)."""
    d, sh = _rss_table(3 * n + w, n, w)
    seeds = (505, 606, 707)
    perms = torch.full((3 * n,), -1, dtype=torch.int32, device=DEV)
    fss.rss_shuffle_prepare(n, seeds, perms)
    fss.rss_shuffle_prepare(n, seeds, perms)
    torch.cuda.synchronize()
    got_p = U(perms).reshape(3, n)
    p12, p23, p31 = (osh.permutation(seeds[0], osh.P12, n), osh.permutation(seeds[1], osh.P23, n),
                     osh.permutation(seeds[2], osh.P31, n))
    np.testing.assert_array_equal(got_p[0], np.argsort(p12))
    np.testing.assert_array_equal(got_p[1], np.argsort(p31))
    np.testing.assert_array_equal(got_p[2], p23)
    out = [torch.empty(n * w, dtype=torch.int32, device=DEV) for _ in range(3)]
    fss.rss_shuffle_prepared(n, w, [T(s.ravel()) for s in sh], seeds, perms, out)
    torch.cuda.synchronize()
    want = osh.sec_shuffle(sh, *seeds)
    for i in range(3):
        np.testing.assert_array_equal(U(out[i]).reshape(n, w), want[i])


@pytest.mark.parametrize("method", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("n", [1025, 5000, 65573, (1 << 20) + 100])
def test_permutations_by_every_method(fss, n, method):
    """Every way the library has of making a permutation gives the oracle's:
    the radix pass with exact comparisons in each run (0) or with sorting
    networks in the lanes (1); buckets ordered in LDS with networks (2, the
    default), with exact comparisons in each run (3), or by comparing every
    pair of a bucket (4, the path of a bucket too large for LDS).  Exact
    comparisons are what a network falls back on (two rows of a run sharing
    their leading 25 key bits, runs longer than 128 rows), which random keys
    at these sizes almost never produce, so they are checked on their own."""
    seeds = (11 * n, 12 * n + 1, 13 * n + 2)
    perms = torch.full((3 * n,), -1, dtype=torch.int32, device=DEV)
    fss.set_shuffle_tuning(method)
    try:
        fss.rss_shuffle_prepare(n, seeds, perms)
        torch.cuda.synchronize()
    finally:
        fss.set_shuffle_tuning(2)
    got = U(perms).reshape(3, n)
    p12, p23, p31 = (osh.permutation(seeds[0], osh.P12, n), osh.permutation(seeds[1], osh.P23, n),
                     osh.permutation(seeds[2], osh.P31, n))
    np.testing.assert_array_equal(got[0], np.argsort(p12))
    np.testing.assert_array_equal(got[1], np.argsort(p31))
    np.testing.assert_array_equal(got[2], p23)


@pytest.mark.parametrize("n", [1 << 23, (1 << 23) + 5])
def test_permutations_at_the_bucket_limit(fss, n):
    """The default method at its largest table (2^23 rows: 2048 buckets, 1024
    counting workgroups) and just past it, where the radix method takes over:
    both permutations equal the oracle's."""
    seeds = (n, n + 1, n + 2)
    perms = torch.full((3 * n,), -1, dtype=torch.int32, device=DEV)
    fss.rss_shuffle_prepare(n, seeds, perms)
    torch.cuda.synchronize()
    got = U(perms).reshape(3, n)
    np.testing.assert_array_equal(got[0], np.argsort(osh.permutation(seeds[0], osh.P12, n)))
    np.testing.assert_array_equal(got[1], np.argsort(osh.permutation(seeds[2], osh.P31, n)))
    np.testing.assert_array_equal(got[2], osh.permutation(seeds[1], osh.P23, n))


def test_prepared_skips_out_of_range_entries(fss):
    """Permutation entries outside [0, nrows) leave their rows unwritten and
    are never used as indices: with every entry out of range the outputs keep
    what they held."""
    n, w = 3000, 16
    d, sh = _rss_table(23, n, w)
    perms = torch.full((3 * n,), -1, dtype=torch.int32, device=DEV)     # 0xffffffff
    out = [torch.full((n * w,), 7, dtype=torch.int32, device=DEV) for _ in range(3)]
    fss.rss_shuffle_prepared(n, w, [T(s.ravel()) for s in sh], (1, 2, 3), perms, out)
    torch.cuda.synchronize()
    for o in out:
        assert bool((o == 7).all())


def test_shutdown_between_shuffles(fss):
    """fss_shutdown drains and destroys the shuffle's own streams; the next
    shuffle makes them again and gives the same shares."""
    n, w = 5000, 4
    d, sh = _rss_table(17, n, w)
    seeds = (31, 32, 33)
    outs = []
    for _ in range(2):
        out = [torch.empty(n * w, dtype=torch.int32, device=DEV) for _ in range(3)]
        fss.rss_shuffle(n, w, [T(s.ravel()) for s in sh], seeds, out)
        assert fss.LIB.fss_shutdown() == fss.OK
        torch.cuda.synchronize()
        outs.append([U(o) for o in out])
    want = osh.sec_shuffle(sh, *seeds)
    for got in outs:
        for i in range(3):
            np.testing.assert_array_equal(got[i].reshape(n, w), want[i])


def test_shuffle_full_size_is_a_permutation(fss):
    """At 2^22 records of 64 bytes (the measured size), where the oracle's
    permutations are out of reach: every record comes out whole, each exactly
    once, in an order that is not the input's, and no share alone is the table."""
    n, w = 1 << 22, 16
    g = torch.Generator(device=DEV).manual_seed(5)
    row = torch.arange(n, dtype=torch.int64, device=DEV)
    cols = torch.arange(w, dtype=torch.int64, device=DEV)
    d = (row[:, None] * 0x9E3779B1 + cols[None, :] * 0x85EBCA77) & 0xFFFFFFFF     # word 0: the row number
    d[:, 0] = row
    d32 = (d - (d >= 2**31).to(torch.int64) * 2**32).to(torch.int32)
    del d
    s1 = torch.randint(-2**31, 2**31, (n, w), dtype=torch.int32, device=DEV, generator=g)
    s2 = torch.randint(-2**31, 2**31, (n, w), dtype=torch.int32, device=DEV, generator=g)
    sh = [s1.ravel(), s2.ravel(), (d32 ^ s1 ^ s2).ravel()]
    del s1, s2
    out = [torch.empty(n * w, dtype=torch.int32, device=DEV) for _ in range(3)]
    fss.rss_shuffle(n, w, sh, (41, 42, 43), out)
    rec = (out[0] ^ out[1] ^ out[2]).view(n, w)
    torch.cuda.synchronize()
    ids = rec[:, 0].to(torch.int64) & 0xFFFFFFFF
    assert torch.equal(torch.sort(ids).values, row)
    assert torch.equal(rec, d32[ids])
    assert (ids != row).float().mean().item() > 0.99
    for o in out:
        assert not torch.equal(o.view(n, w), d32)


def test_shuffle_full_size_shares_equal_oracle_at_sampled_rows(fss):
    """At 2^22 records of 64 bytes, all three output shares equal the oracle's
    at 514 sampled rows (the first, the last and 512 at random): R1 and R2 are
    the pairs' ChaCha12 mask words of those rows, and R3 = D[pi(i)] ^ R1 ^ R2
    with pi the oracle's composed permutation (its T masks cancel)."""
    from oracle import chacha
    n, w = 1 << 22, 16
    seeds = (51, 52, 53)
    g = torch.Generator(device=DEV).manual_seed(6)
    sh = [torch.randint(-2**31, 2**31, (n * w,), dtype=torch.int32, device=DEV, generator=g) for _ in range(3)]
    out = [torch.empty(n * w, dtype=torch.int32, device=DEV) for _ in range(3)]
    fss.rss_shuffle(n, w, sh, seeds, out)
    torch.cuda.synchronize()
    rng = np.random.default_rng(10)
    rows = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 512, replace=False)])).astype(np.int64)
    comp = osh.composed_permutation(*seeds, n)
    idx = torch.from_numpy(rows).to(DEV)
    src = torch.from_numpy(comp[rows].astype(np.int64)).to(DEV)
    d_at = U(sh[0].view(n, w)[src] ^ sh[1].view(n, w)[src] ^ sh[2].view(n, w)[src])

    def masks(seed, table):
        r = rows.astype(np.uint64)
        blk = osh._slices(chacha.blocks(osh.pair_key(seed), r, np.zeros_like(r), table, w, osh.ROUNDS))
        return blk.reshape(len(rows), 16)[:, :w]

    r1, r2 = masks(seeds[2], osh.R1), masks(seeds[0], osh.R2)
    got = [U(o.view(n, w)[idx]) for o in out]
    np.testing.assert_array_equal(got[0], r1)
    np.testing.assert_array_equal(got[1], r2)
    np.testing.assert_array_equal(got[2], d_at ^ r1 ^ r2)


def test_fetch_many_full_size(fss):
    """secFetch Case II at the measured size (2^22 records: the bit word and 15
    words, about half kept): the count is the number of set bits, the kept
    records are exactly those rows' records (word 1 carries the row number)
    in increasing shuffled position, and at 256 sampled kept records the three
    shares equal the oracle's shuffle output at that position (R1, R2 from the
    pairs' masks, R3 = D[pi(i)] ^ R1 ^ R2)."""
    from oracle import chacha
    n, w = 1 << 22, 16
    seeds = (61, 62, 63)
    g = torch.Generator(device=DEV).manual_seed(7)
    row = torch.arange(n, dtype=torch.int32, device=DEV)
    d = torch.randint(-2**31, 2**31, (n, w), dtype=torch.int32, device=DEV, generator=g)
    d[:, 0] &= 1                                          # the predicate bit
    d[:, 1] = row
    s1 = torch.randint(-2**31, 2**31, (n, w), dtype=torch.int32, device=DEV, generator=g)
    s2 = torch.randint(-2**31, 2**31, (n, w), dtype=torch.int32, device=DEV, generator=g)
    sh = [s1.ravel(), s2.ravel(), (d ^ s1 ^ s2).ravel()]
    out = [torch.empty(n * (w - 1), dtype=torch.int32, device=DEV) for _ in range(3)]
    pos = torch.full((n,), -1, dtype=torch.int32, device=DEV)
    cnt = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    fss.rss_fetch_many(n, w, sh, seeds, out, pos, cnt)
    torch.cuda.synchronize()
    k = int(cnt.item())
    bits = d[:, 0].cpu().numpy()
    assert k == int(bits.sum())
    got_pos = U(pos)[:k].astype(np.int64)
    assert np.all(np.diff(got_pos) > 0)
    rec = (out[0][:k * (w - 1)] ^ out[1][:k * (w - 1)] ^ out[2][:k * (w - 1)]).view(k, w - 1)
    ids = rec[:, 0].cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(np.sort(ids), np.flatnonzero(bits == 1))
    assert torch.equal(rec, d[torch.from_numpy(ids).to(DEV), 1:])
    # the shares of sampled kept records against the oracle's shuffle output
    comp = osh.composed_permutation(*seeds, n)
    rng = np.random.default_rng(11)
    ks = np.sort(rng.choice(k, 256, replace=False))
    at = got_pos[ks]

    def masks(seed, table):
        r = at.astype(np.uint64)
        blk = osh._slices(chacha.blocks(osh.pair_key(seed), r, np.zeros_like(r), table, w, osh.ROUNDS))
        return blk.reshape(len(at), 16)[:, :w]

    r1, r2 = masks(seeds[2], osh.R1), masks(seeds[0], osh.R2)
    src = torch.from_numpy(comp[at].astype(np.int64)).to(DEV)
    r3 = U(d[src]) ^ r1 ^ r2
    kidx = torch.from_numpy(ks.astype(np.int64)).to(DEV)
    got = [U(o.view(-1, w - 1)[:k][kidx]) for o in out]
    for j, want in enumerate((r1, r2, r3)):
        np.testing.assert_array_equal(got[j], want[:, 1:], err_msg=f"share {j + 1}")


@pytest.mark.parametrize("n,w", [(1000, 8), (513, 4)])
def test_shuffle_unaligned_buffers(fss, n, w):
    """Inputs and outputs 4 bytes past a 16-byte boundary: the gathers and the
    mask tables written into the outputs take the word-by-word path."""
    d, sh = _rss_table(n * w + 5, n, w)
    seeds = (11, 22, 33)
    out = [empty_off(n * w) for _ in range(3)]
    fss.rss_shuffle(n, w, [T_off(s.ravel()) for s in sh], seeds, out)
    torch.cuda.synchronize()
    want = osh.sec_shuffle(sh, *seeds)
    for i in range(3):
        np.testing.assert_array_equal(U(out[i]).reshape(n, w), want[i])


def test_fetch_unique(fss):
    n, w = 5000, 4
    rng = np.random.default_rng(7)
    d, rows = _rss_table(9, n, w)
    x = np.zeros(n, np.uint8)
    x[4321] = 1
    xs1 = rng.integers(0, 2, n, dtype=np.uint8)
    xs2 = rng.integers(0, 2, n, dtype=np.uint8)
    xsh = [xs1, xs2, x ^ xs1 ^ xs2]
    out = [torch.full((w,), 7, dtype=torch.int32, device=DEV) for _ in range(3)]
    fss.rss_fetch_unique(n, w, [T(ofss.pack_bits(v)) for v in xsh], [T(r.ravel()) for r in rows], out)
    want = osh.fetch_case1(xsh, rows)
    got = [U(o) for o in out]
    for i in range(3):
        np.testing.assert_array_equal(got[i], want[i])
    np.testing.assert_array_equal(got[0] ^ got[1] ^ got[2], d[4321])


@pytest.mark.parametrize("n,w", [(1, 2), (1000, 5), (1024, 3), (1025, 3), (4000, 3), (200003, 4)])
def test_fetch_many(fss, n, w):
    """Case II against the oracle: the kept positions, the three shares of the
    kept records, their number (written over whatever the count held) and
    their reconstruction.  Up to 1024 records the open, scan and compaction
    run in one workgroup; 200003 records put them over many workgroups."""
    rng = np.random.default_rng(11 + n)
    d, rows = _rss_table(13 + n, n, w)
    x = (rng.random(n) < 0.1).astype(np.uint8)
    xs1 = rng.integers(0, 2, n, dtype=np.uint8)
    xs2 = rng.integers(0, 2, n, dtype=np.uint8)
    xsh = [xs1, xs2, x ^ xs1 ^ xs2]
    table = [np.concatenate([xsh[i].astype(np.uint32)[:, None], rows[i]], axis=1) for i in range(3)]
    seeds = (5, 6, 7)
    out = [torch.empty(n * w, dtype=torch.int32, device=DEV) for _ in range(3)]
    pos = torch.empty(n, dtype=torch.int32, device=DEV)
    cnt = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    fss.rss_fetch_many(n, w + 1, [T(t.ravel()) for t in table], seeds, out, pos, cnt)
    torch.cuda.synchronize()
    k = int(cnt.item())
    keep, want = osh.fetch_case2(xsh, rows, *seeds)
    assert k == keep.size == x.sum()
    np.testing.assert_array_equal(U(pos)[:k], keep)
    got = [U(o)[:k * w].reshape(k, w) for o in out]
    for i in range(3):
        np.testing.assert_array_equal(got[i], want[i])
    rec = got[0] ^ got[1] ^ got[2]
    assert sorted(map(tuple, rec.tolist())) == sorted(map(tuple, d[x == 1].tolist()))


@pytest.mark.parametrize("n,w", [(1, 3), (999, 2), (1024, 70), (3001, 7), (5003, 20), (70001, 16), (131075, 4)])
def test_compact_valid(fss, n, w):
    """The secAccess filter against the oracle: records whose bits XOR to 1 are
    kept in shuffled order (every third record an all-zero dummy), with their
    shuffled positions, count and shares."""
    from oracle import access
    rng = np.random.default_rng(n)
    recs = rng.integers(0, 2**32, (n, w), dtype=np.uint64).astype(np.uint32)
    recs[::3] = 0
    s1 = rng.integers(0, 2**32, (n, w), dtype=np.uint64).astype(np.uint32)
    s2 = rng.integers(0, 2**32, (n, w), dtype=np.uint64).astype(np.uint32)
    sh = [s1, s2, recs ^ s1 ^ s2]
    seeds = (71, 72, 73)
    out = [torch.empty(n * w, dtype=torch.int32, device=DEV) for _ in range(3)]
    pos = torch.empty(n, dtype=torch.int32, device=DEV)
    cnt = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    fss.rss_compact_valid(n, w, [T(t.ravel()) for t in sh], seeds, out, pos, cnt)
    torch.cuda.synchronize()
    k = int(cnt.item())
    keep, want = access.compact_valid(sh, seeds)
    assert k == keep.size
    np.testing.assert_array_equal(U(pos)[:k], keep)
    got = [U(o)[:k * w].reshape(k, w) for o in out]
    for i in range(3):
        np.testing.assert_array_equal(got[i], want[i])
    par = np.bitwise_xor.reduce(recs, axis=1)
    odd = np.array([bin(int(v)).count("1") & 1 for v in par], bool)
    rec = got[0] ^ got[1] ^ got[2]
    assert k == int(odd.sum())
    assert sorted(map(tuple, rec.tolist())) == sorted(map(tuple, recs[odd].tolist()))


def test_sec_access_composed(fss):
    """Alg. 6 composed from the library calls (selection product + re-share,
    shuffled parity filter, attribute selection + re-share) equals the oracle
    share for share, and reconstructs to the plaintext neighbours."""
    from oracle import access
    rng = np.random.default_rng(21)
    c_count, x_count, wd = 40, 100, 2
    adj = [sorted(rng.choice(x_count, rng.integers(0, 9), replace=False).tolist()) for _ in range(c_count)]
    attr = rng.integers(0, 2**32, (x_count, wd), dtype=np.uint64).astype(np.uint32)
    post, lmax = access.encode_posting_lists(adj, x_count, 5)
    wx = post.shape[2]
    post_sh = access.rss_split(post, 6)
    attr_sh = access.rss_split(attr, 7)
    prf, m = [3, 4, 5], 17
    seeds = (10, 20, 30)
    idm = np.zeros(c_count, np.uint8)
    idm[m] = 1
    s1 = rng.integers(0, 2, c_count, dtype=np.uint8)
    s2 = rng.integers(0, 2, c_count, dtype=np.uint8)
    idm_sh = [s1, s2, idm ^ s1 ^ s2]
    want_ids, want_attrs = access.sec_access(idm_sh, post_sh, attr_sh, x_count, prf, seeds)
    # 1. posting list of the matched vertex: selection product, then re-share
    rec_words = lmax * wx
    add = [torch.empty(rec_words, dtype=torch.int32, device=DEV) for _ in range(3)]
    fss.rss_fetch_unique(c_count, rec_words, [T(ofss.pack_bits(v)) for v in idm_sh],
                         [T(p.reshape(c_count, rec_words).ravel()) for p in post_sh], add)
    pm = [torch.empty(rec_words, dtype=torch.int32, device=DEV) for _ in range(3)]
    fss.rss_reshare(32 * rec_words, add, prf, 0, pm)
    # 2. shuffled parity filter
    ids = [torch.empty(rec_words, dtype=torch.int32, device=DEV) for _ in range(3)]
    pos = torch.empty(lmax, dtype=torch.int32, device=DEV)
    cnt = torch.zeros(1, dtype=torch.int32, device=DEV)
    fss.rss_compact_valid(lmax, wx, pm, seeds, ids, pos, cnt)
    torch.cuda.synchronize()
    k = int(cnt.item())
    assert k == len(adj[m]) == want_ids[0].shape[0]
    got_ids = [U(t)[:k * wx].reshape(k, wx) for t in ids]
    for i in range(3):
        np.testing.assert_array_equal(got_ids[i], want_ids[i])
    # 3. attributes of each kept neighbour
    for j in range(k):
        a = [torch.empty(wd, dtype=torch.int32, device=DEV) for _ in range(3)]
        fss.rss_fetch_unique(x_count, wd, [T(got_ids[i][j]) for i in range(3)], [T(s.ravel()) for s in attr_sh], a)
        d = [torch.empty(wd, dtype=torch.int32, device=DEV) for _ in range(3)]
        fss.rss_reshare(32 * wd, a, prf, 1 + j, d)
        for i in range(3):
            np.testing.assert_array_equal(U(d[i]), want_attrs[i][j])
    rec = got_ids[0] ^ got_ids[1] ^ got_ids[2]
    assert sorted(int(access.unpack_onehot(r, x_count)[0]) for r in rec) == adj[m]


@pytest.mark.parametrize("ncand,wi,wv", [(1, 1, 1), (37, 3, 2), (5000, 2, 0), (1025, 0, 4)])
def test_fetch_table(fss, ncand, wi, wv):
    """secFetch's table {x || id || d}: the predicate bit in bit 0 of word 0,
    then the id and value records, for each share."""
    rng = np.random.default_rng(ncand + wi)
    bits = [rng.integers(0, 2, ncand, dtype=np.uint8) for _ in range(3)]
    ids = [rng.integers(0, 2**32, (ncand, wi), dtype=np.uint64).astype(np.uint32) for _ in range(3)]
    vals = [rng.integers(0, 2**32, (ncand, wv), dtype=np.uint64).astype(np.uint32) for _ in range(3)]
    out = [torch.full((ncand * (1 + wi + wv),), -1, dtype=torch.int32, device=DEV) for _ in range(3)]
    fss.rss_fetch_table(ncand, [T(ofss.pack_bits(b)) for b in bits], wi, [T(x.ravel()) for x in ids] if wi else None,
                        wv, [T(x.ravel()) for x in vals] if wv else None, out)
    for j in range(3):
        want = np.concatenate([bits[j].astype(np.uint32)[:, None], ids[j], vals[j]], axis=1)
        np.testing.assert_array_equal(U(out[j]).reshape(ncand, 1 + wi + wv), want)
