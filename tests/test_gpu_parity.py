"""Parity of the HIP path (through the C ABI) with the CPU oracle: bit-exact
key batches, bit-exact share words, reconstructions equal to the plaintext
functions and to brute-force subgraph matching.  Sizes span several 1024-row
workgroups and ragged tails; edge cases cover empty inputs, one row, empty
ranges and every small domain width the tests pin."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import DEV, B, T, T_off, U, column_shares, empty_off, plan_outputs, run_query_gpu
from keylayout import from_device, to_device
from oracle import fss as ofss
from oracle import match as omatch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_03526_amd import fss as lib
    torch.cuda.set_device(0)
    return lib


def _rand_u32(seed, n):
    return np.random.default_rng(seed).integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)


# --------------------------------------------------------------------------- masked open

@pytest.mark.parametrize("n", [1, 3, 255, 1024, 1000003])
def test_mask_open(fss, n):
    """Aligned buffers take the 16-byte path (with a ragged tail of n mod 4 rows)."""
    x0, x1, r = _rand_u32(1, n), _rand_u32(2, n), _rand_u32(3, n)
    out = torch.empty(n, dtype=torch.int32, device=DEV)
    fss.fss_mask_open(T(x0), T(x1), T(r), out)
    np.testing.assert_array_equal(U(out), ofss.mask_open(x0, x1, r))


@pytest.mark.parametrize("n", [5, 100003])
def test_mask_open_unaligned(fss, n):
    """A buffer 4 bytes past a 16-byte boundary takes the word path."""
    x0, x1, r = _rand_u32(4, n), _rand_u32(5, n), _rand_u32(6, n)
    out = empty_off(n)
    fss.fss_mask_open(T(x0), T_off(x1), T(r), out)
    np.testing.assert_array_equal(U(out), ofss.mask_open(x0, x1, r))


# --------------------------------------------------------------------------- dealer keygen

KG_CASES = [(kind, nbits, n) for kind in (0, 1) for nbits in (8, 12, 32) for n in (1, 65, 1000)] + \
           [(0, 32, 4099), (1, 32, 4099), (0, 20, 2048), (1, 17, 333), (0, 9, 64), (1, 9, 70), (1, 25, 129),
            (0, 31, 100), (1, 31, 100)]


@pytest.mark.parametrize("kind,nbits,n", KG_CASES)
def test_keygen_bit_exact(fss, kind, nbits, n):
    seed, query, pred = 0xC0FFEE + n, 7, 3 + kind
    r = _rand_u32(n + nbits, n)
    if kind == 0:
        a, hi = (n * 2654435761) % (1 << nbits), 0
        k0, k1 = ofss.keygen_eq(nbits, seed, query, pred, a, r)
    else:
        lo = (n * 40503) % (1 << nbits)
        hi = min((1 << nbits) - 1, lo + (1 << (nbits - 2)))
        a = lo
        k0, k1 = ofss.keygen_range(nbits, seed, query, pred, lo, hi, r)
    kb = fss.KeyBatch(kind, nbits, n)
    fss.fss_keygen(seed, query, pred, a, hi, T(r), kb)
    torch.cuda.synchronize()
    nbytes = kb.bytes_per_party
    for b, want in ((0, k0), (1, k1)):
        got = from_device(kind, nbits, n, B(kb.key[b], nbytes))
        assert got.tobytes() == want.tobytes(), f"party {b} keys differ"


# --------------------------------------------------------------------------- eval on oracle keys

@pytest.mark.parametrize("kind,nbits,n", [(0, 32, 3001), (1, 32, 3001), (0, 8, 70), (1, 12, 129), (0, 12, 1),
                                          (1, 32, 64)])
def test_eval_on_oracle_keys(fss, kind, nbits, n):
    seed = 99 + n
    r = _rand_u32(seed, n)
    x = _rand_u32(seed + 1, n) & np.uint32((1 << nbits) - 1 if nbits < 32 else 0xFFFFFFFF)
    if kind == 0:
        a = int(x[n // 2])
        k0, k1 = ofss.keygen_eq(nbits, seed, 1, 1, a, r)
    else:
        a, hi = sorted((int(x[0]), int(x[-1])))
        k0, k1 = ofss.keygen_range(nbits, seed, 1, 1, a, hi, r)
    xhat = (x.astype(np.uint64) + r).astype(np.uint32)
    kb = fss.KeyBatch(kind, nbits, n)
    for b, k in ((0, k0), (1, k1)):
        kb.key[b][:kb.bytes_per_party].copy_(torch.from_numpy(to_device(kind, nbits, k)).to(DEV))
    ev = ofss.eval_eq if kind == 0 else ofss.eval_range
    gpu_eval = fss.fss_eval_eq if kind == 0 else fss.fss_eval_lt
    nw = (n + 31) // 32
    shares = []
    for b, k in ((0, k0), (1, k1)):
        out = torch.full((nw,), -1, dtype=torch.int32, device=DEV)
        gpu_eval(b, kb, T(xhat), out)
        got = U(out)
        want = ofss.pack_bits(ev(nbits, b, k, xhat))
        np.testing.assert_array_equal(got, want)
        shares.append(got)
    recon = ofss.unpack_bits(shares[0] ^ shares[1], n)
    truth = (x == a) if kind == 0 else ((x >= a) & (x < hi))
    np.testing.assert_array_equal(recon, truth.astype(np.uint8))


def _gpu_pred(fss, kind, nbits, a, hi, x, r, seed, pred):
    n = x.size
    kb = fss.KeyBatch(kind, nbits, n)
    rt = T(r)
    fss.fss_keygen(seed, 1, pred, a, hi, rt, kb)
    xhat = (x.astype(np.uint64) + r).astype(np.uint32)
    nw = (n + 31) // 32
    outs = []
    for b in (0, 1):
        o = torch.empty(nw, dtype=torch.int32, device=DEV)
        (fss.fss_eval_eq if kind == 0 else fss.fss_eval_lt)(b, kb, T(xhat), o)
        outs.append(o)
    return [U(o) for o in outs]


def test_dpf_exhaustive_8bit(fss):
    xs = np.arange(256, dtype=np.uint32)
    for alpha in range(256):
        r = _rand_u32(1000 + alpha, 256)
        s0, s1 = _gpu_pred(fss, 0, 8, alpha, 0, xs, r, 5, alpha)
        np.testing.assert_array_equal(ofss.unpack_bits(s0 ^ s1, 256), (xs == alpha).astype(np.uint8))
        if alpha % 37 == 0:
            k0, _ = ofss.keygen_eq(8, 5, 1, alpha, alpha, r)
            np.testing.assert_array_equal(s0, ofss.pack_bits(ofss.eval_eq(8, 0, k0, (xs + r).astype(np.uint32))))


def test_range_8bit(fss):
    xs = np.arange(256, dtype=np.uint32)
    rng = np.random.default_rng(5)
    pairs = [(0, 0), (0, 255), (254, 255), (17, 18), (100, 100)]
    pairs += [tuple(sorted(int(v) for v in rng.integers(0, 256, 2))) for _ in range(120)]
    for i, (lo, hi) in enumerate(pairs):
        r = _rand_u32(2000 + i, 256)
        s0, s1 = _gpu_pred(fss, 1, 8, lo, hi, xs, r, 6, i)
        np.testing.assert_array_equal(ofss.unpack_bits(s0 ^ s1, 256), ((xs >= lo) & (xs < hi)).astype(np.uint8))


def test_12bit_domain(fss):
    xs = np.arange(4096, dtype=np.uint32)
    for i, alpha in enumerate([0, 1, 4095, 2048, 1234, 3000]):
        r = _rand_u32(3000 + i, 4096)
        s0, s1 = _gpu_pred(fss, 0, 12, alpha, 0, xs, r, 7, i)
        np.testing.assert_array_equal(ofss.unpack_bits(s0 ^ s1, 4096), (xs == alpha).astype(np.uint8))
        lo, hi = min(alpha, 4000), 4095
        s0, s1 = _gpu_pred(fss, 1, 12, lo, hi, xs, r, 8, i)
        np.testing.assert_array_equal(ofss.unpack_bits(s0 ^ s1, 4096), ((xs >= lo) & (xs < hi)).astype(np.uint8))


def test_32bit_edges(fss):
    """32-bit domain at its edges: bounds 0 and 2^32 - 1, empty ranges, x at and
    around every bound, masks 0, 2^32 - 1 and random (so L > U wraps occur)."""
    top = 2**32 - 1
    cases = [(0, 0), (0, 1), (0, top), (top - 1, top), (5, 5), (1, 2**31), (2**31, top), (12345, 12346)]
    for i, (lo, hi) in enumerate(cases):
        pts = {0, 1, top - 1, top, 2**31 - 1, 2**31}
        for b in (lo, hi):
            pts |= {(b + d) % 2**32 for d in (-1, 0, 1)}
        x = np.array(sorted(pts), dtype=np.uint32)
        n = x.size
        for j, r in enumerate([np.zeros(n, np.uint32), np.full(n, top, np.uint32), _rand_u32(4000 + i, n)]):
            s0, s1 = _gpu_pred(fss, 1, 32, lo, hi, x, r, 11, 10 * i + j)
            want = ((x >= lo) & (x < hi)).astype(np.uint8)
            np.testing.assert_array_equal(ofss.unpack_bits(s0 ^ s1, n), want, err_msg=f"[{lo},{hi}) r#{j}")
            a = lo
            s0, s1 = _gpu_pred(fss, 0, 32, a, 0, x, r, 12, 10 * i + j)
            np.testing.assert_array_equal(ofss.unpack_bits(s0 ^ s1, n), (x == a).astype(np.uint8),
                                          err_msg=f"a={a} r#{j}")


@pytest.mark.parametrize("nbits", [9, 17, 25, 31])
def test_odd_domain_widths(fss, nbits):
    """Masked equality and range at widths between the workloads' 8, 12 and 32:
    points at and around the bounds and the domain ends, random masks."""
    top = (1 << nbits) - 1
    rng = np.random.default_rng(nbits)
    lo, hi = int(rng.integers(0, top // 2)), int(rng.integers(top // 2, top))
    pts = {0, 1, top - 1, top} | {(b + d) % (1 << nbits) for b in (lo, hi) for d in (-1, 0, 1)}
    pts |= {int(v) for v in rng.integers(0, top + 1, 200, dtype=np.uint64)}
    x = np.array(sorted(pts), dtype=np.uint32)
    r = _rand_u32(5000 + nbits, x.size)
    s0, s1 = _gpu_pred(fss, 1, nbits, lo, hi, x, r, 13, nbits)
    np.testing.assert_array_equal(ofss.unpack_bits(s0 ^ s1, x.size), ((x >= lo) & (x < hi)).astype(np.uint8))
    s0, s1 = _gpu_pred(fss, 0, nbits, lo, 0, x, r, 14, nbits)
    np.testing.assert_array_equal(ofss.unpack_bits(s0 ^ s1, x.size), (x == lo).astype(np.uint8))


def test_small_domain_ignores_high_bits(fss):
    """With nbits < 32 only the low nbits of xhat are evaluated."""
    x = np.arange(256, dtype=np.uint32)
    r = _rand_u32(9, 256)
    s0, s1 = _gpu_pred(fss, 0, 8, 77, 0, x + np.uint32(0x1200), r, 9, 0)
    np.testing.assert_array_equal(ofss.unpack_bits(s0 ^ s1, 256), (x == 77).astype(np.uint8))


# --------------------------------------------------------------------------- Beaver AND

@pytest.mark.parametrize("nrows", [1, 31, 32, 1000, 65537])
def test_triples_and_per_party(fss, nrows):
    nw = (nrows + 31) // 32
    t0 = torch.empty(3 * nw, dtype=torch.int32, device=DEV)
    t1 = torch.empty(3 * nw, dtype=torch.int32, device=DEV)
    fss.ss_triples(77, 5, 9, nw, t0, t1)
    want = ofss.triples(77, 5, 9, nw)
    g0, g1 = U(t0), U(t1)
    np.testing.assert_array_equal(g0, np.concatenate([want["a"][0], want["b"][0], want["c"][0]]))
    np.testing.assert_array_equal(g1, np.concatenate([want["a"][1], want["b"][1], want["c"][1]]))
    vm = ofss.valid_mask(nrows)
    x = [_rand_u32(10 + b, nw) & vm for b in range(2)]
    y = [_rand_u32(20 + b, nw) & vm for b in range(2)]
    msg = []
    for b, t in ((0, t0), (1, t1)):
        o = torch.empty(2 * nw, dtype=torch.int32, device=DEV)
        fss.ss_and(fss.SS_AND_OPEN, b, nrows, T(x[b]), T(y[b]), t, None, o)
        msg.append(U(o))
    de = msg[0] ^ msg[1]
    z = []
    for b, t in ((0, t0), (1, t1)):
        o = torch.empty(nw, dtype=torch.int32, device=DEV)
        fss.ss_and(fss.SS_AND_CLOSE, b, nrows, None, None, t, T(de), o)
        z.append(U(o))
    wz0, wz1 = ofss.beaver_and((x[0], x[1]), (y[0], y[1]), want, nrows)
    np.testing.assert_array_equal(z[0], wz0)
    np.testing.assert_array_equal(z[1], wz1)
    np.testing.assert_array_equal(z[0] ^ z[1], (x[0] ^ x[1]) & (y[0] ^ y[1]))


# --------------------------------------------------------------------------- edge matching

P = synth.Pred
TINY_QUERIES = [
    synth.Query(1, 1, [P(0, "eq", "label", a=2)]),
    synth.Query(2, 1, [P(0, "range", "attr", lo=3, hi=11), P(0, "eq", "label", a=1)]),
    synth.Query(3, 2, [P(0, "range", "attr", lo=0, hi=9), P(2, "eq", "label", a=0)]),
    synth.Query(4, 2, []),
    synth.Query(5, 3, [P(0, "range", "attr", lo=2, hi=14), P(1, "eq", "label", a=1),
                       P(3, "range", "weight", lo=0, hi=12), P(2, "range", "attr", lo=4, hi=16)]),
    synth.Query(6, 3, [P(1, "range", "attr", lo=0, hi=8), P(1, "range", "attr", lo=4, hi=16),
                       P(4, "eq", "label", a=3), P(3, "eq", "label", a=1), P(4, "range", "weight", lo=5, hi=15)]),
    synth.Query(7, 4, [P(0, "eq", "label", a=1), P(3, "range", "attr", lo=0, hi=12),
                       P(5, "range", "weight", lo=0, hi=14)]),
]


@pytest.mark.parametrize("gseed", [0, 1])
@pytest.mark.parametrize("qi", range(len(TINY_QUERIES)))
def test_match_tiny(fss, gseed, qi):
    q = TINY_QUERIES[qi]
    g = synth.tiny_graph(gseed, n_vertices=10 if q.n_qv == 4 else 12, n_edges=30)
    seed = 500 + 10 * gseed + qi
    shares = column_shares(g, seed)
    masks = synth.pred_masks(seed, q, g)
    plan = run_query_gpu(fss, g, q, shares, masks, seed)
    got = plan_outputs(plan, q, g)
    want = omatch.run_plan(32, seed, g, q, shares, masks)
    for j, (gw, ww) in enumerate(zip(got, want)):
        np.testing.assert_array_equal(gw[0], ww[0], err_msg=f"output {j} party 0")
        np.testing.assert_array_equal(gw[1], ww[1], err_msg=f"output {j} party 1")
    nrows = g.n_vertices if q.n_qv == 1 else g.n_edges
    assert omatch.results_from_bits(g, q, omatch.reconstruct(got, nrows)) == omatch.brute_force(g, q)


def test_match_er_1024(fss):
    g, q = synth.config1(1)
    seed = 4242
    shares = column_shares(g, seed)
    masks = synth.pred_masks(seed, q, g)
    plan = run_query_gpu(fss, g, q, shares, masks, seed)
    got = plan_outputs(plan, q, g)
    want = omatch.run_plan(32, seed, g, q, shares, masks)
    np.testing.assert_array_equal(got[0][0], want[0][0])
    np.testing.assert_array_equal(got[0][1], want[0][1])
    res = omatch.results_from_bits(g, q, omatch.reconstruct(got, g.n_edges))
    assert res == omatch.brute_force_pairs(g, q) and len(res) > 0


def test_match_many_predicates(fss):
    """More predicate-party evaluations than one launch carries (12 predicates
    on a 3-vertex path: 24 evaluations): shares equal the oracle's, and the
    reconstruction equals brute force."""
    g = synth.tiny_graph(8, n_vertices=40, n_edges=400, label_range=3, attr_range=64)
    preds = []
    for k in range(12):
        t = k % 5                      # vertices 0..2 and both query edges; predicates on one
        if t < 3:                      # target agree (same label, overlapping ranges)
            preds.append(synth.Pred(t, "range", "attr", lo=k // 3, hi=60 - k) if k >= 5 else
                         synth.Pred(t, "eq", "label", a=t % 3))
        else:
            preds.append(synth.Pred(t, "range", "weight", lo=k // 4, hi=62 - k) if k >= 5 else
                         synth.Pred(t, "eq", "label", a=t % 2))
    q = synth.Query(77, 3, preds)
    seed = 99
    shares = column_shares(g, seed)
    masks = synth.pred_masks(seed, q, g)
    plan = run_query_gpu(fss, g, q, shares, masks, seed)
    got = plan_outputs(plan, q, g)
    want = omatch.run_plan(32, seed, g, q, shares, masks)
    for j in range(q.n_qv - 1):
        for b in range(2):
            np.testing.assert_array_equal(got[j][b], want[j][b])
    res = omatch.results_from_bits(g, q, omatch.reconstruct(got, g.n_edges))
    assert res == omatch.brute_force(g, q) and len(res) > 0


def test_match_rejects_bad_plans(fss):
    g, q = synth.config1(1)
    kb = fss.KeyBatch(fss.EQ, 32, g.n_vertices)
    xhat = torch.zeros(g.n_vertices, dtype=torch.int32, device=DEV)
    plan = fss.Plan(1, 1, 2, g.n_vertices, g.n_edges, [(5, kb, xhat)], T(g.src), T(g.dst)).allocate()
    with pytest.raises(fss.FssError) as e:
        fss.match_query(plan)
    assert e.value.code == fss.EINVAL
    plan = fss.Plan(1, 1, 2, g.n_vertices, g.n_edges, [(2, kb, xhat)], T(g.src), T(g.dst)).allocate()
    with pytest.raises(fss.FssError):      # edge predicate with vertex-sized keys
        fss.match_query(plan)
    plan = fss.Plan(1, 1, 1, g.n_vertices, 0, [(0, kb, xhat)]).allocate()
    with pytest.raises(fss.FssError) as e:
        fss.match_query(plan, party_mask=4)
    assert e.value.code == fss.EINVAL


def test_empty_inputs_are_noops(fss):
    kb = fss.KeyBatch(fss.RANGE, 32, 0)
    fss.fss_keygen(1, 1, 1, 0, 5, torch.zeros(1, dtype=torch.int32, device=DEV), kb)
    fss.fss_eval_lt(0, kb, torch.zeros(1, dtype=torch.int32, device=DEV), torch.zeros(1, dtype=torch.int32, device=DEV))
    torch.cuda.synchronize()


@pytest.mark.parametrize("n,off", [(1, 0), (1000, 0), (70001, 12345)])
def test_dealer_masks(fss, n, off):
    out = torch.empty(n, dtype=torch.int32, device=DEV)
    fss.fss_dealer_masks(31337, 8, 2, n, out, row_offset=off)
    np.testing.assert_array_equal(U(out), ofss.masks(31337, 8, 2, n, row_offset=off))
