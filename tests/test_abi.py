"""CPU-side checks of the C ABI: the built library loads, exports every
function include/oblivgm_fss.h declares, reports the documented key sizes and
rejects bad arguments on the host before any kernel is enqueued."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oblivgm_fss.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\**\s+\**([a-z_0-9]+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def fss():
    from paper_2209_03526_amd import fss as lib
    return lib


def test_every_declared_symbol_is_exported(fss):
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(fss.LIB, name), name
        assert name in fss.EXPORTS, name


def test_key_sizes(fss):
    assert fss.fss_key_bytes(fss.EQ, 32) == 432
    assert fss.fss_key_bytes(fss.RANGE, 32) == 872
    assert fss.fss_key_bytes(fss.EQ, 8) == 16 * (8 - 5)
    assert fss.fss_key_bytes(fss.RANGE, 12) == 2 * (16 * (12 - 5) + 4)
    assert fss.fss_key_bytes(fss.EQ, 7) == 0 and fss.fss_key_bytes(fss.RANGE, 33) == 0
    assert fss.fss_key_bytes(5, 32) == 0
    assert fss.fss_keybatch_bytes(fss.RANGE, 32, 65) == 872 * 128
    assert fss.fss_keybatch_bytes(fss.EQ, 32, 0) == 0


def _kb(fss, kind, nbits, n, p0=256, p1=512):
    return fss.fss_keybatch(kind, nbits, n, (ctypes.c_void_p * 2)(p0, p1))


def test_keygen_argument_errors(fss):
    L = fss.LIB
    r = ctypes.c_void_p(4096)
    assert L.fss_keygen(1, 1, 1, 9, 3, r, ctypes.byref(_kb(fss, fss.RANGE, 32, 10)), None) == fss.EINVAL
    assert b"lo" in L.fss_last_error()
    assert L.fss_keygen(1, 1, 1, 0, 256, r, ctypes.byref(_kb(fss, fss.RANGE, 8, 10)), None) == fss.EINVAL
    assert L.fss_keygen(1, 1, 1, 300, 0, r, ctypes.byref(_kb(fss, fss.EQ, 8, 10)), None) == fss.EINVAL
    assert L.fss_keygen(1, 1, 1, 0, 0, r, ctypes.byref(_kb(fss, fss.EQ, 40, 10)), None) == fss.EINVAL
    assert L.fss_keygen(1, 1, 1, 0, 0, r, ctypes.byref(_kb(fss, 3, 32, 10)), None) == fss.EINVAL
    assert L.fss_keygen(1, 1, 1, 0, 0, None, ctypes.byref(_kb(fss, fss.EQ, 32, 10)), None) == fss.EINVAL
    assert L.fss_keygen(1, 1, 1, 0, 0, r, ctypes.byref(_kb(fss, fss.EQ, 32, 10, 256, 300)), None) == fss.EINVAL
    assert b"aligned" in L.fss_last_error()
    assert L.fss_keygen(1, 1, 1, 0, 0, r, None, None) == fss.EINVAL
    assert L.fss_keygen(1, 1, 1, 0, 0, r, ctypes.byref(_kb(fss, fss.EQ, 32, 2**33)), None) == fss.EUNSUPPORTED


def test_eval_and_argument_errors(fss):
    L = fss.LIB
    kb = _kb(fss, fss.EQ, 32, 10)
    buf = ctypes.c_void_p(4096)
    assert L.fss_eval_eq(2, ctypes.byref(kb), buf, buf, None) == fss.EINVAL
    assert L.fss_eval_lt(0, ctypes.byref(kb), buf, buf, None) == fss.EINVAL      # kind mismatch
    assert L.fss_eval_eq(0, None, buf, buf, None) == fss.EINVAL
    assert L.fss_eval_eq(0, ctypes.byref(kb), None, buf, None) == fss.EINVAL
    assert L.ss_and(7, 0, 64, buf, buf, buf, buf, buf, None) == fss.EINVAL
    assert L.ss_and(0, 3, 64, buf, buf, buf, buf, buf, None) == fss.EINVAL
    assert L.ss_and(1, 0, 64, None, None, buf, None, buf, None) == fss.EINVAL
    assert L.ss_triples(1, 1, 1, 10, None, buf, None) == fss.EINVAL
    assert L.fss_mask_open(5, None, buf, buf, buf, None) == fss.EINVAL
    # zero-sized work is a no-op that touches nothing
    assert L.fss_mask_open(0, None, None, None, None, None) == fss.OK
    assert L.ss_triples(1, 1, 1, 0, None, None, None) == fss.OK


def test_match_plan_validation(fss):
    L = fss.LIB
    plan = fss.match_plan()
    plan.n_qv = 0
    assert L.match_query(ctypes.byref(plan), 3, None) == fss.EINVAL
    plan.n_qv = 9
    assert L.match_query(ctypes.byref(plan), 3, None) == fss.EINVAL
    plan.n_qv = 1
    assert L.match_query(ctypes.byref(plan), 0, None) == fss.EINVAL     # party_mask outside 1..3
    assert L.match_query(ctypes.byref(plan), 4, None) == fss.EINVAL
    assert L.match_query(ctypes.byref(plan), 3, None) == fss.EINVAL     # no outputs
    plan.d_out[0] = 256
    plan.d_out[1] = 512
    plan.n_vertices = 100
    assert L.match_query(ctypes.byref(plan), 3, None) == fss.ENOMEM     # no workspace
    assert L.match_workspace_bytes(ctypes.byref(plan)) > 0
    plan.n_qv = 2
    plan.n_edges = 10
    assert L.match_query(ctypes.byref(plan), 3, None) == fss.EINVAL     # no endpoints


def _two_vertex_plan(fss, keep):
    """Query vertex 0 with two predicates (share bits given: fake, aligned,
    never dereferenced), vertex 1 and the edge without: one AND, then a hop
    whose result is the gathered bits of m_0."""
    preds = (fss.fss_pred * 2)()
    for k in range(2):
        preds[k] = fss.fss_pred(0, 0, None, None, (ctypes.c_void_p * 2)(1 << 20, 1 << 21))
    plan = fss.match_plan()
    plan.n_qv, plan.n_pred = 2, 2
    plan.preds = ctypes.cast(preds, ctypes.POINTER(fss.fss_pred))
    plan.n_vertices, plan.n_edges = 100, 50
    plan.d_src, plan.d_dst = 1 << 22, 1 << 23
    plan.d_out[0], plan.d_out[1] = 1 << 24, 1 << 25
    plan.d_workspace = 1 << 26
    plan.workspace_bytes = fss.LIB.match_workspace_bytes(ctypes.byref(plan))
    keep.append(preds)
    return plan


def test_match_single_party_arguments(fss):
    """Single-party (party_mask 1 / 2) rounds: schedule and argument errors,
    all caught before anything is enqueued."""
    L = fss.LIB
    keep = []
    plan = _two_vertex_plan(fss, keep)
    assert plan.workspace_bytes > 0
    n = ctypes.c_uint32()
    words = (ctypes.c_uint64 * 4)()
    assert L.match_rounds(ctypes.byref(plan), ctypes.byref(n), words, 4) == fss.OK
    assert n.value == 1 and words[0] == 2 * ((100 + 31) // 32)     # one AND over 100 vertex rows: d || e
    assert L.match_rounds(ctypes.byref(plan), None, None, 0) == fss.EINVAL
    assert L.match_rounds(None, ctypes.byref(n), None, 0) == fss.EINVAL
    plan.round = 2
    assert L.match_query(ctypes.byref(plan), 1, None) == fss.EINVAL and b"round" in L.fss_last_error()
    plan.round, plan.d_peer_msg, plan.d_msg = 1, None, None
    assert L.match_query(ctypes.byref(plan), 2, None) == fss.EINVAL and b"peer" in L.fss_last_error()
    plan.round = 0
    assert L.match_query(ctypes.byref(plan), 1, None) == fss.EINVAL and b"d_msg" in L.fss_last_error()
    # one party's bits missing
    keep[0][1].d_bits[1] = None
    assert L.match_query(ctypes.byref(plan), 2, None) == fss.EINVAL and b"bits of party 1" in L.fss_last_error()
    assert L.match_query(ctypes.byref(plan), 3, None) == fss.EINVAL


def test_eval_all_batch_argument_errors(fss):
    kb = _kb(fss, fss.RANGE, 12, 3)
    req = fss.fss_eval_all_req(0, 0, ctypes.pointer(kb), 1, 4096, 4096)
    assert fss.LIB.fss_eval_all_batch(None, 1, None) == fss.EINVAL
    assert fss.LIB.fss_eval_all_batch(ctypes.byref(req), 0, None) == fss.OK
    bad = fss.fss_eval_all_req(2, 0, ctypes.pointer(kb), 1, 4096, 4096)
    assert fss.LIB.fss_eval_all_batch(ctypes.byref(bad), 1, None) == fss.EINVAL and b"party" in fss.LIB.fss_last_error()
    bad = fss.fss_eval_all_req(0, 0, ctypes.pointer(kb), 3, 4096, 4096)
    assert fss.LIB.fss_eval_all_batch(ctypes.byref(bad), 1, None) == fss.EINVAL and b"row" in fss.LIB.fss_last_error()
    bad = fss.fss_eval_all_req(0, 0, ctypes.pointer(kb), 0, 4097, 4096)
    assert fss.LIB.fss_eval_all_batch(ctypes.byref(bad), 1, None) == fss.EINVAL and b"points" in fss.LIB.fss_last_error()


def test_triples_counter_limit(fss):
    """The Beaver stream's 32-bit block counter bounds the triple words."""
    p = ctypes.c_void_p(4096)
    assert fss.LIB.ss_triples(1, 1, 0, (1 << 32) // 5 * 4 + 4, p, p, None) == fss.EUNSUPPORTED
    assert b"too many" in fss.LIB.fss_last_error()


def test_shuffle_and_fetch_argument_errors(fss):
    """The shuffle and fetch calls reject sizes beyond their limits and NULL
    arguments on the host, before any workspace sizing or launch."""
    L = fss.LIB
    fake = ctypes.c_void_p(1 << 20)                         # never dereferenced: rejected first
    three = (ctypes.c_void_p * 3)(fake, fake, fake)
    seeds = (ctypes.c_uint64 * 3)(1, 2, 3)
    # empty work is a no-op
    assert L.rss_shuffle(0, 4, three, seeds, three, None, 0, None) == fss.OK
    # row indices are 31-bit
    assert L.rss_shuffle(1 << 31, 4, three, seeds, three, fake, 1 << 40, None) == fss.EUNSUPPORTED
    assert b"2^31" in fss.LIB.fss_last_error()
    assert L.rss_fetch_many(1 << 31, 4, three, seeds, three, fake, fake, fake, 1 << 40, None) == fss.EUNSUPPORTED
    assert L.rss_compact_valid(1 << 31, 4, three, seeds, three, fake, fake, fake, 1 << 40, None) == fss.EUNSUPPORTED
    # NULL shares, tables and outputs
    assert L.rss_shuffle(8, 4, None, seeds, three, fake, 1 << 40, None) == fss.EINVAL
    null_one = (ctypes.c_void_p * 3)(fake, None, fake)
    assert L.rss_shuffle(8, 4, null_one, seeds, three, fake, 1 << 40, None) == fss.EINVAL
    assert L.rss_fetch_many(8, 4, three, seeds, null_one, fake, fake, fake, 1 << 40, None) == fss.EINVAL
    assert L.rss_compact_valid(8, 4, three, seeds, three, None, fake, fake, 1 << 40, None) == fss.EINVAL
    # Case II needs the bit word and at least one more word per record
    assert L.rss_fetch_many(8, 1, three, seeds, three, fake, fake, fake, 1 << 40, None) == fss.EINVAL
    assert L.rss_compact_valid(8, 0, three, seeds, three, fake, fake, fake, 1 << 40, None) == fss.EINVAL
    # the two-part shuffle: the same limits, NULL checks, and a short workspace
    # for the data-dependent part (its size needs no device query)
    assert L.rss_shuffle_prepare(0, seeds, None, None, 0, None) == fss.OK
    assert L.rss_shuffle_prepare(1 << 31, seeds, fake, fake, 1 << 40, None) == fss.EUNSUPPORTED
    assert L.rss_shuffle_prepare(8, seeds, None, fake, 1 << 40, None) == fss.EINVAL
    assert L.rss_shuffle_prepare(8, None, fake, fake, 1 << 40, None) == fss.EINVAL
    assert L.rss_shuffle_prepared(0, 4, three, seeds, fake, three, None, 0, None) == fss.OK
    assert L.rss_shuffle_prepared(1 << 31, 4, three, seeds, fake, three, fake, 1 << 40, None) == fss.EUNSUPPORTED
    assert L.rss_shuffle_prepared(8, 4, three, seeds, None, three, fake, 1 << 40, None) == fss.EINVAL
    assert L.rss_shuffle_prepared(8, 4, null_one, seeds, fake, three, fake, 1 << 40, None) == fss.EINVAL
    assert L.rss_shuffle_prepared_workspace_bytes(8, 4) == 2 * 256 + 4096
    assert L.rss_shuffle_prepared(8, 4, three, seeds, fake, three, fake, 2 * 256 + 4095, None) == fss.ENOMEM
    assert L.rss_shuffle_prepared(8, 4, three, seeds, fake, three, None, 1 << 40, None) == fss.ENOMEM
    # Case I words per record
    assert L.rss_fetch_unique(8, 65536, three, three, three, None) == fss.EUNSUPPORTED
    assert L.rss_fetch_unique(8, 4, None, three, three, None) == fss.EINVAL


def test_access_and_conversion_argument_errors(fss):
    """The Alg. 1 / Alg. 6 calls and the two-party conversion reject bad
    arguments on the host, before anything is enqueued."""
    L = fss.LIB
    fake = 1 << 20
    three = (ctypes.c_void_p * 3)(fake, fake, fake)
    two = (ctypes.c_void_p * 2)(fake, fake)
    keys3 = (ctypes.c_uint64 * 3)(1, 2, 3)
    keys2 = (ctypes.c_uint64 * 2)(1, 2)
    # rss_from_fss
    assert L.rss_from_fss(64, None, keys3, 0, three, None) == fss.EINVAL
    assert L.rss_from_fss(64, two, keys3, 0, (ctypes.c_void_p * 3)(fake, None, fake), None) == fss.EINVAL
    assert L.rss_from_fss(0, None, None, 0, None, None) == fss.OK           # nothing to do
    # rss_enc_posting_lists
    assert L.rss_enc_posting_lists(4, 0, fake, fake, fake, fake, 8, keys2, 0, three, fake, 1 << 20, None) == fss.EINVAL
    assert L.rss_enc_posting_lists(4, 64, None, fake, fake, fake, 8, keys2, 0, three, fake, 1 << 20, None) == fss.EINVAL
    assert L.rss_enc_posting_lists(4, 64, fake, fake, fake, fake, 8, keys2, 0, three, fake, 16, None) == fss.ENOMEM
    # rss_sec_access
    ws = L.rss_sec_access_workspace_bytes(24, 2000, 2)
    assert ws > 0
    args = dict(ncand=100, x_bits=2000, idm=three, off=fake, lmax=24, post=three, aw=2, attr=three, keys=keys3,
                counter=0, seeds=keys3, ids=three, attrs=three, rows=fake, count=fake, work=fake, wbytes=ws)

    def call(**kw):
        a = dict(args, **kw)
        return L.rss_sec_access(a["ncand"], a["x_bits"], a["idm"], a["off"], a["lmax"], a["post"], a["aw"],
                                a["attr"], a["keys"], a["counter"], a["seeds"], a["ids"], a["attrs"], a["rows"],
                                a["count"], a["work"], a["wbytes"], None)

    assert call(lmax=0) == fss.EINVAL and b"lmax" in L.fss_last_error()
    assert call(lmax=70000) == fss.EINVAL
    assert call(x_bits=0) == fss.EINVAL
    assert call(off=None) == fss.EINVAL
    assert call(attrs=(ctypes.c_void_p * 3)(fake, fake, None)) == fss.EINVAL
    assert call(wbytes=ws - 1) == fss.ENOMEM


def _star_plan(fss, keep, edges):
    """Three query vertices: two predicates on vertex 0, one on each of 1 and 2
    (share bits given: fake, aligned, never dereferenced); query edges as
    given (None: the path)."""
    preds = (fss.fss_pred * 4)()
    for k, t in enumerate((0, 0, 1, 2)):
        preds[k] = fss.fss_pred(t, 0, None, None, (ctypes.c_void_p * 2)(1 << 20, 1 << 21))
    plan = fss.match_plan()
    plan.n_qv, plan.n_pred = 3, 4
    plan.preds = ctypes.cast(preds, ctypes.POINTER(fss.fss_pred))
    plan.n_vertices, plan.n_edges = 100, 50
    plan.d_src, plan.d_dst = 1 << 22, 1 << 23
    plan.d_out[0], plan.d_out[1] = 1 << 24, 1 << 25
    plan.d_workspace = 1 << 26
    if edges is not None:
        flat = (ctypes.c_uint32 * max(1, 2 * len(edges)))(*[v for e in edges for v in e])
        plan.n_qe = len(edges)
        plan.q_edges = ctypes.cast(flat, ctypes.POINTER(ctypes.c_uint32))
        keep.append(flat)
    plan.workspace_bytes = fss.LIB.match_workspace_bytes(ctypes.byref(plan))
    keep.append(preds)
    return plan


def _rounds(fss, plan):
    n = ctypes.c_uint32()
    words = (ctypes.c_uint64 * 8)()
    assert fss.LIB.match_rounds(ctypes.byref(plan), ctypes.byref(n), words, 8) == fss.OK
    return [int(words[r]) for r in range(n.value)]


def test_query_edges_schedule_and_errors(fss):
    """Query graphs (Def. 2): the AND levels follow the query edges given, and
    malformed query graphs are refused before anything is enqueued."""
    L = fss.LIB
    keep = []
    wv, we = (100 + 31) // 32, (50 + 31) // 32
    # path 0 -> 1 -> 2: the hop 1 -> 2 is ready in round 0, the hop 0 -> 1 after m_0's fold
    assert _rounds(fss, _star_plan(fss, keep, None)) == [2 * wv + 2 * we, 2 * we]
    assert _rounds(fss, _star_plan(fss, keep, [(0, 1), (1, 2)])) == [2 * wv + 2 * we, 2 * we]
    # out-star 0 -> 1, 0 -> 2: both hops wait for m_0's fold
    star = _star_plan(fss, keep, [(0, 1), (0, 2)])
    assert _rounds(fss, star) == [2 * wv, 4 * we]
    assert star.workspace_bytes > 0
    # a triangle has three hops
    assert _rounds(fss, _star_plan(fss, keep, [(0, 1), (1, 2), (2, 0)])) == [2 * wv + 2 * we, 4 * we]
    bad = [[(0, 0), (1, 2)], [(0, 1), (0, 1), (1, 2)], [(0, 3), (1, 2)], [(0, 1)], [(0, 1)] * 17]
    for edges in bad:
        plan = _star_plan(fss, keep, edges)
        assert plan.workspace_bytes == 0, edges
        plan.workspace_bytes = 1 << 20
        assert L.match_query(ctypes.byref(plan), 3, None) == fss.EINVAL, edges
        assert L.match_rounds(ctypes.byref(plan), ctypes.byref(ctypes.c_uint32()), None, 0) == fss.EINVAL
    plan = _star_plan(fss, keep, [(0, 1), (0, 2)])
    plan.q_edges = None
    assert L.match_query(ctypes.byref(plan), 3, None) == fss.EINVAL and b"q_edges" in L.fss_last_error()
    # a predicate on query edge 2 of a two-edge query
    plan = _star_plan(fss, keep, [(0, 1), (0, 2)])
    keep[-1][3].target = 5
    assert L.match_workspace_bytes(ctypes.byref(plan)) == 0
    assert L.match_query(ctypes.byref(plan), 3, None) == fss.EINVAL and b"targets" in L.fss_last_error()
    # one vertex with an edge
    one = fss.match_plan()
    one.n_qv, one.n_vertices, one.n_qe = 1, 10, 1
    one.q_edges = ctypes.cast((ctypes.c_uint32 * 2)(0, 0), ctypes.POINTER(ctypes.c_uint32))
    one.d_out[0], one.d_out[1] = 256, 512
    assert L.match_workspace_bytes(ctypes.byref(one)) == 0


def test_sec_access_batch_arguments(fss):
    """The batch form rejects NULL arrays before anything is enqueued and
    takes count 0 as nothing to do."""
    L = fss.LIB
    three = (ctypes.c_void_p * 3)(16, 32, 48)
    keys = (ctypes.c_uint64 * 3)(1, 2, 3)
    assert L.rss_sec_access_batch(0, 10, 64, None, None, 4, None, 1, None, None, None, None, None, None, None, None,
                                  None, 0, None) == fss.OK
    assert L.rss_sec_access_batch(2, 10, 64, None, 8, 4, three, 1, three, keys, (ctypes.c_uint32 * 2)(1, 3),
                                  (ctypes.c_uint64 * 6)(*range(6)), three, three, 64, 72, 256, 1 << 20,
                                  None) == fss.EINVAL and b"NULL" in L.fss_last_error()
    idm = (ctypes.c_void_p * 6)(16, 32, 48, 16, None, 48)
    assert L.rss_sec_access_batch(2, 10, 64, idm, 8, 4, three, 1, three, keys, (ctypes.c_uint32 * 2)(1, 3),
                                  (ctypes.c_uint64 * 6)(*range(6)), three, three, 64, 72, 256, 1 << 20,
                                  None) == fss.EINVAL and b"matched-ID share 4" in L.fss_last_error()


def test_tuning_limits(fss):
    L = fss.LIB
    assert L.fss_set_keygen_tuning(0) == fss.EINVAL and L.fss_set_keygen_tuning(9) == fss.EINVAL
    assert L.fss_set_keygen_tuning(4) == fss.OK and fss.get_keygen_tuning() == 4
    assert L.fss_set_keygen_tuning(1) == fss.OK and fss.get_keygen_tuning() == 1
    assert L.rss_set_shuffle_tuning(5) == fss.EINVAL and fss.get_shuffle_tuning() == 2
    assert L.rss_set_shuffle_tuning(0) == fss.OK and fss.get_shuffle_tuning() == 0
    assert L.rss_set_shuffle_tuning(2) == fss.OK and fss.get_shuffle_tuning() == 2
    assert L.fss_set_tuning(0, 1) == fss.EINVAL and L.fss_set_tuning(1, 3) == fss.EINVAL
