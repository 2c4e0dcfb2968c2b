"""One server's half of secMatch (Alg. 2): match_query with party_mask 1 / 2,
run round by round with the messages carried between the two parties through
caller buffers.  Each party's result shares must equal those of the fused
both-party run (party_mask 3) and the oracle's, bit for bit."""
import numpy as np
import pytest
import torch

import synth
from oracle import match as omatch
from gpu_util import DEV, T, column_shares, plan_outputs

from test_gpu_parity import TINY_QUERIES

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fss():
    from paper_2209_03526_amd import fss as f
    return f


def _inputs(fss, g, q, shares, masks, seed):
    """Opened values and both parties' keys of every predicate (the dealer)."""
    preds = []
    for k, p in enumerate(q.preds):
        on_edge = p.target >= q.n_qv
        x0, x1 = shares[("e:" if on_edge else "") + p.column]
        rows = g.n_edges if on_edge else g.n_vertices
        r = T(masks[k])
        xhat = torch.empty(max(rows, 1), dtype=torch.int32, device=DEV)
        fss.fss_mask_open(T(x0), T(x1), r, xhat)
        kb = fss.KeyBatch(fss.EQ if p.kind == "eq" else fss.RANGE, 32, rows)
        fss.fss_keygen(seed, q.query_id, k, p.a if p.kind == "eq" else p.lo, p.hi, r, kb)
        preds.append((p.target, kb, xhat))
    return preds


def _plan(fss, g, q, preds, seed):
    src = T(g.src) if g.n_edges else None
    dst = T(g.dst) if g.n_edges else None
    return fss.Plan(seed, q.query_id, q.n_qv, g.n_vertices, g.n_edges, preds, src, dst, q.edges).allocate()


def _run_parties(fss, plans):
    """Both servers' rounds; plans[b] is party b's plan (its own workspace and
    outputs).  Returns the number of rounds."""
    sizes = fss.match_rounds(plans[0])
    assert sizes == fss.match_rounds(plans[1])
    R = len(sizes)
    msgs = [[torch.full((max(1, w),), -1, dtype=torch.int32, device=DEV) for w in sizes] for _ in range(2)]
    for r in range(R + 1):
        for b in (1, 0):                      # either order: a round reads only the peer's previous message
            fss.match_query(plans[b], party_mask=b + 1, round=r,
                            peer_msg=msgs[1 - b][r - 1] if r > 0 else None,
                            msg=msgs[b][r] if r < R else None)
    torch.cuda.synchronize()
    return R


def _check(fss, g, q, seed):
    shares = column_shares(g, seed)
    masks = synth.pred_masks(seed, q, g)
    preds = _inputs(fss, g, q, shares, masks, seed)
    both = _plan(fss, g, q, preds, seed)
    fss.match_query(both, 3)
    parties = [_plan(fss, g, q, preds, seed) for _ in range(2)]
    for pl in parties:                       # the other party's output stays untouched
        for o in pl.out:
            o.fill_(-1)
    R = _run_parties(fss, parties)
    got3 = plan_outputs(both, q, g)
    want = omatch.run_plan(32, seed, g, q, shares, masks)
    for b in range(2):
        got = plan_outputs(parties[b], q, g)
        for j in range(len(want)):
            np.testing.assert_array_equal(got[j][b], got3[j][b], err_msg=f"party {b} output {j} vs party_mask 3")
            np.testing.assert_array_equal(got[j][b], want[j][b], err_msg=f"party {b} output {j} vs oracle")
            assert (got[j][1 - b] == 0xFFFFFFFF).all()
    return R


@pytest.mark.parametrize("qi", range(len(TINY_QUERIES)))
def test_single_party_rounds_tiny(fss, qi):
    q = TINY_QUERIES[qi]
    g = synth.tiny_graph(1, n_vertices=10 if q.n_qv == 4 else 12, n_edges=30)
    _check(fss, g, q, 700 + qi)


def test_single_party_rounds_er_1024(fss):
    g, q = synth.config1(1)
    assert _check(fss, g, q, 4243) == 2        # no fold ANDs; the hop: endpoints at level 1, with q_0 at 2


def test_single_party_rounds_deep_folds(fss):
    """Folds of depth 1..3 on different targets, so ANDs open in different
    rounds and hop ANDs wait for the deepest fold they read; several tiles of
    edges (4 x 1024 words) and a ragged tail."""
    g = synth.tiny_graph(21, n_vertices=3000, n_edges=(4 << 15) + 77, label_range=3, attr_range=64)
    P = synth.Pred
    q = synth.Query(91, 3, [P(0, "eq", "label", a=1), P(0, "range", "attr", lo=3, hi=60),
                            P(1, "range", "attr", lo=0, hi=50), P(1, "range", "attr", lo=5, hi=64),
                            P(1, "eq", "label", a=2), P(1, "range", "attr", lo=1, hi=63),
                            P(3, "range", "weight", lo=0, hi=40), P(4, "eq", "label", a=1)])
    R = _check(fss, g, q, 31)
    assert R == 5          # vertex 1: 3 fold levels; hop 0 AND at 4, AND with q_0 at 5


def test_single_party_batch(fss):
    """match_query_batch with party_mask 1 / 2: every plan's round r in one call
    per party; results equal the per-plan runs (and the oracle)."""
    g = synth.tiny_graph(5, n_vertices=200, n_edges=3000, label_range=3, attr_range=64)
    seeds = [11, 12, 13]
    qs = [TINY_QUERIES[4], TINY_QUERIES[5], TINY_QUERIES[1]]
    plans, want = [[], []], []
    for q, seed in zip(qs, seeds):
        shares = column_shares(g, seed)
        masks = synth.pred_masks(seed, q, g)
        preds = _inputs(fss, g, q, shares, masks, seed)
        for b in range(2):
            plans[b].append(_plan(fss, g, q, preds, seed))
        want.append(omatch.run_plan(32, seed, g, q, shares, masks))
    sizes = [fss.match_rounds(p) for p in plans[0]]
    R = max(len(s) for s in sizes)
    msgs = [[[torch.empty(max(1, w), dtype=torch.int32, device=DEV) for w in s] for s in sizes] for _ in range(2)]
    queue = fss.Queue(16)
    for r in range(R + 1):
        for b in range(2):
            live = [i for i in range(len(qs)) if r <= len(sizes[i])]
            for i in live:
                Ri = len(sizes[i])
                fss.set_round(plans[b][i], r, msgs[1 - b][i][r - 1] if r > 0 else None,
                              msgs[b][i][r] if r < Ri else None)
            fss.match_query_batch([plans[b][i] for i in live], queue, party_mask=b + 1)
    torch.cuda.synchronize()
    for i, q in enumerate(qs):
        for b in range(2):
            got = plan_outputs(plans[b][i], q, g)
            for j in range(len(want[i])):
                np.testing.assert_array_equal(got[j][b], want[i][j][b], err_msg=f"plan {i} party {b} output {j}")


def test_single_party_rounds_full_size(fss):
    """One server's half at the full path query's size (Chung-Lu 2^22 vertices /
    2^25 edges, 4 vertex + 2 edge predicates): each party run alone in rounds
    gives the same shares as both at once, and sampled rows equal the
    oracle's."""
    from oracle import fss as ofss
    g, q = synth.config3(3)
    seed = 4244
    shares = column_shares(g, seed)
    masks = synth.pred_masks(seed, q, g)
    preds = _inputs(fss, g, q, shares, masks, seed)
    both = _plan(fss, g, q, preds, seed)
    fss.match_query(both, 3)
    parties = [_plan(fss, g, q, preds, seed) for _ in range(2)]
    R = _run_parties(fss, parties)
    assert R == 3          # c's fold at level 1; hop b -> c ANDs its endpoints at 2 and q_1 at 3
    rows = np.unique(np.concatenate([[0, 31, g.n_edges - 1], np.random.default_rng(7).integers(0, g.n_edges, 40)]))
    want = omatch.sampled_outputs(32, seed, g, q, shares, masks, rows)
    got3 = plan_outputs(both, q, g)
    for b in range(2):
        got = plan_outputs(parties[b], q, g)
        for j in range(len(got3)):
            np.testing.assert_array_equal(got[j][b], got3[j][b], err_msg=f"party {b} output {j}")
            np.testing.assert_array_equal(ofss.unpack_bits(got[j][b], g.n_edges)[rows], want[j, b])
