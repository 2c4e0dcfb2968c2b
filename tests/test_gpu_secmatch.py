"""The paper's whole secMatch (Alg. 2) on the GPU, composed from the library
calls (replicated-token full-domain evaluations, secEval on one-hot records,
re-share, secFetch's table, shuffle/open/keep, secAccess over the k-grouped
posting lists): every result chain's three ID shares equal the oracle's, hop
by hop, and the client's reconstruction equals plaintext path matching; the
Sec. II-A example joined at the client gives the paper's two subgraphs."""
import numpy as np
import pytest
import torch

import synth
from fixtures import fig1_typed
from gpu_util import DEV
from oracle import secmatch as osm
from test_oracle_secmatch import DEGREES, DOMAINS, N, QUERIES, TREES

pytestmark = pytest.mark.gpu
T = synth.TypedTarget
K, SLOT_SEED, PRF, COUNTER = 2, 300, (11, 12, 13), 7


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_03526_amd import fss, secmatch
    torch.cuda.set_device(0)
    return fss, secmatch


def _gpu_graph(lib, tg, shares, slot_seed):
    fss, secmatch = lib
    padded = secmatch.padded_lengths(tg.adj, K)
    slots = {pair: synth.posting_slots(slot_seed + e, np.array([len(a) for a in tg.adj[pair]], np.uint32),
                                       padded[pair])
             for e, pair in enumerate(sorted(tg.adj))}
    domains = {(t, name): dom for t, d in tg.attrs.items() for name, (_, dom) in d.items()}
    return secmatch.encode_graph(tg.n, domains, shares, tg.adj, slots, K, device=DEV)


def _both(lib, tg, q, seed):
    fss, secmatch = lib
    shares = synth.typed_shares(seed, tg)
    enc = osm.encode(tg, shares, K, SLOT_SEED + seed)
    want, _ = osm.sec_match(tg, enc, q, 40 + seed, PRF, COUNTER, 500 + seed)
    eg = _gpu_graph(lib, tg, shares, SLOT_SEED + seed)
    got = secmatch.sec_match(eg, q, 40 + seed, PRF, COUNTER, 500 + seed, device=DEV)
    assert len(got) == len(want)
    for c, (gc, wc) in enumerate(zip(got, want)):
        for h, (gr, wr) in enumerate(zip(gc, wc)):
            for j in range(3):
                np.testing.assert_array_equal(gr[j], wr[j], err_msg=f"chain {c} hop {h} share {j + 1}")
    return osm.reconstruct(tg, q, got)


@pytest.mark.parametrize("gseed", [1, 2])
@pytest.mark.parametrize("qi", range(len(QUERIES)))
def test_sec_match_equals_oracle(lib, gseed, qi):
    tg = synth.typed_graph(gseed, N, DOMAINS, DEGREES)
    q = QUERIES[qi]
    print(f"graph {gseed} query {qi}", flush=True)
    assert _both(lib, tg, q, gseed) == osm.brute_force(tg, q)


def test_sec_match_larger_graph(lib):
    """Several hundred candidates per hop, posting lists of up to 12 entries,
    records of several words."""
    n = {"U": 40, "P": 700, "C": 90}
    domains = {"U": {"city": 40}, "P": {"age": 100, "level": 8}, "C": {"industry": 12}}
    degrees = {("U", "P"): 12, ("P", "C"): 3, ("P", "P"): 4}
    tg = synth.typed_graph(7, n, domains, degrees)
    q = synth.TypedQuery(21, [T("U", "city", "range", lo=0, hi=20), T("P", "age", "range", lo=20, hi=70),
                              T("C", "industry", "range", lo=2, hi=9)])
    print("larger graph", flush=True)
    got = _both(lib, tg, q, 7)
    assert got == osm.brute_force(tg, q) and len(got) > 0


def test_fig1_through_the_paper_protocol(lib):
    tg, names = fig1_typed()
    paths = []
    for qid, field in ((11, 1), (12, 2)):
        q = synth.TypedQuery(qid, [T("U", "city", "eq", a=1), T("P", "age", "range", lo=30, hi=41),
                                   T("C", "industry", "eq", a=field)])
        paths.append(_both(lib, tg, q, qid))
    joined = osm.join_on_first(paths[0], paths[1], "UPC", "UPC")
    got = {tuple(names[t][v] for t, v in zip("UPCPC", r)) for r in joined}
    assert got == {("U1", "P1", "C1", "P3", "C2"), ("U1", "P2", "C1", "P3", "C2")}


def test_sec_match_empty_start_and_empty_groups(lib):
    """No vertex matches the first target: no chain and no secAccess call;
    a query over a graph where some kept vertices have no neighbours of the
    next type: their groups are empty and take no randomness, as in the
    oracle."""
    tg = synth.typed_graph(3, N, DOMAINS, DEGREES)
    q = synth.TypedQuery(9, [T("U", "city", "range", lo=2, hi=2), T("P", "age", "range", lo=0, hi=64)])
    assert _both(lib, tg, q, 3) == set()
    sparse = synth.typed_graph(4, N, DOMAINS, {("U", "P"): 1, ("P", "C"): 1, ("P", "P"): 1})
    assert any(len(a) == 0 for a in sparse.adj[("U", "P")])
    q2 = synth.TypedQuery(10, [T("U", "city", "range", lo=0, hi=4), T("P", "age", "range", lo=0, hi=64),
                               T("C", "industry", "range", lo=0, hi=4)])
    assert _both(lib, sparse, q2, 4) == osm.brute_force(sparse, q2)


@pytest.mark.parametrize("gseed", [1, 2])
@pytest.mark.parametrize("qi", range(len(TREES)))
def test_sec_match_trees_equal_oracle(lib, gseed, qi):
    tg = synth.typed_graph(gseed, N, DOMAINS, DEGREES)
    q = TREES[qi]
    print(f"graph {gseed} tree {qi}", flush=True)
    assert _both(lib, tg, q, gseed) == osm.brute_force(tg, q)


def test_fig1_tree_natively(lib):
    """Sec. II-A's query as one two-branch tree through Alg. 2 on the GPU."""
    tg, names = fig1_typed()
    q = synth.TypedQuery(13, [T("U", "city", "eq", a=1), T("P", "age", "range", lo=30, hi=41),
                              T("C", "industry", "eq", a=1), T("P", "age", "range", lo=30, hi=41),
                              T("C", "industry", "eq", a=2)], parents=[None, 0, 1, 0, 3])
    got = _both(lib, tg, q, 13)
    assert {tuple(names[t][v] for t, v in zip("UPCPC", r)) for r in got} == \
        {("U1", "P1", "C1", "P3", "C2"), ("U1", "P2", "C1", "P3", "C2")}
