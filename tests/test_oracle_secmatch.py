"""Pin of the oracle's whole secure matching protocol (Alg. 2 over the
paper's own encoding: secEval, re-share, secFetch Case II, secAccess over the
k-grouped posting lists): the client's reconstruction equals plaintext path
matching over the typed graph (Def. 2, by enumeration), for several graphs,
predicate kinds and path lengths, with repeated vertex types (where a chain
may revisit a vertex), and on the Sec. II-A example, where the two
root-to-leaf paths joined at the client give exactly the paper's two
printed subgraphs."""
import numpy as np
import pytest

import synth
from fixtures import fig1_typed
from oracle import secmatch

T = synth.TypedTarget
N = {"U": 5, "P": 14, "C": 6}
DOMAINS = {"U": {"city": 4}, "P": {"age": 64, "level": 8}, "C": {"industry": 4}}
DEGREES = {("U", "P"): 5, ("P", "C"): 2, ("P", "P"): 3}

QUERIES = [
    synth.TypedQuery(1, [T("U", "city", "range", lo=0, hi=3), T("P", "age", "range", lo=10, hi=50)]),
    synth.TypedQuery(2, [T("P", "level", "eq", a=3), T("C", "industry", "range", lo=1, hi=4)]),
    synth.TypedQuery(3, [T("U", "city", "range", lo=1, hi=4), T("P", "age", "range", lo=0, hi=40),
                         T("C", "industry", "eq", a=2)]),
    synth.TypedQuery(4, [T("P", "level", "range", lo=0, hi=6), T("P", "age", "range", lo=0, hi=64),
                         T("P", "level", "range", lo=0, hi=8)]),
]


def _run(tg, q, seed):
    shares = synth.typed_shares(seed, tg)
    enc = secmatch.encode(tg, shares, 2, 300 + seed)
    chains, _ = secmatch.sec_match(tg, enc, q, 40 + seed, (11, 12, 13), 7, 500 + seed)
    return secmatch.reconstruct(tg, q, chains)


@pytest.mark.parametrize("gseed", [1, 2])
@pytest.mark.parametrize("qi", range(len(QUERIES)))
def test_sec_match_equals_plaintext_matching(gseed, qi):
    tg = synth.typed_graph(gseed, N, DOMAINS, DEGREES)
    q = QUERIES[qi]
    want = secmatch.brute_force(tg, q)
    assert _run(tg, q, gseed) == want
    if qi == 3:     # P -> P -> P: some walks come back to their first vertex and are dropped
        walks = 0
        for a in range(tg.n["P"]):
            for b in tg.adj[("P", "P")][a]:
                walks += sum(1 for c in tg.adj[("P", "P")][b] if c == a)
        assert gseed != 1 or walks > 0


def test_empty_start():
    tg = synth.typed_graph(3, N, DOMAINS, DEGREES)
    q = synth.TypedQuery(9, [T("U", "city", "range", lo=2, hi=2), T("P", "age", "range", lo=0, hi=64)])
    assert _run(tg, q, 3) == set() == secmatch.brute_force(tg, q)


def test_fig1_through_the_paper_protocol():
    """Sec. II-A: U in Harbin -> P aged 30..40 -> C in software, and the same
    with C in Internet, each through Alg. 2; joined at the root with distinct
    persons, exactly g1 and g2."""
    tg, names = fig1_typed()
    harbin, software, internet = 1, 1, 2
    paths = []
    for qid, field in ((11, software), (12, internet)):
        q = synth.TypedQuery(qid, [T("U", "city", "eq", a=harbin), T("P", "age", "range", lo=30, hi=41),
                                   T("C", "industry", "eq", a=field)])
        got = _run(tg, q, qid)
        assert got == secmatch.brute_force(tg, q)
        paths.append(got)
    nm = lambda t, i: names[t][i]
    assert {tuple(nm(t, v) for t, v in zip("UPC", r)) for r in paths[0]} == {("U1", "P1", "C1"), ("U1", "P2", "C1")}
    assert {tuple(nm(t, v) for t, v in zip("UPC", r)) for r in paths[1]} == {("U1", "P3", "C2")}
    joined = secmatch.join_on_first(paths[0], paths[1], "UPC", "UPC")
    got = {tuple(nm(t, v) for t, v in zip("UPCPC", r)) for r in joined}
    assert got == {("U1", "P1", "C1", "P3", "C2"), ("U1", "P2", "C1", "P3", "C2")}


TREES = [
    # a star: U with two P branches
    synth.TypedQuery(41, [T("U", "city", "range", lo=0, hi=3), T("P", "age", "range", lo=0, hi=40),
                          T("P", "level", "range", lo=2, hi=8)], parents=[None, 0, 0]),
    # Fig. 1's shape: U -> P -> C and U -> P -> C
    synth.TypedQuery(42, [T("U", "city", "range", lo=0, hi=4), T("P", "age", "range", lo=10, hi=60),
                          T("C", "industry", "range", lo=0, hi=2), T("P", "level", "range", lo=0, hi=6),
                          T("C", "industry", "range", lo=2, hi=4)], parents=[None, 0, 1, 0, 3]),
    # a branch below the first hop
    synth.TypedQuery(43, [T("P", "level", "range", lo=0, hi=6), T("C", "industry", "range", lo=0, hi=3),
                          T("P", "age", "range", lo=0, hi=50)], parents=[None, 0, 0]),
]


@pytest.mark.parametrize("gseed", [1, 2])
@pytest.mark.parametrize("qi", range(len(TREES)))
def test_sec_match_trees_equal_plaintext_matching(gseed, qi):
    tg = synth.typed_graph(gseed, N, DOMAINS, DEGREES)
    q = TREES[qi]
    want = secmatch.brute_force(tg, q)
    assert _run(tg, q, gseed) == want
    assert gseed == 2 or len(want) > 0


def test_fig1_tree_natively():
    """Sec. II-A's query as the paper writes its token (Eq. enc_subg): U in
    Harbin with two branches, P aged 30..40 -> C in software and P aged 30..40
    -> C in Internet, in one run of Alg. 2: exactly g1 and g2."""
    tg, names = fig1_typed()
    q = synth.TypedQuery(13, [T("U", "city", "eq", a=1), T("P", "age", "range", lo=30, hi=41),
                              T("C", "industry", "eq", a=1), T("P", "age", "range", lo=30, hi=41),
                              T("C", "industry", "eq", a=2)], parents=[None, 0, 1, 0, 3])
    got = _run(tg, q, 13)
    assert got == secmatch.brute_force(tg, q)
    assert {tuple(names[t][v] for t, v in zip("UPCPC", r)) for r in got} == \
        {("U1", "P1", "C1", "P3", "C2"), ("U1", "P2", "C1", "P3", "C2")}


@pytest.mark.parametrize("gseed", [1, 2, 5])
def test_plaintext_match_equals_brute_force(gseed):
    """The adjacency walk used at larger sizes finds exactly the tuples the
    product enumeration finds, for paths and trees."""
    tg = synth.typed_graph(gseed, N, DOMAINS, DEGREES)
    for q in QUERIES + TREES:
        assert secmatch.plaintext_match(tg, q) == secmatch.brute_force(tg, q)
