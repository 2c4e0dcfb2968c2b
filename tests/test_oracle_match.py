"""Pin of the oracle's share-level query plan: the client's reconstruction of
the two parties' result shares equals plaintext attributed subgraph matching
(Def. 2) found by enumerating every injective map of query vertices to graph
vertices, on tiny graphs and on the 1,024-vertex ER workload."""
import numpy as np
import pytest

import synth
from oracle import match


def _shares(graph, seed):
    sh = {k: synth.share_column(np.random.default_rng([seed, i]), v)
          for i, (k, v) in enumerate(sorted(graph.vcols.items()))}
    sh.update({"e:" + k: synth.share_column(np.random.default_rng([seed, 100 + i]), v)
               for i, (k, v) in enumerate(sorted(graph.ecols.items()))})
    return sh


def _run(graph, query, nbits=32, seed=99):
    out = match.run_plan(nbits, seed, graph, query, _shares(graph, seed), synth.pred_masks(seed, query, graph))
    nrows = graph.n_vertices if query.n_qv == 1 else graph.n_edges
    for o in out:  # pad bits are zero in both shares
        if nrows % 32:
            assert (o[0][-1] >> (nrows % 32)) == 0 and (o[1][-1] >> (nrows % 32)) == 0
    return match.results_from_bits(graph, query, match.reconstruct(out, nrows))


P = synth.Pred
QUERIES = [
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


@pytest.mark.parametrize("gseed", [0, 1, 2])
@pytest.mark.parametrize("qi", range(len(QUERIES)))
def test_tiny_graphs_match_brute_force(gseed, qi):
    g = synth.tiny_graph(gseed, n_vertices=10 if QUERIES[qi].n_qv == 4 else 12, n_edges=30)
    q = QUERIES[qi]
    assert _run(g, q, seed=gseed * 7 + qi) == match.brute_force(g, q)


def test_empty_result():
    g = synth.tiny_graph(5)
    q = synth.Query(9, 2, [P(0, "range", "attr", lo=3, hi=3)])
    assert _run(g, q) == set() == match.brute_force(g, q)


def test_small_domain_widths():
    g = synth.tiny_graph(4)
    q = synth.Query(11, 2, [P(0, "range", "attr", lo=1, hi=10), P(2, "eq", "label", a=2)])
    for nbits in (8, 12):
        assert _run(g, q, nbits=nbits) == match.brute_force(g, q)


def test_er_1024_workload():
    g, q = synth.config1(1)
    got = _run(g, q)
    assert got == match.brute_force_pairs(g, q)
    assert len(got) > 0


@pytest.mark.parametrize("qi", range(len(QUERIES)))
def test_sampled_rows_equal_full_plan(qi):
    """The row-by-row oracle used for full-size sampling gives the same share
    bits as the whole-table plan."""
    q = QUERIES[qi]
    g = synth.tiny_graph(qi, n_vertices=10 if q.n_qv == 4 else 12, n_edges=30)
    sh = _shares(g, 5)
    masks = synth.pred_masks(5, q, g)
    full = match.run_plan(32, 9, g, q, sh, masks)
    nrows = g.n_vertices if q.n_qv == 1 else g.n_edges
    rows = np.arange(nrows)[::-1]
    samp = match.sampled_outputs(32, 9, g, q, sh, masks, rows)
    for j, o in enumerate(full):
        for b in range(2):
            np.testing.assert_array_equal(match.fss.unpack_bits(o[b], nrows)[rows], samp[j, b])


# --------------------------------------------------------------------------- query graphs beyond paths (Def. 2)

SHAPES = [
    # out-star: one vertex with two out-edges
    synth.Query(21, 3, [P(0, "range", "attr", lo=2, hi=14), P(1, "eq", "label", a=1),
                        P(4, "range", "weight", lo=0, hi=12)], edges=[(0, 1), (0, 2)]),
    # in-star, edge predicates only on the first edge
    synth.Query(22, 3, [P(0, "eq", "label", a=2), P(3, "range", "weight", lo=3, hi=16),
                        P(3, "eq", "label", a=0)], edges=[(1, 0), (2, 0)]),
    # directed triangle (a cycle: the last edge closes on a joined vertex)
    synth.Query(23, 3, [P(0, "range", "attr", lo=0, hi=12)], edges=[(0, 1), (1, 2), (2, 0)]),
    # diamond, with a reversed edge order
    synth.Query(24, 4, [P(3, "range", "attr", lo=4, hi=16), P(1, "eq", "label", a=1),
                        P(2, "range", "attr", lo=0, hi=10)], edges=[(2, 3), (1, 3), (0, 2), (0, 1)]),
    # no predicate at all on a branching query
    synth.Query(25, 3, [], edges=[(1, 0), (1, 2)]),
    # two-edge cycle between the same pair, both directions
    synth.Query(26, 2, [P(0, "eq", "label", a=1), P(3, "range", "weight", lo=0, hi=8)], edges=[(0, 1), (1, 0)]),
]


@pytest.mark.parametrize("gseed", [0, 3])
@pytest.mark.parametrize("qi", range(len(SHAPES)))
def test_query_graphs_match_brute_force(gseed, qi):
    """Stars, a triangle, a diamond and a two-cycle: the reconstructed matches
    are the injective maps found by enumeration (Def. 2)."""
    q = SHAPES[qi]
    g = synth.tiny_graph(gseed + 10 * qi, n_vertices=9 if q.n_qv == 4 else 10, n_edges=40)
    want = match.brute_force(g, q)
    assert _run(g, q, seed=gseed * 11 + qi) == want
    if qi != 4:
        assert len(want) < len(match.brute_force(g, synth.Query(q.query_id, q.n_qv, [], edges=q.edges)))


def test_fig1_worked_example():
    """Sec. II-A, Fig. 1: exactly the two subgraphs the paper prints, by
    enumeration and through the shares."""
    from fixtures import fig1_example
    g, q, expected, names = fig1_example()
    assert len(expected) == 2
    assert match.brute_force(g, q) == expected
    assert _run(g, q, seed=2209) == expected
    for nbits in (8, 12):
        assert _run(g, q, nbits=nbits, seed=3526) == expected


def test_path_edges_are_the_default():
    """A query given the path's edges explicitly is the same plan: same ANDs,
    same share bits."""
    g = synth.tiny_graph(7)
    q = QUERIES[5]
    q2 = synth.Query(q.query_id, q.n_qv, q.preds, edges=[(0, 1), (1, 2)])
    sh = _shares(g, 3)
    masks = synth.pred_masks(3, q, g)
    a = match.run_plan(32, 1, g, q, sh, masks)
    b = match.run_plan(32, 1, g, q2, sh, masks)
    for x, y in zip(a, b):
        for p in range(2):
            np.testing.assert_array_equal(x[p], y[p])


@pytest.mark.parametrize("edges", [[], [(0, 0)], [(0, 1), (0, 1)], [(0, 3)], [(0, 1)]])
def test_rejected_query_graphs(edges):
    """No edge for several vertices, a self loop, an edge given twice, an
    endpoint outside the query, a vertex on no edge (n_qv = 3)."""
    q = synth.Query(30, 3, [], edges=edges)
    with pytest.raises(ValueError):
        match.check_query(q)
    with pytest.raises(ValueError):
        match.check_query(synth.Query(31, 1, [], edges=[(0, 1)]))


@pytest.mark.parametrize("qi", range(len(SHAPES)))
def test_sampled_rows_equal_full_plan_shapes(qi):
    q = SHAPES[qi]
    g = synth.tiny_graph(qi + 40, n_vertices=9, n_edges=40)
    sh = _shares(g, 6)
    masks = synth.pred_masks(6, q, g)
    full = match.run_plan(32, 8, g, q, sh, masks)
    rows = np.arange(g.n_edges)[::-1]
    samp = match.sampled_outputs(32, 8, g, q, sh, masks, rows)
    assert len(full) == q.n_qe
    for j, o in enumerate(full):
        for b in range(2):
            np.testing.assert_array_equal(match.fss.unpack_bits(o[b], g.n_edges)[rows], samp[j, b])


def random_query(seed: int):
    """A random valid query graph (Def. 2): 2-4 vertices, a random spanning
    tree plus extra edges (cycles, reversed pairs), 0-4 predicates on vertices
    and edges."""
    rng = np.random.default_rng(seed)
    nv = int(rng.integers(2, 5))
    edges = []
    for v in range(1, nv):
        u = int(rng.integers(0, v))
        edges.append((u, v) if rng.random() < 0.5 else (v, u))
    for _ in range(int(rng.integers(0, 3))):
        a, b = (int(x) for x in rng.choice(nv, 2, replace=False))
        if (a, b) not in edges:
            edges.append((a, b))
    preds = []
    for _ in range(int(rng.integers(0, 5))):
        t = int(rng.integers(0, nv + len(edges)))
        if t < nv:
            preds.append(P(t, "range", "attr", lo=int(rng.integers(0, 8)), hi=int(rng.integers(8, 17)))
                         if rng.random() < 0.5 else P(t, "eq", "label", a=int(rng.integers(0, 3))))
        else:
            preds.append(P(t, "range", "weight", lo=int(rng.integers(0, 8)), hi=int(rng.integers(8, 17)))
                         if rng.random() < 0.5 else P(t, "eq", "label", a=int(rng.integers(0, 3))))
    return synth.Query(300 + seed, nv, preds, edges=edges)


@pytest.mark.parametrize("qseed", range(24))
def test_random_query_graphs_match_brute_force(qseed):
    q = random_query(qseed)
    match.check_query(q)
    g = synth.tiny_graph(qseed + 500, n_vertices=8, n_edges=28, label_range=3)
    assert _run(g, q, seed=qseed) == match.brute_force(g, q)
