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
