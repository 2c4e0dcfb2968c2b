"""Loaders of the worked examples under tests/golden/ (inputs only)."""
import json
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def fig1_example():
    """The attributed graph and query of the Sec. II-A example (Fig. 1), and
    the paper's two results as tuples of edge rows, one per query edge.

    Returns (graph, query, expected, vertex names)."""
    with open(os.path.join(GOLDEN, "fig1_university_query.json")) as f:
        d = json.load(f)
    names = [v["name"] for v in d["vertices"]]
    vid = {n: i for i, n in enumerate(names)}
    cols = ("type", "city", "age", "industry")
    vcols = {c: np.array([v[c] for v in d["vertices"]], np.uint32) for c in cols}
    src = np.array([vid[e[0]] for e in d["edges"]], np.uint32)
    dst = np.array([vid[e[1]] for e in d["edges"]], np.uint32)
    ecols = {"etype": np.array([e[2] for e in d["edges"]], np.uint32)}
    g = synth.Graph(len(names), src, dst, vcols, ecols)
    qv = {n: i for i, n in enumerate(d["query"]["vertices"])}
    qedges = [(qv[a], qv[b]) for a, b in d["query"]["edges"]]
    n_qv = len(qv)
    preds = []
    for p in d["query"]["vertex_predicates"]:
        if p[1] == "eq":
            preds.append(synth.Pred(qv[p[0]], "eq", p[2], a=p[3]))
        else:
            preds.append(synth.Pred(qv[p[0]], "range", p[2], lo=p[3], hi=p[4]))
    for p in d["query"]["edge_predicates"]:
        preds.append(synth.Pred(n_qv + p[0], "eq", p[2], a=p[3]))
    q = synth.Query(query_id=201, n_qv=n_qv, preds=preds, edges=qedges)
    row = {(int(u), int(w)): e for e, (u, w) in enumerate(zip(src, dst))}
    expected = set()
    for m in d["expected"]:
        f = {qv[k]: vid[v] for k, v in m.items()}
        expected.add(tuple(row[(f[a], f[b])] for a, b in qedges))
    return g, q, expected, names
