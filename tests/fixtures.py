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


def fig1_typed():
    """The same example as a typed graph in the paper's own model (Sec. V-A):
    types U, P, C with IDs per type in the order of the fixture, attributes
    U.city, P.age, C.industry, and edge types graduate_from (U -> P), work_at
    (P -> C) and friend (P -> P).  Returns (typed graph, names per type)."""
    with open(os.path.join(GOLDEN, "fig1_university_query.json")) as f:
        d = json.load(f)
    tname = {v: k for k, v in d["codes"]["type"].items()}
    per = {"U": [], "P": [], "C": []}
    for v in d["vertices"]:
        per[tname[v["type"]]].append(v)
    idx = {v["name"]: (t, i) for t, vs in per.items() for i, v in enumerate(vs)}
    field = {"U": ("city", 4), "P": ("age", 64), "C": ("industry", 4)}
    attrs = {t: {field[t][0]: (np.array([v[field[t][0]] for v in vs], np.uint32), field[t][1])}
             for t, vs in per.items()}
    adj = {}
    for a, b, et in d["edges"]:
        (ta, ia), (tb, ib) = idx[a], idx[b]
        adj.setdefault((ta, tb), [[] for _ in per[ta]])[ia].append(ib)
    adj = {k: [np.array(sorted(x), np.uint32) for x in v] for k, v in adj.items()}
    tg = synth.TypedGraph({t: len(vs) for t, vs in per.items()}, attrs, adj)
    return tg, {t: [v["name"] for v in vs] for t, vs in per.items()}
