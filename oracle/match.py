"""Oracle for the whole query plan on shares, and the client-side reconstruction.

TEST INFRASTRUCTURE ONLY (see ``oracle/fss.py``).

Plan semantics (what both the oracle and the product compute):

1. Predicate k of the query (plan order) on a column of the target table:
   the dealer makes per-row keys with ``pred = k`` (Sec. V-C token generation,
   masked-input form), the servers open xhat = x0 + x1 + r (Sec. V-C), and each
   party evaluates its keys on xhat, giving one packed share bit per row
   (Alg. 3 line "evaluate" in its masked-input form; bits packed as in
   Sec. VII-A).
2. Per query vertex, then per query edge, its predicates are combined by AND
   (Sec. V-D, multi-predicate aggregation) as a left fold in plan order.  A
   vertex or edge with no predicate contributes the public constant 1.
3. Per hop j (query edge v_j -> v_{j+1}), each party gathers its share bits of
   v_j's result at the public ``src`` of every edge row and of v_{j+1}'s result
   at ``dst``; then h_j = (m_j[src] AND m_{j+1}[dst]) AND q_j over edge rows.
   (Alg. 2 matches vertex by vertex and follows neighbours; here endpoints are
   public row indices -- a documented deviation -- so following a neighbour is
   a gather.)
4. ANDs are numbered 0, 1, 2, ... in the order they are performed (vertex folds
   in vertex order, edge folds in edge order, then two per hop); AND number i
   consumes the Beaver triple stream (seed, query_id, and_id = i).  An AND with
   a public-1 operand is the other operand and consumes no number.
5. Pad bits (rows beyond the table in the last word) are zero in every share.

The result is h_0 .. h_{k-2} over edge rows (for a one-vertex query: m_0 over
vertex rows), as the two parties' packed shares.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import fss

PUBLIC_ONE = None


def _rows(graph, query, target):
    return graph.n_vertices if target < query.n_qv else graph.n_edges


def predicate_shares(nbits, seed, graph, query, shares, masks, k):
    """Step 1 for predicate k: both parties' packed share bits."""
    p = query.preds[k]
    table = shares[p.column] if p.target < query.n_qv else shares["e:" + p.column]
    x0, x1 = table
    r = masks[k]
    xhat = fss.mask_open(x0, x1, r)
    if p.kind == "eq":
        k0, k1 = fss.keygen_eq(nbits, seed, query.query_id, k, p.a, r)
        b0 = fss.eval_eq(nbits, 0, k0, xhat)
        b1 = fss.eval_eq(nbits, 1, k1, xhat)
    else:
        k0, k1 = fss.keygen_range(nbits, seed, query.query_id, k, p.lo, p.hi, r)
        b0 = fss.eval_range(nbits, 0, k0, xhat)
        b1 = fss.eval_range(nbits, 1, k1, xhat)
    return fss.pack_bits(b0), fss.pack_bits(b1)


def gather_shares(m, idx, nrows_src):
    """Each party's share bit of row idx[e] (a public index), packed over e."""
    if m is PUBLIC_ONE:
        return PUBLIC_ONE
    out = []
    for b in range(2):
        bits = fss.unpack_bits(m[b], nrows_src)
        out.append(fss.pack_bits(bits[idx]))
    return tuple(out)


class _AndCounter:
    def __init__(self, seed, query_id):
        self.seed = seed
        self.query_id = query_id
        self.next_id = 0

    def __call__(self, x, y, nrows):
        if x is PUBLIC_ONE:
            return y
        if y is PUBLIC_ONE:
            return x
        nwords = (nrows + 31) // 32
        trip = fss.triples(self.seed, self.query_id, self.next_id, nwords)
        self.next_id += 1
        return fss.beaver_and(x, y, trip, nrows)


def materialize(m, nrows):
    """Shares of the public constant 1: party 0 holds the valid-row mask."""
    if m is PUBLIC_ONE:
        return fss.valid_mask(nrows), np.zeros((nrows + 31) // 32, np.uint32)
    return m


def run_plan(nbits, seed, graph, query, shares, masks):
    """Both parties' shares of the query result (semantics in the module doc).

    ``shares``: column name -> (x0, x1) for vertex columns, "e:" + name for edge
    columns; ``masks``: one uint32 array per predicate."""
    pred_bits = [predicate_shares(nbits, seed, graph, query, shares, masks, k)
                 for k in range(len(query.preds))]
    AND = _AndCounter(seed, query.query_id)
    n_qv = query.n_qv
    m = []
    for i in range(n_qv):
        acc = PUBLIC_ONE
        for k, p in enumerate(query.preds):
            if p.target == i:
                acc = pred_bits[k] if acc is PUBLIC_ONE else AND(acc, pred_bits[k], graph.n_vertices)
        m.append(acc)
    q = []
    for j in range(n_qv - 1):
        acc = PUBLIC_ONE
        for k, p in enumerate(query.preds):
            if p.target == n_qv + j:
                acc = pred_bits[k] if acc is PUBLIC_ONE else AND(acc, pred_bits[k], graph.n_edges)
        q.append(acc)
    if n_qv == 1:
        return [materialize(m[0], graph.n_vertices)]
    hops = []
    for j in range(n_qv - 1):
        g = gather_shares(m[j], graph.src, graph.n_vertices)
        h = gather_shares(m[j + 1], graph.dst, graph.n_vertices)
        r1 = AND(g, h, graph.n_edges)
        r2 = AND(r1, q[j], graph.n_edges)
        hops.append(materialize(r2, graph.n_edges))
    return hops


def reconstruct(outputs, nrows):
    """XOR of the two parties' shares, unpacked to one 0/1 per row."""
    return [fss.unpack_bits(o[0] ^ o[1], nrows) for o in outputs]


def results_from_bits(graph, query, bits):
    """Client side: turn reconstructed bits into matched subgraphs.

    One-vertex query: the set of matching vertex ids.  Path query: every chain
    of edge rows (e_0, ..., e_{k-2}) with h_j[e_j] = 1, dst[e_j] = src[e_{j+1}]
    and pairwise distinct vertices (Def. 2 asks for a bijection)."""
    if query.n_qv == 1:
        return {(int(v),) for v in np.flatnonzero(bits[0])}
    src, dst = graph.src, graph.dst
    out_edges = {}
    for j in range(1, len(bits)):
        d = {}
        for e in np.flatnonzero(bits[j]).tolist():
            d.setdefault(int(src[e]), []).append(e)
        out_edges[j] = d
    results = set()
    for e0 in np.flatnonzero(bits[0]).tolist():
        chains = [([e0], [int(src[e0]), int(dst[e0])])]
        for j in range(1, len(bits)):
            nxt = []
            for edges, verts in chains:
                for e in out_edges[j].get(verts[-1], []):
                    nxt.append((edges + [e], verts + [int(dst[e])]))
            chains = nxt
        for edges, verts in chains:
            if len(set(verts)) == len(verts):
                results.add(tuple(edges))
    return results


def brute_force(graph, query):
    """Plaintext attributed subgraph matching by enumeration (Def. 2): every
    injective map of query vertices to graph vertices whose attribute
    predicates hold, combined with every choice of edge rows between mapped
    consecutive vertices whose edge predicates hold.  Only for tiny graphs."""
    n_qv = query.n_qv
    vpreds = [[p for p in query.preds if p.target == i] for i in range(n_qv)]
    epreds = [[p for p in query.preds if p.target == n_qv + j] for j in range(n_qv - 1)]

    def vertex_ok(i, v):
        return all(bool(p.holds(np.array([graph.vcols[p.column][v]]))[0]) for p in vpreds[i])

    def edge_ok(j, e):
        return all(bool(p.holds(np.array([graph.ecols[p.column][e]]))[0]) for p in epreds[j])

    edges_between = {}
    for e in range(graph.n_edges):
        edges_between.setdefault((int(graph.src[e]), int(graph.dst[e])), []).append(e)

    results = set()
    for vmap in itertools.permutations(range(graph.n_vertices), n_qv):
        if not all(vertex_ok(i, v) for i, v in enumerate(vmap)):
            continue
        if n_qv == 1:
            results.add((vmap[0],))
            continue
        choices = []
        for j in range(n_qv - 1):
            ok = [e for e in edges_between.get((vmap[j], vmap[j + 1]), []) if edge_ok(j, e)]
            choices.append(ok)
        for combo in itertools.product(*choices):
            results.add(tuple(combo))
    return results


def brute_force_pairs(graph, query):
    """Def. 2 by enumeration for a two-vertex path on a graph too large for the
    generic enumerator: all ordered pairs (u, w), u != w, tested as a boolean
    matrix, then all edge rows u -> w whose predicates hold."""
    assert query.n_qv == 2
    nv = graph.n_vertices
    ok0 = np.ones(nv, bool)
    ok1 = np.ones(nv, bool)
    for p in query.preds:
        if p.target == 0:
            ok0 &= p.holds(graph.vcols[p.column])
        elif p.target == 1:
            ok1 &= p.holds(graph.vcols[p.column])
    pair_ok = np.outer(ok0, ok1)
    np.fill_diagonal(pair_ok, False)
    eok = np.ones(graph.n_edges, bool)
    for p in query.preds:
        if p.target == 2:
            eok &= p.holds(graph.ecols[p.column])
    results = set()
    for e in range(graph.n_edges):
        u, w = int(graph.src[e]), int(graph.dst[e])
        if pair_ok[u, w] and eok[e]:
            results.add((e,))
    return results
