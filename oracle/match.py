"""Oracle for the whole query plan on shares, and the client-side reconstruction.

TEST INFRASTRUCTURE ONLY (see ``oracle/fss.py``).

Plan semantics (what both the oracle and the product compute).  The query
graph (Def. 2) has vertices 0 .. n_qv-1 and directed edges (a_j, b_j),
j = 0 .. n_qe-1 (a path v_0 -> v_1 -> ... unless given otherwise):

1. Predicate k of the query (plan order) on a column of the target table:
   the dealer makes per-row keys with ``pred = k`` (Sec. V-C token generation,
   masked-input form), the servers open xhat = x0 + x1 + r (Sec. V-C), and each
   party evaluates its keys on xhat, giving one packed share bit per row
   (the evaluation step of Alg. 3, in its masked-input form; bits packed as in
   Sec. VII-A).
2. Per query vertex, then per query edge, its predicates are combined by AND
   (Sec. V-D, multi-predicate aggregation) as a left fold in plan order.  A
   vertex or edge with no predicate contributes the public constant 1.
3. Per query edge j, each party gathers its share bits of a_j's result m_{a_j}
   at the public ``src`` of every edge row and of b_j's result m_{b_j} at
   ``dst``; then h_j = (m_{a_j}[src] AND m_{b_j}[dst]) AND q_j over edge rows.
   (Alg. 2 matches vertex by vertex and follows neighbours; here endpoints are
   public row indices -- a documented deviation -- so following a neighbour is
   a gather.)
4. ANDs are numbered 0, 1, 2, ... in the order they are performed (vertex folds
   in vertex order, edge folds in edge order, then two per query edge); AND
   number i consumes the Beaver triple stream (seed, query_id, and_id = i).  An
   AND with a public-1 operand is the other operand and consumes no number.
5. Pad bits (rows beyond the table in the last word) are zero in every share.

The result is h_0 .. h_{n_qe-1} over edge rows (for a one-vertex query: m_0
over vertex rows), as the two parties' packed shares.  The client joins the
h_j on their shared query vertices (``results_from_bits``).
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


def check_query(query):
    """The query graphs the plan accepts: no edge for one vertex; otherwise
    edges between distinct query vertices, no ordered pair twice, and every
    query vertex on some edge (its matches appear only through the edges)."""
    qe = query.qedges
    if query.n_qv < 1:
        raise ValueError("a query has at least one vertex")
    if query.n_qv == 1:
        if qe:
            raise ValueError("a one-vertex query has no edges")
        return
    if not qe:
        raise ValueError("a query of several vertices needs edges")
    seen = set()
    for a, b in qe:
        if not (0 <= a < query.n_qv and 0 <= b < query.n_qv) or a == b:
            raise ValueError(f"query edge ({a}, {b}) is not between two distinct query vertices")
        if (a, b) in seen:
            raise ValueError(f"query edge ({a}, {b}) given twice")
        seen.add((a, b))
    if {v for e in qe for v in e} != set(range(query.n_qv)):
        raise ValueError("a query vertex is on no edge")


def run_plan(nbits, seed, graph, query, shares, masks):
    """Both parties' shares of the query result (semantics in the module doc).

    ``shares``: column name -> (x0, x1) for vertex columns, "e:" + name for edge
    columns; ``masks``: one uint32 array per predicate."""
    check_query(query)
    pred_bits = [predicate_shares(nbits, seed, graph, query, shares, masks, k)
                 for k in range(len(query.preds))]
    AND = _AndCounter(seed, query.query_id)
    n_qv = query.n_qv
    qedges = query.qedges
    m = []
    for i in range(n_qv):
        acc = PUBLIC_ONE
        for k, p in enumerate(query.preds):
            if p.target == i:
                acc = pred_bits[k] if acc is PUBLIC_ONE else AND(acc, pred_bits[k], graph.n_vertices)
        m.append(acc)
    q = []
    for j in range(len(qedges)):
        acc = PUBLIC_ONE
        for k, p in enumerate(query.preds):
            if p.target == n_qv + j:
                acc = pred_bits[k] if acc is PUBLIC_ONE else AND(acc, pred_bits[k], graph.n_edges)
        q.append(acc)
    if n_qv == 1:
        return [materialize(m[0], graph.n_vertices)]
    hops = []
    for j, (a, b) in enumerate(qedges):
        g = gather_shares(m[a], graph.src, graph.n_vertices)
        h = gather_shares(m[b], graph.dst, graph.n_vertices)
        r1 = AND(g, h, graph.n_edges)
        r2 = AND(r1, q[j], graph.n_edges)
        hops.append(materialize(r2, graph.n_edges))
    return hops


def reconstruct(outputs, nrows):
    """XOR of the two parties' shares, unpacked to one 0/1 per row."""
    return [fss.unpack_bits(o[0] ^ o[1], nrows) for o in outputs]


def results_from_bits(graph, query, bits):
    """Client side: turn reconstructed bits into matched subgraphs.

    One-vertex query: the set of matching vertex ids.  Otherwise every tuple of
    edge rows (e_0, ..., e_{n_qe-1}) with h_j[e_j] = 1 such that one injective
    map f of query vertices to graph vertices has src[e_j] = f(a_j) and
    dst[e_j] = f(b_j) for every query edge j (Def. 2 asks for a bijection).
    The edges are joined in an order in which each one after the first shares
    a query vertex with an earlier one, where the query graph allows it."""
    if query.n_qv == 1:
        return {(int(v),) for v in np.flatnonzero(bits[0])}
    qe = query.qedges
    src, dst = graph.src, graph.dst
    rows = [np.flatnonzero(b).tolist() for b in bits]
    by_src = [{} for _ in qe]
    by_dst = [{} for _ in qe]
    for j, rj in enumerate(rows):
        for e in rj:
            by_src[j].setdefault(int(src[e]), []).append(e)
            by_dst[j].setdefault(int(dst[e]), []).append(e)
    order, seen = [], set()
    while len(order) < len(qe):
        rest = [j for j in range(len(qe)) if j not in order]
        touch = [j for j in rest if qe[j][0] in seen or qe[j][1] in seen]
        j = (touch or rest)[0]
        order.append(j)
        seen.update(qe[j])
    results = set()
    chosen = [None] * len(qe)

    def extend(i, f, used):
        if i == len(order):
            results.add(tuple(chosen))
            return
        j = order[i]
        a, b = qe[j]
        if a in f:
            cands = by_src[j].get(f[a], [])
        elif b in f:
            cands = by_dst[j].get(f[b], [])
        else:
            cands = rows[j]
        for e in cands:
            u, w = int(src[e]), int(dst[e])
            if (a in f and f[a] != u) or (b in f and f[b] != w):
                continue
            new = {}
            if a not in f:
                new[a] = u
            if b not in f:
                new[b] = w
            vals = list(new.values())
            if len(set(vals)) < len(vals) or any(v in used for v in vals):
                continue                      # f must stay injective
            chosen[j] = e
            f.update(new)
            extend(i + 1, f, used | set(vals))
            for k in new:
                del f[k]

    extend(0, {}, frozenset())
    return results


def brute_force(graph, query):
    """Plaintext attributed subgraph matching by enumeration (Def. 2): every
    injective map of query vertices to graph vertices whose attribute
    predicates hold, combined with every choice, per query edge (a, b), of an
    edge row from the image of a to the image of b whose edge predicates hold.
    Only for tiny graphs."""
    check_query(query)
    n_qv = query.n_qv
    qe = query.qedges
    vpreds = [[p for p in query.preds if p.target == i] for i in range(n_qv)]
    epreds = [[p for p in query.preds if p.target == n_qv + j] for j in range(len(qe))]

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
        for j, (a, b) in enumerate(qe):
            ok = [e for e in edges_between.get((vmap[a], vmap[b]), []) if edge_ok(j, e)]
            choices.append(ok)
        for combo in itertools.product(*choices):
            results.add(tuple(combo))
    return results


def brute_force_pairs(graph, query):
    """Def. 2 by enumeration for a two-vertex path on a graph too large for the
    generic enumerator: all ordered pairs (u, w), u != w, tested as a boolean
    matrix, then all edge rows u -> w whose predicates hold."""
    assert query.n_qv == 2 and query.qedges == [(0, 1)]
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


# --------------------------------------------------------------------------- sampled rows

def _and_schedule(query, n_vertices, n_edges):
    """The and_id of every AND the plan performs, found by walking the plan
    with public-ness only (no data): returns (vertex_fold, edge_fold, hop)
    where vertex_fold[i] / edge_fold[j] list (pred index, and_id or None) in
    fold order and hop[j] = (and_id of m_{a_j}[src] AND m_{b_j}[dst] or None,
    and_id of that AND q_j or None)."""
    n_qv = query.n_qv
    qe = query.qedges
    next_id = [0]

    def take():
        next_id[0] += 1
        return next_id[0] - 1

    vertex_fold, edge_fold, public_v, public_e = [], [], [], []
    for i in range(n_qv):
        steps, pub = [], True
        for k, p in enumerate(query.preds):
            if p.target == i:
                steps.append((k, None if pub else take()))
                pub = False
        vertex_fold.append(steps)
        public_v.append(pub)
    for j in range(len(qe)):
        steps, pub = [], True
        for k, p in enumerate(query.preds):
            if p.target == n_qv + j:
                steps.append((k, None if pub else take()))
                pub = False
        edge_fold.append(steps)
        public_e.append(pub)
    hop = []
    for j, (a, b) in enumerate(qe):
        gh_public = public_v[a] and public_v[b]
        a1 = take() if (not public_v[a] and not public_v[b]) else None
        a2 = take() if (not gh_public and not public_e[j]) else None
        hop.append((a1, a2))
    return vertex_fold, edge_fold, hop, public_v, public_e


def sampled_outputs(nbits, seed, graph, query, shares, masks, out_rows):
    """Both parties' share bits of the plan's outputs at the given rows only,
    computed row by row (keys of the needed rows, triple words of the needed
    positions).  ``out_rows``: vertex rows for a one-vertex query, else edge
    rows (the same rows are read from every hop).  Returns an array of shape
    (n_outputs, 2, len(out_rows)) of 0/1."""
    n_qv = query.n_qv
    vfold, efold, hop, public_v, public_e = _and_schedule(query, graph.n_vertices, graph.n_edges)
    qid = query.query_id

    def pred_bits(k, rows):
        p = query.preds[k]
        on_edge = p.target >= n_qv
        x0, x1 = shares[("e:" if on_edge else "") + p.column]
        r = masks[k][rows]
        xhat = fss.mask_open(x0[rows], x1[rows], r)
        if p.kind == "eq":
            k0, k1 = fss.keygen_eq(nbits, seed, qid, k, p.a, r, rows=rows)
            return np.stack([fss.eval_eq(nbits, 0, k0, xhat), fss.eval_eq(nbits, 1, k1, xhat)])
        k0, k1 = fss.keygen_range(nbits, seed, qid, k, p.lo, p.hi, r, rows=rows)
        return np.stack([fss.eval_range(nbits, 0, k0, xhat), fss.eval_range(nbits, 1, k1, xhat)])

    def and_bits(x, y, and_id, rows):
        words = (rows // 32).astype(np.uint32)
        t = fss.triples(seed, qid, and_id, 0, words=words)
        sh = (rows % 32).astype(np.uint32)
        bit = lambda w: ((w >> sh) & 1).astype(np.uint8)
        a = [bit(t["a"][b]) for b in range(2)]
        bb = [bit(t["b"][b]) for b in range(2)]
        c = [bit(t["c"][b]) for b in range(2)]
        d = (x[0] ^ a[0]) ^ (x[1] ^ a[1])
        e = (y[0] ^ bb[0]) ^ (y[1] ^ bb[1])
        z0 = c[0] ^ (d & bb[0]) ^ (e & a[0]) ^ (d & e)
        z1 = c[1] ^ (d & bb[1]) ^ (e & a[1])
        return np.stack([z0, z1])

    def fold(steps, rows, public):
        if public:
            return np.stack([np.ones(rows.size, np.uint8), np.zeros(rows.size, np.uint8)])
        acc = None
        for k, and_id in steps:
            pb = pred_bits(k, rows)
            acc = pb if and_id is None else and_bits(acc, pb, and_id, rows)
        return acc

    check_query(query)
    out_rows = np.asarray(out_rows, dtype=np.int64)
    if n_qv == 1:
        return fold(vfold[0], out_rows, public_v[0])[None]
    outs = []
    for j, (a, b) in enumerate(query.qedges):
        src = graph.src[out_rows].astype(np.int64)
        dst = graph.dst[out_rows].astype(np.int64)
        g = fold(vfold[a], src, public_v[a])
        h = fold(vfold[b], dst, public_v[b])
        q = fold(efold[j], out_rows, public_e[j])
        a1, a2 = hop[j]
        if a1 is not None:
            r1 = and_bits(g, h, a1, out_rows)
        else:
            r1 = h if public_v[a] else g
        r1_public = public_v[a] and public_v[b]
        if a2 is not None:
            r2 = and_bits(r1, q, a2, out_rows)
        else:
            r2 = q if r1_public else r1
        outs.append(r2)
    return np.stack(outs)
