"""Oracle for the whole query plan on shares, and the client-side reconstruction.

TEST INFRASTRUCTURE ONLY (see ``oracle/fss.py``).

Plan semantics (what both the oracle and the product compute):

1. Predicate k of the query (plan order) on a column of the target table:
   the dealer makes per-row keys with ``pred = k`` (Sec. V-C token generation,
   masked-input form), the servers open xhat = x0 + x1 + r (Sec. V-C), and each
   party evaluates its keys on xhat, giving one packed share bit per row
   (the evaluation step of Alg. 3, in its masked-input form; bits packed as in
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


# --------------------------------------------------------------------------- sampled rows

def _and_schedule(query, n_vertices, n_edges):
    """The and_id of every AND the plan performs, found by walking the plan
    with public-ness only (no data): returns (vertex_fold, edge_fold, hop)
    where vertex_fold[i] / edge_fold[j] list (pred index, and_id or None) in
    fold order and hop[j] = (and_id of m_j[src] AND m_{j+1}[dst] or None,
    and_id of that AND q_j or None)."""
    n_qv = query.n_qv
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
    for j in range(n_qv - 1):
        steps, pub = [], True
        for k, p in enumerate(query.preds):
            if p.target == n_qv + j:
                steps.append((k, None if pub else take()))
                pub = False
        edge_fold.append(steps)
        public_e.append(pub)
    hop = []
    for j in range(n_qv - 1):
        gh_public = public_v[j] and public_v[j + 1]
        a1 = take() if (not public_v[j] and not public_v[j + 1]) else None
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

    out_rows = np.asarray(out_rows, dtype=np.int64)
    if n_qv == 1:
        return fold(vfold[0], out_rows, public_v[0])[None]
    outs = []
    for j in range(n_qv - 1):
        src = graph.src[out_rows].astype(np.int64)
        dst = graph.dst[out_rows].astype(np.int64)
        g = fold(vfold[j], src, public_v[j])
        h = fold(vfold[j + 1], dst, public_v[j + 1])
        q = fold(efold[j], out_rows, public_e[j])
        a1, a2 = hop[j]
        if a1 is not None:
            r1 = and_bits(g, h, a1, out_rows)
        else:
            r1 = h if public_v[j] else g
        r1_public = public_v[j] and public_v[j + 1]
        if a2 is not None:
            r2 = and_bits(r1, q, a2, out_rows)
        else:
            r2 = q if r1_public else r1
        outs.append(r2)
    return np.stack(outs)
