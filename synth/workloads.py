"""Workload generators (see the package docstring).

Graph model: a directed attributed graph (Def. 1) given as a vertex table and an
edge table.  Vertex ``i`` has uint32 attribute columns ``vcols[name][i]``; edge
row ``e`` goes from ``src[e]`` to ``dst[e]`` and has columns ``ecols[name][e]``.
A query graph (Def. 2) has query vertices 0 .. n_qv-1 and directed query edges
``qedges[j] = (a_j, b_j)``; by default it is the path v_0 -> v_1 -> ... ->
v_{k-1} (edge j = (j, j+1)).  Each predicate targets one query vertex
(``target < n_qv``) or one query edge (``target = n_qv + j``), and is an
equality ``x == a`` or a half-open range ``lo <= x < hi`` on one column.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

U32 = np.uint32


def _rng(*key) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(k) for k in key])))


@dataclass
class Pred:
    target: int
    kind: str            # "eq" | "range"
    column: str
    a: int = 0
    lo: int = 0
    hi: int = 0

    def holds(self, x: np.ndarray) -> np.ndarray:
        x = x.astype(np.uint64)
        if self.kind == "eq":
            return x == self.a
        return (x >= self.lo) & (x < self.hi)


@dataclass
class Query:
    query_id: int
    n_qv: int
    preds: list = field(default_factory=list)
    edges: list = None      # [(a_j, b_j), ...]; None: the path (j, j+1)

    @property
    def qedges(self) -> list:
        if self.edges is None:
            return [(j, j + 1) for j in range(self.n_qv - 1)]
        return [(int(a), int(b)) for a, b in self.edges]

    @property
    def n_qe(self) -> int:
        return len(self.qedges)


@dataclass
class Graph:
    n_vertices: int
    src: np.ndarray
    dst: np.ndarray
    vcols: dict
    ecols: dict
    _order: object = field(default=None, repr=False, compare=False)

    @property
    def n_edges(self) -> int:
        return int(self.src.size)

    def edge_order(self) -> tuple:
        """Edge rows sorted by (larger endpoint, row), and the sorted larger
        endpoints: the edges whose endpoints are both below r are the first
        searchsorted(keys, r) rows of this order (computed once per graph)."""
        if self._order is None:
            key = np.maximum(self.src, self.dst)
            order = np.argsort(key, kind="stable")
            self._order = (order, key[order])
        return self._order


def rows_of_target(graph: Graph, query: Query, target: int) -> int:
    return graph.n_vertices if target < query.n_qv else graph.n_edges


def column_of(graph: Graph, query: Query, pred: Pred) -> np.ndarray:
    return graph.vcols[pred.column] if pred.target < query.n_qv else graph.ecols[pred.column]


# --------------------------------------------------------------------------- distributions

def zipf_column(rng: np.random.Generator, size: int, s: float = 1.1) -> np.ndarray:
    """Zipf(s) ranks k >= 1 over [1, 2^32], returned as k - 1 (ranks above 2^32
    are drawn again)."""
    out = rng.zipf(s, size).astype(np.uint64)
    bad = out > (1 << 32)
    while bad.any():
        out[bad] = rng.zipf(s, int(bad.sum())).astype(np.uint64)
        bad = out > (1 << 32)
    return (out - 1).astype(U32)


def vertex_table(seed: int, n: int) -> dict:
    """Two labels uniform in [0, 64) and two Zipf(1.1) integers over [0, 2^32)."""
    rng = _rng(seed, 11)
    return {
        "l0": rng.integers(0, 64, n, dtype=U32),
        "l1": rng.integers(0, 64, n, dtype=U32),
        "z0": zipf_column(rng, n),
        "z1": zipf_column(rng, n),
    }


def er_graph(seed: int, n_vertices: int, n_edges: int) -> tuple:
    """Erdos-Renyi G(n, m): m distinct directed pairs (u, v), u != v."""
    rng = _rng(seed, 21)
    assert n_edges <= n_vertices * (n_vertices - 1)
    chosen = set()
    src, dst = [], []
    while len(src) < n_edges:
        need = n_edges - len(src)
        u = rng.integers(0, n_vertices, 2 * need)
        v = rng.integers(0, n_vertices, 2 * need)
        for a, b in zip(u.tolist(), v.tolist()):
            if a != b and (a, b) not in chosen:
                chosen.add((a, b))
                src.append(a)
                dst.append(b)
                if len(src) == n_edges:
                    break
    return np.array(src, U32), np.array(dst, U32)


def chung_lu_graph(seed: int, n_vertices: int, n_edges: int, gamma: float = 2.1) -> tuple:
    """Chung-Lu power-law graph: endpoints drawn with probability proportional to
    w_i = (i + 1)^(-1 / (gamma - 1)); self-loops are drawn again, multi-edges kept."""
    rng = _rng(seed, 31)
    w = np.arange(1, n_vertices + 1, dtype=np.float64) ** (-1.0 / (gamma - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]

    # index of the first cdf entry above u (searchsorted, side="right"), sped up
    # by a guide table over [0,1) and a vectorised binary search in each bucket
    buckets = 1 << 22
    guide = np.searchsorted(cdf, np.arange(buckets + 1) / buckets, side="right")

    def draw(k):
        u = rng.random(k)
        j = np.minimum((u * buckets).astype(np.int64), buckets - 1)
        lo, hi = guide[j].copy(), guide[j + 1].copy()
        act = np.flatnonzero(lo < hi)
        while act.size:
            mid = (lo[act] + hi[act]) // 2
            right = cdf[mid] <= u[act]
            lo[act] = np.where(right, mid + 1, lo[act])
            hi[act] = np.where(right, hi[act], mid)
            act = act[lo[act] < hi[act]]
        return np.minimum(lo, n_vertices - 1)

    src = draw(n_edges)
    dst = draw(n_edges)
    loop = src == dst
    while loop.any():
        dst[loop] = draw(int(loop.sum()))
        loop = src == dst
    return src.astype(U32), dst.astype(U32)


# --------------------------------------------------------------------------- shares and masks

def share_column(rng: np.random.Generator, x: np.ndarray) -> tuple:
    """Two-party additive shares mod 2^32: x0 uniform, x1 = x - x0."""
    x0 = rng.integers(0, 1 << 32, x.size, dtype=np.uint64).astype(U32)
    x1 = (x.astype(np.uint64) - x0.astype(np.uint64)).astype(U32)
    return x0, x1


def share_columns(seed: int, cols: dict) -> dict:
    return {name: share_column(_rng(seed, 41, i), cols[name]) for i, name in enumerate(sorted(cols))}


def pred_masks(seed: int, query: Query, graph: Graph) -> list:
    """One fresh uint32 mask per (query, predicate, row)."""
    return [_rng(seed, 51, query.query_id, k).integers(0, 1 << 32, rows_of_target(graph, query, p.target),
                                                       dtype=np.uint64).astype(U32)
            for k, p in enumerate(query.preds)]


def onehot_rss(seed: int, values: np.ndarray, npos: int) -> np.ndarray:
    """Three binary shares of the one-hot encoding of each value (Sec. V-B):
    shares 1 and 2 uniform, share 3 = onehot ^ share 1 ^ share 2.
    Returns a (3, C, npos) array of 0/1."""
    rng = _rng(seed, 121)
    c = values.size
    onehot = np.zeros((c, npos), np.uint8)
    onehot[np.arange(c), values.astype(np.int64)] = 1
    s1 = rng.integers(0, 2, (c, npos), dtype=np.uint8)
    s2 = rng.integers(0, 2, (c, npos), dtype=np.uint8)
    return np.stack([s1, s2, onehot ^ s1 ^ s2])


def pack_word_major(bits: np.ndarray) -> np.ndarray:
    """(C, npos) 0/1 -> uint32 words laid out [word][candidate]: word w of
    candidate c holds positions 32w .. 32w+31 (position p at bit p % 32)."""
    c, npos = bits.shape
    nw = (npos + 31) // 32
    padded = np.zeros((c, nw * 32), np.uint8)
    padded[:, :npos] = bits
    words = np.packbits(padded.reshape(c, nw, 32), axis=2, bitorder="little").view("<u4").reshape(c, nw)
    return np.ascontiguousarray(words.T).astype(np.uint32)


def posting_slots(seed: int, lengths: np.ndarray, padded: np.ndarray) -> np.ndarray:
    """The data owner's random placement of true IDs among the dummy IDs of a
    padded posting list: for vertex v, the first lengths[v] entries of a
    seeded permutation of range(padded[v]).  Flat, aligned with the
    adjacency's CSR order (slot of each true neighbour)."""
    out = np.zeros(int(np.sum(lengths)), np.uint32)
    at = 0
    for v, (n, p) in enumerate(zip(lengths, padded)):
        if n:
            out[at:at + n] = _rng(seed, 131, v).permutation(int(p))[:n]
        at += n
    return out


def posting_graph(seed: int, n: int, x_count: int, max_degree: int, n_types: int = 2) -> tuple:
    """A candidate table for secAccess: n vertices of n_types types, each with
    a posting list of distinct neighbour IDs in [0, x_count) (lengths uniform
    in [0, max_degree], power-law-ish: a few long lists), and one 64-bit
    attribute record per neighbour ID.  Returns (types, adjacency lists,
    attributes (x_count, 2) uint32)."""
    rng = _rng(seed, 141)
    types = rng.integers(0, n_types, n).astype(np.uint32)
    deg = np.minimum(rng.zipf(1.8, n) - 1, max_degree)
    adj = [np.sort(rng.choice(x_count, int(d), replace=False)).astype(np.uint32) for d in deg]
    attr = rng.integers(0, 2**32, (x_count, 2), dtype=np.uint64).astype(np.uint32)
    return types, adj, attr


# --------------------------------------------------------------------------- workloads

def tiny_graph(seed: int, n_vertices: int = 12, n_edges: int = 30, label_range: int = 4,
               attr_range: int = 16, multi_edges: bool = True) -> Graph:
    """A very small graph (for brute force over every injective vertex map).
    Multi-edges are allowed so that distinct edge rows between one vertex pair
    show up as distinct results."""
    rng = _rng(seed, 61)
    src = rng.integers(0, n_vertices, n_edges)
    dst = rng.integers(0, n_vertices, n_edges)
    loop = src == dst
    while loop.any():
        dst[loop] = rng.integers(0, n_vertices, int(loop.sum()))
        loop = src == dst
    if not multi_edges:
        pairs = {}
        for e, (u, v) in enumerate(zip(src.tolist(), dst.tolist())):
            pairs.setdefault((u, v), e)
        keep = np.array(sorted(pairs.values()))
        src, dst = src[keep], dst[keep]
    vcols = {"label": rng.integers(0, label_range, n_vertices, dtype=U32),
             "attr": rng.integers(0, attr_range, n_vertices, dtype=U32)}
    ecols = {"label": rng.integers(0, label_range, src.size, dtype=U32),
             "weight": rng.integers(0, attr_range, src.size, dtype=U32)}
    return Graph(n_vertices, src.astype(U32), dst.astype(U32), vcols, ecols)


def config1(seed: int = 1) -> tuple:
    """Tiny plain query: ER graph of 1,024 vertices and 8,192 edges; vertex label
    in [0,16), vertex attribute in [0,2^20), edge label in [0,4).  Query v1 -> v2
    with v1.label == A, lo <= v2.attr < hi (hi = lo + 2^18) and edge label == C."""
    src, dst = er_graph(seed, 1024, 8192)
    rng = _rng(seed, 71)
    vcols = {"label": rng.integers(0, 16, 1024, dtype=U32),
             "attr": rng.integers(0, 1 << 20, 1024, dtype=U32)}
    ecols = {"label": rng.integers(0, 4, 8192, dtype=U32)}
    g = Graph(1024, src, dst, vcols, ecols)
    lo = int(rng.integers(0, (1 << 20) - (1 << 18)))
    q = Query(query_id=1, n_qv=2, preds=[
        Pred(0, "eq", "label", a=int(rng.integers(0, 16))),
        Pred(1, "range", "attr", lo=lo, hi=lo + (1 << 18)),
        Pred(2, "eq", "label", a=int(rng.integers(0, 4))),
    ])
    return g, q


def _quartile_range(col: np.ndarray) -> tuple:
    lo, hi = np.quantile(col.astype(np.float64), [0.25, 0.75])
    lo, hi = int(lo), int(hi)
    if hi <= lo:
        hi = lo + 1
    return lo, hi


def config2(seed: int = 2, n: int = 1 << 22) -> tuple:
    """Vertex filtering at scale: n rows x (l0, l1, z0, z1); one query with
    l0 == A, l1 == B, z0 in [q25, q75), z1 in [q25, q75)."""
    cols = vertex_table(seed, n)
    rng = _rng(seed, 81)
    z0 = _quartile_range(cols["z0"])
    z1 = _quartile_range(cols["z1"])
    g = Graph(n, np.zeros(0, U32), np.zeros(0, U32), cols, {})
    q = Query(query_id=2, n_qv=1, preds=[
        Pred(0, "eq", "l0", a=int(rng.integers(0, 64))),
        Pred(0, "eq", "l1", a=int(rng.integers(0, 64))),
        Pred(0, "range", "z0", lo=z0[0], hi=z0[1]),
        Pred(0, "range", "z1", lo=z1[0], hi=z1[1]),
    ])
    return g, q


def config3(seed: int = 3, n_vertices: int = 1 << 22, n_edges: int = 1 << 25) -> tuple:
    """Full plain query: Chung-Lu (gamma 2.1) graph; vertex columns as config2,
    edge label in [0,4), edge weight in [0,2^16).  Path a -> b -> c with
    a.l0 == A, b.z0 in [q25,q75), c.l1 == B and c.z1 in [q25,q75),
    e_ab.label == C, e_bc.weight in [w_lo, w_lo + 2^14)."""
    src, dst = chung_lu_graph(seed, n_vertices, n_edges)
    cols = vertex_table(seed, n_vertices)
    rng = _rng(seed, 91)
    ecols = {"label": rng.integers(0, 4, n_edges, dtype=U32),
             "weight": rng.integers(0, 1 << 16, n_edges, dtype=U32)}
    g = Graph(n_vertices, src, dst, cols, ecols)
    z0 = _quartile_range(cols["z0"])
    z1 = _quartile_range(cols["z1"])
    w_lo = int(rng.integers(0, (1 << 16) - (1 << 14)))
    q = Query(query_id=3, n_qv=3, preds=[
        Pred(0, "eq", "l0", a=int(rng.integers(0, 64))),
        Pred(1, "range", "z0", lo=z0[0], hi=z0[1]),
        Pred(2, "eq", "l1", a=int(rng.integers(0, 64))),
        Pred(2, "range", "z1", lo=z1[0], hi=z1[1]),
        Pred(3, "eq", "label", a=int(rng.integers(0, 4))),
        Pred(4, "range", "weight", lo=w_lo, hi=w_lo + (1 << 14)),
    ])
    return g, q


def candidate_view(graph: Graph, rows: int) -> tuple:
    """A query's candidate tables over ``rows`` rows: vertices [0, rows) and,
    among the edges whose endpoints are both below ``rows`` (a public filter),
    the first ``rows`` in the order of ``Graph.edge_order`` -- so every
    candidate edge table is a prefix of one fixed order of the edge table.
    Returns (view graph, edge rows of the view in the full table)."""
    r = min(rows, graph.n_vertices)
    order, keys = graph.edge_order()
    erows = order[:min(rows, int(np.searchsorted(keys, keys.dtype.type(r), side="left")))]
    view = Graph(r, graph.src[erows], graph.dst[erows], {k: v[:r] for k, v in graph.vcols.items()},
                 {k: v[erows] for k, v in graph.ecols.items()})
    return view, erows


def view_shares(shares: dict, graph: Graph, view: Graph, erows: np.ndarray) -> dict:
    """The servers' shares restricted to a candidate view (same share values)."""
    out = {}
    for k, (x0, x1) in shares.items():
        if k.startswith("e:"):
            out[k] = (x0[erows], x1[erows])
        else:
            out[k] = (x0[:view.n_vertices], x1[:view.n_vertices])
    return out


def batch_queries(seed: int, graph: Graph, count: int = 64, min_log_rows: int = 12,
                  max_log_rows: int = 22) -> list:
    """Uneven query mix: 1-5 predicates (equality : range = 1 : 1) over 1-4 query
    vertices (path shaped); candidate table size R log-uniform in
    [2^min_log_rows, 2^max_log_rows] (candidates are rows [0, R)).  Returns a
    list of (query, R)."""
    rng = _rng(seed, 101)
    out = []
    vcols = sorted(graph.vcols)
    ecols = sorted(graph.ecols)
    for i in range(count):
        n_qv = int(rng.integers(1, 5))
        n_pred = int(rng.integers(1, 6))
        rows = int(round(2.0 ** rng.uniform(min_log_rows, max_log_rows)))
        rows = max(1, min(rows, graph.n_vertices))
        preds = []
        for k in range(n_pred):
            on_edge = n_qv > 1 and ecols and rng.random() < 0.3
            target = n_qv + int(rng.integers(0, n_qv - 1)) if on_edge else int(rng.integers(0, n_qv))
            cols = ecols if on_edge else vcols
            col = cols[int(rng.integers(0, len(cols)))]
            values = (graph.ecols if on_edge else graph.vcols)[col]
            if rng.random() < 0.5:
                preds.append(Pred(target, "eq", col, a=int(values[int(rng.integers(0, values.size))])))
            else:
                sample = values[rng.integers(0, values.size, 4096)]
                lo, hi = _quartile_range(sample)
                preds.append(Pred(target, "range", col, lo=lo, hi=hi))
        out.append((Query(query_id=1000 + i, n_qv=n_qv, preds=preds), rows))
    return out


# --------------------------------------------------------------------------- typed graphs (the paper's own encoding)

@dataclass
class TypedGraph:
    """Def. 1 with vertex types: type T has n[T] vertices, IDs 0 .. n[T]-1 per
    type; attrs[T][name] = (values uint32[n[T]], domain size) is an attribute
    of the type's vertices (values below the domain size, for one-hot
    encoding); adj[(T, T2)] lists, per vertex of type T, the sorted IDs of its
    neighbours of type T2 (one edge type per ordered pair of vertex types)."""
    n: dict
    attrs: dict
    adj: dict


@dataclass
class TypedTarget:
    """One target vertex of a path query in the paper's form (Sec. V-C): its
    type, the attribute its predicate reads, and the predicate on that
    attribute's value (equality, or a half-open range)."""
    vtype: str
    attr: str
    kind: str            # "eq" | "range"
    a: int = 0
    lo: int = 0
    hi: int = 0

    def holds(self, x) -> bool:
        x = int(x)
        return x == self.a if self.kind == "eq" else self.lo <= x < self.hi


@dataclass
class TypedQuery:
    """A tree query over a typed graph: target i > 0 is a neighbour (of its
    type) of target parents[i] < i; parents None is the path V_1 -> V_2 ->
    ... (target i's parent is i - 1)."""
    query_id: int
    targets: list
    parents: list = None

    def parent(self, i: int):
        if i == 0:
            return None
        return i - 1 if self.parents is None else self.parents[i]


def typed_graph(seed: int, n: dict, domains: dict, degrees: dict) -> TypedGraph:
    """Random typed graph: per type T, n[T] vertices and one attribute per
    (name, domain size) in domains[T], uniform over the domain; per ordered
    type pair (T, T2) in degrees, each vertex of T gets a uniform number in
    [0, degrees[(T, T2)]] of distinct neighbours of type T2 (no self loop when
    T == T2)."""
    rng = _rng(seed, 151)
    attrs = {t: {name: (rng.integers(0, dom, n[t]).astype(U32), int(dom)) for name, dom in sorted(domains[t].items())}
             for t in sorted(n)}
    adj = {}
    for (t, t2), dmax in sorted(degrees.items()):
        lists = []
        for v in range(n[t]):
            pool = np.array([u for u in range(n[t2]) if not (t == t2 and u == v)], np.int64)
            d = int(rng.integers(0, dmax + 1))
            lists.append(np.sort(rng.choice(pool, min(d, pool.size), replace=False)).astype(U32))
        adj[(t, t2)] = lists
    return TypedGraph(dict(n), attrs, adj)


def typed_shares(seed: int, tg: TypedGraph) -> dict:
    """The data owner's one-hot binary RSS of the typed graph's IDs and
    attributes (Sec. V-B), packed record-major (one record of ceil(n/32)
    words per vertex): {("id", T): (3, n_T, words), ("attr", T, name): (3,
    n_T, words)}; shares 1 and 2 uniform, share 3 the one-hot ^ both."""
    out = {}
    for i, t in enumerate(sorted(tg.n)):
        out[("id", t)] = pack_records(onehot_rss(seed * 1000 + i, np.arange(tg.n[t], dtype=U32), tg.n[t]))
        for j, (name, (vals, dom)) in enumerate(sorted(tg.attrs[t].items())):
            out[("attr", t, name)] = pack_records(onehot_rss(seed * 1000 + 100 + 10 * i + j, vals, dom))
    return out


def pack_records(bits: np.ndarray) -> np.ndarray:
    """(..., R, npos) 0/1 -> (..., R, ceil(npos/32)) uint32, position p of a
    record at bit p % 32 of word p // 32."""
    *lead, npos = bits.shape
    nw = (npos + 31) // 32
    padded = np.zeros((*lead, nw * 32), np.uint8)
    padded[..., :npos] = bits
    return np.packbits(padded.reshape(*lead, nw, 32), axis=-1, bitorder="little").view("<u4").reshape(
        *lead, nw).astype(U32)
