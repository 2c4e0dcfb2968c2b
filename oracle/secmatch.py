"""Oracle for the paper's whole secure matching protocol, Alg. 2 (secMatch),
over the paper's own encoding, for tree queries (a path V_1 -> V_2 -> ... ->
V_q, or targets each hanging off an earlier one, as Fig. 1's).

TEST INFRASTRUCTURE ONLY (see ``oracle/fss.py``).

Alg. 2 composed from the rows the oracle already pins:
- secEval (Alg. 3, Eq. predEval; ``rss.server_shares`` with the replicated
  token ``rss.token``), then the re-share of its three-out-of-three bits into
  RSS (``rss.reshare``);
- secFetch Case II (Alg. 4): the table {x || id || d} shuffled (Alg. 5), the
  shuffled x opened, the rows with 1 kept (``shuffle.fetch_case2``);
- secAccess (Alg. 6) over the posting lists of Alg. 1 (``access.sec_access_csr``):
  the matched vertex's neighbours of the next target's type, with their
  one-hot IDs and the one-hot value of the attribute the next predicate reads.

Readings (Alg. 2 leaves these open):
1. Target i's candidates come in groups.  Target 0 has one group, every
   vertex of type T_0.  Every vertex kept at target p gives one group at each
   child target i of p (parent(i) = p): the neighbours secAccess returns for
   it.  secEval runs per group, and secFetch once per group, so a kept vertex
   stays tied to the kept vertex whose neighbour it is (its parent) -- the
   reorganisation into subgraphs at the end of Alg. 2 needs that tie.
2. Randomness: the re-shares take PRF counters in order from ``counter0``
   (secEval's re-share one, secAccess two); the shuffles take seed triples in
   order from ``seed0``, the s-th shuffle (secFetch's and secAccess's alike)
   the triple (seed0 + 3s, seed0 + 3s + 1, seed0 + 3s + 2).  Predicate i's
   token is made with pred = i.
3. Order: target by target in index order; within a target, first every
   group's secEval, re-share and secFetch, group by group in order of
   creation; then, group by group, for each child target in index order and
   each kept vertex in kept order, its secAccess.  An empty group takes no
   randomness.  (For a path this is hop by hop.)  Taking a target's secFetch
   steps before its secAccess steps lets the servers run all of a target's
   fetches before they learn any group's count, and all of its secAccess
   calls after.
4. The result is every assignment of one kept vertex per target, each target's
   vertex in the group its parent's vertex made, as the three shares of each
   target's one-hot ID record.  The client reconstructs the IDs and drops
   results that use a vertex twice (Def. 2 asks for a bijection).

The encoded graph (``synth.typed_shares``: one-hot IDs and attribute values
in binary RSS) and the posting lists' placement of true IDs
(``synth.posting_slots``) are inputs; the posting lists are encoded here with
Alg. 1's k-groups (``access.group_k``, ``access.encode_posting_lists_k``,
``access.rss_split_prf``).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

import synth

from . import access, fss, rss, shuffle


@dataclass
class Encoded:
    """The servers' view of a typed graph: shares[("id", T)] and
    shares[("attr", T, name)] (3, n_T, words) record-major; per type pair
    (T, T2) the posting lists' three shares (CSR records of ceil(n_T2/32)
    words) and their offsets."""
    shares: dict
    post: dict = field(default_factory=dict)
    off: dict = field(default_factory=dict)


def encode(tg, shares: dict, k: int, slot_seed: int, split_keys=(1001, 1002), counter: int = 4) -> Encoded:
    """Alg. 1 over the typed graph: per vertex type, its vertices grouped k at
    a time by the vector of their posting-list lengths (one group for all
    the type's list types, in sorted order of the neighbour type), each list
    padded to its group's longest; true IDs at the seeded slots (the e-th
    edge type in sorted order with slot seed slot_seed + e), records split
    into binary RSS with the PRF."""
    enc = Encoded(dict(shares))
    pairs = sorted(tg.adj)
    padded_of = {}
    for t in sorted({p[0] for p in pairs}):
        mine = [p for p in pairs if p[0] == t]
        lengths = np.array([[len(a) for a in tg.adj[p]] for p in mine], np.int64)
        padded, _ = access.group_k(lengths, np.zeros(lengths.shape[1], np.uint32), k)
        for row, p in enumerate(mine):
            padded_of[p] = padded[row]
    for e, (t, t2) in enumerate(pairs):
        lists = tg.adj[(t, t2)]
        lengths = np.array([len(a) for a in lists], np.uint32)
        padded = padded_of[(t, t2)]
        slots = synth.posting_slots(slot_seed + e, lengths, padded)
        rec, off = access.encode_posting_lists_k(lists, tg.n[t2], padded, slots)
        enc.post[(t, t2)] = access.rss_split_prf(rec, split_keys[0], split_keys[1], counter)
        enc.off[(t, t2)] = off
    return enc


@dataclass
class _Group:
    parent: object        # (hop, group, kept row) of the parent, None at hop 0
    ids: list             # three (n, wi) share tables of one-hot ID records
    vals: list            # three (n, wv) share tables of one-hot attribute records
    kept_ids: list = None # after secFetch: three (k, wi) tables


def _unpack(records: np.ndarray, nbits: int) -> np.ndarray:
    """(R, W) uint32 -> (R, nbits) 0/1."""
    return np.unpackbits(records.astype("<u4").view(np.uint8).reshape(records.shape[0], -1), axis=1,
                         bitorder="little")[:, :nbits]


def sec_match(tg, enc: Encoded, query, tok_seed: int, prf_keys, counter0: int, seed0: int):
    """Alg. 2 for a tree query (readings in the module doc).  Returns
    (results, groups): results is a list of per-target lists of three (wi,)
    share records; groups the per-target groups (for tests)."""
    counter, step = counter0, 0
    tg_n = tg.n
    q = len(query.targets)
    children = [[c for c in range(1, q) if query.parent(c) == i] for i in range(q)]
    t0 = query.targets[0]
    groups = [[] for _ in range(q)]
    groups[0].append(_Group(None, [enc.shares[("id", t0.vtype)][j] for j in range(3)],
                            [enc.shares[("attr", t0.vtype, t0.attr)][j] for j in range(3)]))
    for i, tgt in enumerate(query.targets):
        npos = tg.attrs[tgt.vtype][tgt.attr][1]
        keys, nb = rss.token(tgt.kind, npos, tok_seed, query.query_id, i, a=tgt.a, lo=tgt.lo, hi=tgt.hi)
        for gi, g in enumerate(groups[i]):
            n = g.ids[0].shape[0]
            if n == 0:
                g.kept_ids = [np.zeros((0, g.ids[0].shape[1]), np.uint32) for _ in range(3)]
                continue
            # secEval: each server's additive share, re-shared into RSS
            bits = np.stack([_unpack(g.vals[j], npos) for j in range(3)])
            x3 = rss.server_shares(tgt.kind, npos, keys, nb, bits)
            z = rss.reshare([fss.pack_bits(x3[j]) for j in range(3)], prf_keys, counter, n)
            counter += 1
            zb = [fss.unpack_bits(z[j], n) for j in range(3)]
            # secFetch Case II on {x || id || d}
            wi = g.ids[0].shape[1]
            rows = [np.concatenate([g.ids[j], g.vals[j]], axis=1) for j in range(3)]
            _, kept = shuffle.fetch_case2(zb, rows, seed0 + 3 * step, seed0 + 3 * step + 1, seed0 + 3 * step + 2)
            step += 1
            g.kept_ids = [kept[j][:, :wi] for j in range(3)]
        # secAccess of every kept vertex of every group, for each child target
        for gi, g in enumerate(groups[i]):
            for c in children[i]:
                nt = query.targets[c]
                pair = (tgt.vtype, nt.vtype)
                attr_sh = [enc.shares[("attr", nt.vtype, nt.attr)][j] for j in range(3)]
                for r in range(g.kept_ids[0].shape[0]):
                    idm = [_unpack(g.kept_ids[j][r:r + 1], tg_n[tgt.vtype])[0] for j in range(3)]
                    seeds = (seed0 + 3 * step, seed0 + 3 * step + 1, seed0 + 3 * step + 2)
                    ids_ne, vals_ne = access.sec_access_csr(idm, enc.post[pair], enc.off[pair], attr_sh,
                                                            tg_n[nt.vtype], prf_keys, seeds, counter)
                    counter += 2
                    step += 1
                    groups[c].append(_Group((i, gi, r), list(ids_ne), list(vals_ne)))
    return _results(groups, query), groups


def _results(groups, query):
    """Every assignment of one kept vertex per target, each in the group its
    parent's vertex made (targets in index order)."""
    q = len(query.targets)
    out = []

    def walk(i, chosen):
        if i == q:
            out.append([[groups[t][gi].kept_ids[j][r] for j in range(3)] for t, (gi, r) in enumerate(chosen)])
            return
        if i == 0:
            cands = [0]
        else:
            p = query.parent(i)
            cands = [gi for gi, g in enumerate(groups[i]) if g.parent == (p,) + chosen[p]]
        for gi in cands:
            g = groups[i][gi]
            for r in range(g.kept_ids[0].shape[0] if g.kept_ids is not None else 0):
                walk(i + 1, chosen + [(gi, r)])

    if groups[0]:
        walk(0, [])
    return out


def reconstruct(tg, query, chains) -> set:
    """Client side: the vertex ID of every target of every result (the one
    set bit of the XOR of the three shares), results using a vertex twice
    dropped."""
    out = set()
    for ch in chains:
        ids = []
        for tgt, rec in zip(query.targets, ch):
            bits = _unpack((rec[0] ^ rec[1] ^ rec[2])[None, :], tg.n[tgt.vtype])[0]
            pos = np.flatnonzero(bits)
            assert pos.size == 1, "a kept record is not one-hot"
            ids.append(int(pos[0]))
        verts = [(t.vtype, v) for t, v in zip(query.targets, ids)]
        if len(set(verts)) == len(verts):
            out.add(tuple(ids))
    return out


def brute_force(tg, query) -> set:
    """Plaintext matching (Def. 2) of a tree query over the typed graph: every
    assignment v_0, ..., v_{q-1} with v_i of type T_i, its predicate holding on
    v_i's attribute, v_i a neighbour of v_{parent(i)}, and no vertex used
    twice."""
    t = query.targets
    ok = [[v for v in range(tg.n[x.vtype]) if x.holds(tg.attrs[x.vtype][x.attr][0][v])] for x in t]
    nbrs = {pair: [set(a.tolist()) for a in lists] for pair, lists in tg.adj.items()}

    def linked(i, combo):
        p = query.parent(i)
        lists = nbrs.get((t[p].vtype, t[i].vtype))
        return lists is not None and combo[i] in lists[combo[p]]

    out = set()
    for combo in itertools.product(*ok):
        if not all(linked(i, combo) for i in range(1, len(t))):
            continue
        verts = [(x.vtype, v) for x, v in zip(t, combo)]
        if len(set(verts)) == len(verts):
            out.add(tuple(combo))
    return out


def plaintext_match(tg, query) -> set:
    """The same matching as ``brute_force``, found by walking the adjacency
    from each root candidate (target by target in index order, each target's
    vertex among its parent's neighbours) instead of trying every tuple: for
    typed graphs too large for the product.  Equal to ``brute_force`` on small
    graphs (pinned in the tests)."""
    t = query.targets
    ok = [{v for v in range(tg.n[x.vtype]) if x.holds(tg.attrs[x.vtype][x.attr][0][v])} for x in t]
    out = set()

    def walk(i, chosen, used):
        if i == len(t):
            out.add(tuple(chosen))
            return
        p = query.parent(i)
        lists = tg.adj.get((t[p].vtype, t[i].vtype))
        if lists is None:
            return
        for v in lists[chosen[p]].tolist():
            if v in ok[i] and (t[i].vtype, v) not in used:
                walk(i + 1, chosen + [v], used | {(t[i].vtype, v)})

    for r in sorted(ok[0]):
        walk(1, [r], {(t[0].vtype, r)})
    return out


def join_on_first(a: set, b: set, types_a, types_b) -> set:
    """Client-side join of two path results that share their first query
    vertex (a tree query split into root-to-leaf paths, as Fig. 1's): every
    pair with the same root and no other vertex in common (vertices compared
    by type and ID), as the root, then a's other vertices, then b's."""
    out = set()
    for x in a:
        va = {(t, v) for t, v in zip(types_a[1:], x[1:])}
        for y in b:
            if x[0] == y[0] and not va & {(t, v) for t, v in zip(types_b[1:], y[1:])}:
                out.add(x + y[1:])
    return out
