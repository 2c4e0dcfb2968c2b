"""The paper's whole secure matching protocol, Alg. 2 (secMatch), over its own
encoding, on the GPU: for a tree query over a typed graph (a path V_1 -> V_2
-> ... -> V_q, or targets each hanging off an earlier one, as Fig. 1's),
target by target

  secEval (Alg. 3: full-domain evaluations of the replicated token,
           `fss_eval_all`; each server's two terms, `rss_sec_eval_records`),
  the re-share of its three-out-of-three bits into RSS (`rss_reshare`),
  secFetch Case II (Alg. 4: the table {x || id || d}, `rss_fetch_table`;
           shuffle, open, keep, `rss_fetch_many`),
  secAccess (Alg. 6, `rss_sec_access`) of every kept vertex's neighbours of
           the next target's type, over the k-grouped posting lists of Alg. 1
           (`rss_enc_posting_lists`).

All three servers are simulated on one device.  Every step runs in the
library's kernels; this module only orders the calls and reads the counts
that the opens of secFetch and secAccess reveal, two synchronisations per
target: one after all of the target's secFetch calls (their counts decide
how many secAccess calls follow), one after all of its secAccess calls (each
with its lmax-row capacity); between them the calls are enqueued back to
back.

Readings where Alg. 2 leaves the order open: a target's candidates are
grouped by the kept vertex (of its parent target) whose neighbours they are,
and secFetch runs once per group, so each kept vertex keeps its parent (the
final reorganisation into subgraphs needs that tie); targets run in index
order, and within a target every group's secEval, re-share and secFetch come
first (group order), then the secAccess calls of the kept vertices (group by
group, child target by child target);
re-shares take PRF counters in order from `counter0` (secEval's re-share one,
secAccess two); the s-th shuffle (secFetch's and secAccess's alike) takes the
seeds (seed0 + 3s, +1, +2); predicate i's token is made with pred = i; an
empty group takes no randomness.  A result is one kept vertex per target,
each in the group its parent's vertex made, as the three shares of each
target's one-hot ID record; the client reconstructs and drops results that
use a vertex twice.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import fss

# The token's replicated key pairs (Sec. V-C): server CS_1 holds (k_1^1, k_1^2),
# CS_2 (k_2^2, k_1^3), CS_3 (k_2^3, k_2^1); with the one-hot shares (<e>_i,
# <e>_{i+1}) each evaluates Eq. predEval's two terms.  Entries: (party of the
# key, replica j - 1, share index - 1) of each term.
SERVER_TERMS = (((0, 0, 0), (0, 1, 1)),
                ((1, 1, 1), (0, 2, 2)),
                ((1, 2, 2), (1, 0, 0)))


def words(bits: int) -> int:
    return (bits + 31) // 32


def domain_bits(npos: int) -> int:
    """Input width of the token's keys for positions 0 .. npos - 1 (at least 8)."""
    return max(8, int(np.ceil(np.log2(max(npos, 2)))))


@dataclass
class EncodedGraph:
    """A typed graph as the servers hold it, resident on one device: per type
    its vertex count; per attribute its domain size; the three shares of the
    one-hot ID and attribute records (record-major, ceil(n/32) words each);
    per edge type (T, T2) the posting lists (CSR, k-grouped) and offsets."""
    n: dict
    domains: dict
    shares: dict = field(default_factory=dict)
    post: dict = field(default_factory=dict)
    off: dict = field(default_factory=dict)
    lmax: dict = field(default_factory=dict)


def _dev(a: np.ndarray, device):
    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(device)


def padded_lengths(adj: dict, k: int) -> dict:
    """Alg. 1's padded list lengths per edge type (T, T2): each vertex type's
    vertices grouped k at a time over the vector of their list lengths, list
    types in sorted order of the neighbour type (`rss_group_k_lists`)."""
    out = {}
    for t in sorted({p[0] for p in adj}):
        mine = sorted(p for p in adj if p[0] == t)
        lengths = np.array([[len(a) for a in adj[p]] for p in mine], np.uint32)
        padded, _ = fss.rss_group_k_lists(lengths, np.zeros(lengths.shape[1], np.uint32), k)
        for row, p in enumerate(mine):
            out[p] = padded[row]
    return out


def encode_graph(n: dict, domains: dict, shares: dict, adj: dict, slots: dict, k: int, split_keys=(1001, 1002),
                 counter: int = 4, device=None) -> EncodedGraph:
    """The data owner's upload: the one-hot RSS records of IDs and attributes
    (`shares`: {("id", T) | ("attr", T, name): (3, n_T, words) uint32}) moved
    to the device, and Alg. 1 for every edge type (T, T2) of `adj` (lists of
    neighbour IDs per vertex of T): each vertex type's vertices grouped k at a
    time over the vector of their list lengths (`rss_group_k_lists`), true
    IDs at the owner's slots (`slots[(T, T2)]`, flat in adjacency order),
    one-hot records split into RSS with the PRF (`rss_enc_posting_lists`)."""
    dev = device or torch.device("cuda")
    eg = EncodedGraph(dict(n), dict(domains))
    for key, sh in shares.items():
        eg.shares[key] = [_dev(sh[j].ravel(), dev) for j in range(3)]
    padded_of = padded_lengths(adj, k)
    for (t, t2), lists in sorted(adj.items()):
        lengths = np.array([len(a) for a in lists], np.uint32)
        padded = padded_of[(t, t2)]
        off = np.concatenate([[0], np.cumsum(padded, dtype=np.uint64)]).astype(np.uint32)
        adj_off = np.concatenate([[0], np.cumsum(lengths, dtype=np.uint64)]).astype(np.uint32)
        flat = np.concatenate([np.asarray(a, np.uint32) for a in lists]) if lengths.sum() else np.zeros(1, np.uint32)
        nrec = int(off[-1])
        wx = words(n[t2])
        out = [torch.empty(max(1, nrec * wx), dtype=torch.int32, device=dev) for _ in range(3)]
        d_off = _dev(off, dev)
        if nrec:
            fss.rss_enc_posting_lists(len(lists), n[t2], _dev(adj_off, dev), _dev(flat, dev),
                                      _dev(np.asarray(slots[(t, t2)], np.uint32) if lengths.sum() else flat, dev),
                                      d_off, nrec, split_keys, counter, out)
        eg.post[(t, t2)] = out
        eg.off[(t, t2)] = d_off
        eg.lmax[(t, t2)] = max(1, int(padded.max()) if padded.size else 1)
    torch.cuda.synchronize(dev)
    return eg


@dataclass
class _Group:
    parent: object        # (hop, group, kept row) of the parent; None at hop 0
    n: int                # candidates
    ids: list             # three device tensors, n one-hot ID records
    vals: list            # three device tensors, n one-hot attribute records
    kept: list = None     # three device tensors of kept {id || d} records
    nkept: int = 0


def sec_match(eg: EncodedGraph, query, tok_seed: int, prf_keys, counter0: int, seed0: int, device=None):
    """Alg. 2 for a tree query (``query.targets``: vertex type, attribute,
    predicate per target; ``query.parent(i)``: the target that target i hangs
    off, i - 1 for a path; readings in the module doc).  Returns the results,
    each a list over targets of the three shares (numpy uint32 records) of the
    target's one-hot ID."""
    dev = device or torch.device("cuda")
    counter, step = counter0, 0
    q = len(query.targets)
    children = [[c for c in range(1, q) if query.parent(c) == i] for i in range(q)]
    t0 = query.targets[0]
    groups = [[] for _ in range(q)]
    groups[0].append(_Group(None, eg.n[t0.vtype], eg.shares[("id", t0.vtype)], eg.shares[("attr", t0.vtype, t0.attr)]))
    zero3 = torch.zeros(3, dtype=torch.int32, device=dev)
    for i, tgt in enumerate(query.targets):
        npos = eg.domains[(tgt.vtype, tgt.attr)]
        nb = domain_bits(npos)
        kind = fss.EQ if tgt.kind == "eq" else fss.RANGE
        kb = fss.KeyBatch(kind, nb, 3, dev)
        fss.fss_keygen(tok_seed, query.query_id, i, tgt.a if tgt.kind == "eq" else tgt.lo, tgt.hi, zero3, kb)
        ev = {}
        for party in (0, 1):
            for rep in range(3):
                ev[(party, rep)] = torch.empty(words(npos), dtype=torch.int32, device=dev)
                fss.fss_eval_all(party, kb, rep, npos, ev[(party, rep)])
        wi, wv = words(eg.n[tgt.vtype]), words(npos)
        rec = 1 + wi + wv
        live = [gi for gi, g in enumerate(groups[i]) if g.n > 0]
        # every group's secEval, re-share and secFetch, enqueued without waiting
        # (the temporaries are shared by the groups: one stream orders their uses)
        fetched = torch.zeros(max(len(live), 1), dtype=torch.int32, device=dev)
        nmax = max([groups[i][gi].n for gi in live], default=1)
        x3 = [torch.empty(words(nmax), dtype=torch.int32, device=dev) for _ in range(3)]
        z3 = [torch.empty(words(nmax), dtype=torch.int32, device=dev) for _ in range(3)]
        table = [torch.empty(nmax * rec, dtype=torch.int32, device=dev) for _ in range(3)]
        for k, gi in enumerate(live):
            g = groups[i][gi]
            # secEval, then the re-share into RSS
            for s, ((pa, ra, ja), (pb, rb, jb)) in enumerate(SERVER_TERMS):
                fss.rss_sec_eval_records(g.n, npos, ev[(pa, ra)], ev[(pb, rb)], g.vals[ja], g.vals[jb], x3[s])
            fss.rss_reshare(g.n, x3, prf_keys, counter, z3)
            counter += 1
            # secFetch Case II on {x || id || d}
            fss.rss_fetch_table(g.n, z3, wi, g.ids, wv, g.vals, table)
            g.kept = [torch.empty(g.n * (rec - 1), dtype=torch.int32, device=dev) for _ in range(3)]
            pos = torch.empty(g.n, dtype=torch.int32, device=dev)
            work = fss.rss_fetch_many(g.n, rec, table, (seed0 + 3 * step, seed0 + 3 * step + 1, seed0 + 3 * step + 2),
                                      g.kept, pos, fetched[k:k + 1])
            step += 1
            del work, pos                        # stream-ordered: reused only after these calls' kernels
        del x3, z3, table
        # the opens reveal how many candidates of each group match
        for k, m in enumerate(fetched.cpu().tolist()[:len(live)]):
            groups[i][live[k]].nkept = m
        # secAccess of every kept vertex of every group, for each child target:
        # call k (in this order) takes counter + 2k and shuffle step + k; the
        # calls of one child target go to the library as one batch, and the
        # validity opens' counts are read together
        calls = [(gi, c, r) for gi in live for c in children[i] for r in range(groups[i][gi].nkept)]
        made, batches = [None] * len(calls), []
        for c in children[i]:
            ks = [k for k, call in enumerate(calls) if call[1] == c]
            if not ks:
                continue
            nt = query.targets[c]
            pair = (tgt.vtype, nt.vtype)
            wx2, wv2 = words(eg.n[nt.vtype]), words(eg.domains[(nt.vtype, nt.attr)])
            lmax = eg.lmax[pair]
            nc = len(ks)
            idm, counters, seeds = [], [], []
            for k in ks:
                gi, _, r = calls[k]
                idm += [groups[i][gi].kept[j].data_ptr() + 4 * r * (rec - 1) for j in range(3)]
                counters.append(counter + 2 * k)
                seeds += [seed0 + 3 * (step + k) + j for j in range(3)]
            ids3 = [torch.empty(nc * lmax * wx2, dtype=torch.int32, device=dev) for _ in range(3)]
            vals3 = [torch.empty(nc * lmax * wv2, dtype=torch.int32, device=dev) for _ in range(3)]
            rows = torch.empty(nc * lmax, dtype=torch.int32, device=dev)
            cnt = torch.empty(nc, dtype=torch.int32, device=dev)
            work = fss.rss_sec_access_batch(eg.n[tgt.vtype], eg.n[nt.vtype], idm, eg.off[pair], lmax, eg.post[pair],
                                            wv2, eg.shares[("attr", nt.vtype, nt.attr)], prf_keys, counters, seeds,
                                            ids3, vals3, rows, cnt)
            batches.append((ks, cnt))
            del work, rows
            for q_, k in enumerate(ks):
                made[k] = ([t[q_ * lmax * wx2:(q_ + 1) * lmax * wx2] for t in ids3],
                           [t[q_ * lmax * wv2:(q_ + 1) * lmax * wv2] for t in vals3])
        counter += 2 * len(calls)
        step += len(calls)
        opened = [0] * len(calls)
        for ks, cnt in batches:              # the first read waits for all of them
            for k, m in zip(ks, cnt.cpu().tolist()):
                opened[k] = m
        for k, (gi, c, r) in enumerate(calls):
            groups[c].append(_Group((i, gi, r), opened[k], *made[k]))
    return _results(groups, query, eg)


def _results(groups, query, eg):
    """Every assignment of one kept vertex per target, each in the group its
    parent's vertex made (targets in index order), as host share records."""
    q = len(query.targets)
    out = []
    host = {}

    def kept_ids(i, gi):
        if (i, gi) not in host:
            g = groups[i][gi]
            t = query.targets[i]
            wi, wv = words(eg.n[t.vtype]), words(eg.domains[(t.vtype, t.attr)])
            host[(i, gi)] = [g.kept[j][:g.nkept * (wi + wv)].cpu().numpy().view(np.uint32).reshape(
                g.nkept, wi + wv)[:, :wi] for j in range(3)]
        return host[(i, gi)]

    def walk(i, chosen):
        if i == q:
            out.append([[kept_ids(t, gi)[j][r] for j in range(3)] for t, (gi, r) in enumerate(chosen)])
            return
        if i == 0:
            cands = [0]
        else:
            p = query.parent(i)
            cands = [gi for gi, g in enumerate(groups[i]) if g.parent == (p,) + chosen[p]]
        for gi in cands:
            for r in range(groups[i][gi].nkept):
                walk(i + 1, chosen + [(gi, r)])

    if groups[0]:
        walk(0, [])
    return out
