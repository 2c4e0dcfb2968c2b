"""Helpers for GPU tests: numpy <-> device tensors and query setup through the
library's C ABI.  No arithmetic of the method lives here."""
import numpy as np
import torch

import synth

DEV = "cuda:0"


def T(a, dtype=np.uint32):
    """numpy uint32 -> int32 device tensor with the same bits."""
    a = np.ascontiguousarray(a, dtype=dtype)
    return torch.from_numpy(a.view(np.int32)).to(DEV)


def U(t, n=None):
    """device tensor -> numpy uint32 (first n elements)."""
    a = t.detach().cpu().numpy().view(np.uint32)
    return a if n is None else a[:n]


def B(t, nbytes):
    return t.detach().cpu().numpy().view(np.uint8)[:nbytes]


def column_shares(graph, seed):
    sh = {k: synth.share_column(np.random.default_rng([seed, i]), v)
          for i, (k, v) in enumerate(sorted(graph.vcols.items()))}
    sh.update({"e:" + k: synth.share_column(np.random.default_rng([seed, 100 + i]), v)
               for i, (k, v) in enumerate(sorted(graph.ecols.items()))})
    return sh


def run_query_gpu(fss, graph, query, shares, masks, seed, nbits=32):
    """Dealer keygen + open + match_query through the C ABI; returns the plan
    (outputs in plan.out) and the per-predicate key batches."""
    preds = []
    for k, p in enumerate(query.preds):
        on_edge = p.target >= query.n_qv
        x0, x1 = shares[("e:" if on_edge else "") + p.column]
        rows = graph.n_edges if on_edge else graph.n_vertices
        r = T(masks[k])
        xhat = torch.empty(max(rows, 1), dtype=torch.int32, device=DEV)
        fss.fss_mask_open(T(x0), T(x1), r, xhat)
        kb = fss.KeyBatch(fss.EQ if p.kind == "eq" else fss.RANGE, nbits, rows)
        fss.fss_keygen(seed, query.query_id, k, p.a if p.kind == "eq" else p.lo, p.hi, r, kb)
        preds.append((p.target, kb, xhat))
    src = T(graph.src) if graph.n_edges else None
    dst = T(graph.dst) if graph.n_edges else None
    plan = fss.Plan(seed, query.query_id, query.n_qv, graph.n_vertices, graph.n_edges, preds, src, dst,
                    query.edges)
    plan.allocate()
    fss.match_query(plan)
    torch.cuda.synchronize()
    return plan


def plan_outputs(plan, query, graph):
    """[(party0 words, party1 words)] per output (hops, or the vertex result)."""
    if query.n_qv == 1:
        w = (graph.n_vertices + 31) // 32
        return [(U(plan.out[0], w), U(plan.out[1], w))]
    we = (graph.n_edges + 31) // 32
    o0, o1 = U(plan.out[0]), U(plan.out[1])
    return [(o0[j * we:(j + 1) * we], o1[j * we:(j + 1) * we]) for j in range(query.n_qe)]


def T_off(a, dtype=np.uint32):
    """Like T, but the data starts one word into its allocation (a view whose
    address is 4 bytes past a 16-byte boundary)."""
    a = np.ascontiguousarray(a, dtype=dtype)
    buf = torch.empty(a.size + 1, dtype=torch.int32, device=DEV)
    buf[1:].copy_(torch.from_numpy(a.view(np.int32)))
    return buf[1:]


def empty_off(n):
    """An uninitialised int32 device view of n words, 4 bytes past a 16-byte boundary."""
    return torch.empty(n + 1, dtype=torch.int32, device=DEV)[1:]


def job_inputs(fss, view, q, vsh, masks, seed):
    """A runner QueryJob for query q over a candidate view: masks and opened
    values on the device (one fss_mask_open per predicate)."""
    from paper_2209_03526_amd.runner import QueryJob
    preds = []
    for k, p in enumerate(q.preds):
        on_edge = p.target >= q.n_qv
        x0, x1 = vsh[("e:" if on_edge else "") + p.column]
        rows = view.n_edges if on_edge else view.n_vertices
        r = T(masks[k]) if rows else torch.zeros(1, dtype=torch.int32, device=DEV)
        xhat = torch.empty(max(rows, 1), dtype=torch.int32, device=DEV)
        if rows:
            fss.fss_mask_open(T(x0), T(x1), r, xhat)
        preds.append(dict(target=p.target, kind=fss.EQ if p.kind == "eq" else fss.RANGE, rows=rows,
                          a_or_lo=p.a if p.kind == "eq" else p.lo, hi=p.hi, r=r, xhat=xhat))
    src = T(view.src) if view.n_edges else None
    dst = T(view.dst) if view.n_edges else None
    return QueryJob(seed, q.query_id, q.n_qv, view.n_vertices, view.n_edges, preds, src, dst, edges=q.edges)
