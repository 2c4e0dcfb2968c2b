"""hipGraph capture of one query's per-call pipeline -- the open and dealer
keygen of every predicate, then match_query (both parties' evaluation and
the ANDs) -- and its replay.  The pipeline holds no memset, no host copy and
no host wait, so it can be captured whole; a replay redoes the same work
(same seeds, so the same keys) and must give the eager result bit for bit,
every time, with eager work and synchronisations between the replays."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from gpu_util import DEV, U

pytestmark = pytest.mark.gpu

SEED = 4242


@pytest.fixture(scope="module")
def fss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_03526_amd import fss as lib
    torch.cuda.set_device(0)
    return lib


def _pipeline(fss, n, seed):
    graph, query = synth.config2(seed, n=n)
    shares = synth.share_columns(seed, graph.vcols)
    masks = synth.pred_masks(seed, query, graph)

    def T(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(DEV)

    preds = []
    for k, p in enumerate(query.preds):
        x0, x1 = shares[p.column]
        kind = fss.EQ if p.kind == "eq" else fss.RANGE
        preds.append({"p": p, "k": k, "x0": T(x0), "x1": T(x1), "r": T(masks[k]),
                      "xhat": torch.empty(n, dtype=torch.int32, device=DEV),
                      "kb": fss.KeyBatch(kind, 32, n, DEV)})
    plan = fss.Plan(seed, query.query_id, 1, n, 0, [(0, d["kb"], d["xhat"]) for d in preds]).allocate(DEV)

    def step():
        for d in preds:
            p = d["p"]
            fss.fss_mask_open(d["x0"], d["x1"], d["r"], d["xhat"])
            fss.fss_keygen(seed, query.query_id, d["k"], p.a if p.kind == "eq" else p.lo, p.hi, d["r"], d["kb"])
        fss.match_query(plan, 3)

    return plan, step


@pytest.mark.parametrize("n", [1 << 12, (1 << 16) + 37])
def test_captured_query_pipeline_replays_bit_exact(fss, n):
    plan, step = _pipeline(fss, n, SEED + n)
    other_plan, other_step = _pipeline(fss, 3000, SEED + 1)
    step()
    torch.cuda.synchronize()
    want = [o.clone() for o in plan.out]
    # warm up on a side stream, as capture wants, then capture on torch's capture stream
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    other_want = None
    for rep in range(4):
        for o in plan.out:
            o.zero_()                     # a replay that did nothing would leave zeros
        other_step()                      # eager work of another query between replays
        torch.cuda.synchronize()
        if other_want is None:
            other_want = [o.clone() for o in other_plan.out]
        g.replay()
        torch.cuda.synchronize()
        for b in range(2):
            assert torch.equal(plan.out[b], want[b]), (rep, b)
            assert torch.equal(other_plan.out[b], other_want[b]), (rep, b)


def _batch_requests(fss, seed, count):
    """Equality and range requests of uneven sizes, with their keys made eagerly."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        kind = fss.EQ if i % 2 == 0 else fss.RANGE
        n = int(rng.integers(1, 20000))
        r = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        x = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        a, hi = (int(x[n // 2]), 0) if kind == fss.EQ else sorted((int(x[0]), int(x[-1])))
        xhat = (x.astype(np.uint64) + r).astype(np.uint32)

        def T(v):
            return torch.from_numpy(v.view(np.int32)).to(DEV)
        kb = fss.KeyBatch(kind, 32, n, DEV)
        for t in kb.key:
            t.zero_()                     # pad rows are never written: keep them comparable
        reqs.append(dict(kind=kind, n=n, seed=seed + i, a=a, hi=hi, r=T(r), xhat=T(xhat), kb=kb))
    return reqs


def test_captured_batch_calls_replay_bit_exact(fss):
    """The batch calls under capture: more descriptors than a launch carries
    inline, so they are uploaded, and under capture that upload goes by
    kernel arguments.  A graph of one keygen batch and one eval batch replays
    bit for bit four times, with another batch's eager calls (which use the
    pinned staging ring) between the replays."""
    reqs = _batch_requests(fss, 77, 12)
    other = _batch_requests(fss, 99, 12)
    outs = [[torch.empty((rq["n"] + 31) // 32, dtype=torch.int32, device=DEV) for _ in range(2)] for rq in reqs]
    other_outs = [[torch.empty((rq["n"] + 31) // 32, dtype=torch.int32, device=DEV) for _ in range(2)]
                  for rq in other]
    kq, eq = fss.Queue(len(reqs)), fss.Queue(2 * len(reqs))
    okq, oeq = fss.Queue(len(other)), fss.Queue(2 * len(other))

    def run(rs, os_, kqueue, equeue):
        fss.fss_keygen_batch([(rq["seed"], 5, i, rq["a"], rq["hi"], rq["r"], rq["kb"]) for i, rq in enumerate(rs)],
                             kqueue)
        fss.fss_eval_batch([(b, rq["kb"], rq["xhat"], o[b]) for rq, o in zip(rs, os_) for b in range(2)], equeue)

    run(reqs, outs, kq, eq)
    torch.cuda.synchronize()
    want = [[o.clone() for o in pair] for pair in outs]
    keys = [[rq["kb"].key[b].clone() for b in range(2)] for rq in reqs]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run(reqs, outs, kq, eq)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run(reqs, outs, kq, eq)
    torch.cuda.synchronize()
    for rep in range(4):
        for pair in outs:
            for o in pair:
                o.zero_()
        for rq in reqs:
            for b in range(2):
                rq["kb"].key[b].zero_()
        run(other, other_outs, okq, oeq)          # eager batches through the staging ring
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, rq in enumerate(reqs):
            for b in range(2):
                assert torch.equal(rq["kb"].key[b], keys[i][b]), (rep, i, b)
                assert torch.equal(outs[i][b], want[i][b]), (rep, i, b)


def test_captured_query_batch_replays_bit_exact(fss):
    """One keygen batch and one match_query_batch for 8 uneven queries over a
    Chung-Lu graph (their descriptors uploaded as kernel arguments under
    capture), captured and replayed three times with another batch's eager
    calls between: every replay gives the eager outputs bit for bit."""
    from gpu_util import column_shares, plan_outputs
    from test_gpu_batch import _setup_query
    g = synth.Graph(1 << 14, *synth.chung_lu_graph(8, 1 << 14, 1 << 17), synth.vertex_table(8, 1 << 14), {})
    rng = np.random.default_rng(8)
    g.ecols = {"label": rng.integers(0, 4, g.n_edges, dtype=np.uint32),
               "weight": rng.integers(0, 1 << 16, g.n_edges, dtype=np.uint32)}
    shares = column_shares(g, 88)
    seed = 3131

    def batch(mix_seed):
        mix = synth.batch_queries(mix_seed, g, count=8, min_log_rows=8, max_log_rows=14)
        plans, kgs, meta = [], [], []
        for q, rows in mix:
            view, erows = synth.candidate_view(g, rows)
            vsh = synth.view_shares(shares, g, view, erows)
            masks = synth.pred_masks(seed, q, view)
            plan, kg = _setup_query(fss, view, q, vsh, masks, seed)
            plans.append(plan)
            kgs.extend(kg)
            meta.append((q, view))
        kq, mq = fss.Queue(len(kgs)), fss.Queue(sum(2 * p.c.n_pred for p in plans))

        def run():
            fss.fss_keygen_batch(kgs, kq)
            fss.match_query_batch(plans, mq)
        return plans, meta, run

    plans, meta, run = batch(11)
    o_plans, o_meta, o_run = batch(12)
    run()
    o_run()
    torch.cuda.synchronize()
    want = [plan_outputs(p, q, v) for p, (q, v) in zip(plans, meta)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        run()
    torch.cuda.synchronize()
    for rep in range(3):
        for p in plans:
            for o in p.out:
                o.zero_()
        o_run()                            # another batch, eager, through the staging ring
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for i, (p, (q, v)) in enumerate(zip(plans, meta)):
            got = plan_outputs(p, q, v)
            for j, (a, b) in enumerate(zip(got, want[i])):
                np.testing.assert_array_equal(a[0], b[0], err_msg=f"replay {rep} query {i} output {j}")
                np.testing.assert_array_equal(a[1], b[1], err_msg=f"replay {rep} query {i} output {j}")


@pytest.mark.parametrize("n,w", [(1000, 4), (5000, 4), ((1 << 16) + 37, 16)])
def test_captured_shuffle_replays_bit_exact(fss, n, w):
    """rss_shuffle and its two parts (prepare, prepared) captured into one
    graph: under capture the permutations stay on the caller's stream and use
    no memset, so every replay -- with eager shuffles of another table and
    synchronisations between the replays -- gives the oracle's shares.  1000
    records of 4 words take the one-workgroup shuffle, the others the wide
    launches with bucket permutations."""
    from oracle import shuffle as osh
    rng = np.random.default_rng(n + w)
    sh = [rng.integers(0, 2**32, (n, w), dtype=np.uint64).astype(np.uint32) for _ in range(3)]

    def T(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(DEV)

    d3 = [T(x.ravel()) for x in sh]
    seeds = (71, 72, 73)
    want = osh.sec_shuffle(sh, *seeds)
    out = [torch.empty(n * w, dtype=torch.int32, device=DEV) for _ in range(3)]
    out2 = [torch.empty(n * w, dtype=torch.int32, device=DEV) for _ in range(3)]
    perms = torch.empty(3 * n, dtype=torch.int32, device=DEV)
    m, mw = 3001, 3
    other = [T(rng.integers(0, 2**32, m * mw, dtype=np.uint64).astype(np.uint32)) for _ in range(3)]
    other_out = [torch.empty(m * mw, dtype=torch.int32, device=DEV) for _ in range(3)]
    other_want = osh.sec_shuffle([U(o).reshape(m, mw) for o in other], 5, 6, 7)

    def step():
        fss.rss_shuffle(n, w, d3, seeds, out)
        fss.rss_shuffle_prepare(n, seeds, perms)
        fss.rss_shuffle_prepared(n, w, d3, seeds, perms, out2)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    for rep in range(3):
        for o in out + out2:
            o.zero_()
        perms.zero_()
        fss.rss_shuffle(m, mw, other, (5, 6, 7), other_out)     # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(3):
            np.testing.assert_array_equal(U(out[i]).reshape(n, w), want[i], err_msg=f"replay {rep}")
            np.testing.assert_array_equal(U(out2[i]).reshape(n, w), want[i], err_msg=f"replay {rep}")
            np.testing.assert_array_equal(U(other_out[i]).reshape(m, mw), other_want[i])


def test_shuffle_capture_refuses_radix_permutations(fss):
    """With a radix permutation method the shuffle would record memset nodes:
    under capture it returns FSS_EUNSUPPORTED and enqueues nothing."""
    n, w = 5000, 2
    d3 = [torch.zeros(n * w, dtype=torch.int32, device=DEV) for _ in range(3)]
    out = [torch.empty(n * w, dtype=torch.int32, device=DEV) for _ in range(3)]
    work = torch.empty(int(fss.LIB.rss_shuffle_workspace_bytes(n, w)), dtype=torch.uint8, device=DEV)
    marker = torch.zeros(1, dtype=torch.int32, device=DEV)
    seeds = (ctypes.c_uint64 * 3)(1, 2, 3)
    fss.set_shuffle_tuning(1)
    try:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            rc = fss.LIB.rss_shuffle(n, w, fss._ptr3(d3), seeds, fss._ptr3(out), work.data_ptr(), work.numel(),
                                     torch.cuda.current_stream().cuda_stream)
            marker.add_(1)
        assert rc == fss.EUNSUPPORTED and b"capture" in fss.LIB.fss_last_error()
    finally:
        fss.set_shuffle_tuning(2)
    g.replay()
    torch.cuda.synchronize()
    assert int(marker.item()) == 1
