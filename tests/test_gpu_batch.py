"""The batched path (persistent work-queue launches) gives bit-identical
results to the per-request calls, whatever the tile / occupancy tuning, and
a batch of uneven queries over a power-law graph matches both the sequential
per-query path and the oracle on sampled rows."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import DEV, B, T, U, column_shares, job_inputs, plan_outputs
from oracle import fss as ofss
from oracle import match as omatch

pytestmark = pytest.mark.gpu

TUNINGS = [(1, 2), (2, 2), (4, 1), (1, 1), (8, 2)]


@pytest.fixture(scope="module")
def fss():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_03526_amd import fss as lib
    torch.cuda.set_device(0)
    yield lib
    lib.set_tuning(1, 2)
    lib.set_keygen_tuning(1)


def _rand_u32(seed, n):
    return np.random.default_rng(seed).integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)


REQS = [(0, 32, 70000), (1, 32, 3000), (1, 8, 65), (0, 12, 1), (1, 32, 1), (0, 32, 4097), (1, 12, 40000),
        (0, 8, 300)]


def _requests(fss):
    out = []
    for i, (kind, nbits, n) in enumerate(REQS):
        m = (1 << nbits) - 1 if nbits < 32 else 0xFFFFFFFF
        r = _rand_u32(10 + i, n)
        x = _rand_u32(20 + i, n) & np.uint32(m)
        if kind == 0:
            a, hi = int(x[n // 2]), 0
        else:
            a, hi = sorted((int(x[0]), int(x[-1])))
        xhat = (x.astype(np.uint64) + r).astype(np.uint32)
        out.append(dict(kind=kind, nbits=nbits, n=n, seed=1000 + i, q=3, p=i, a=a, hi=hi, r=T(r), xhat=T(xhat), x=x))
    return out


@pytest.mark.parametrize("tile_mult", [1, 3, 8])
@pytest.mark.parametrize("wg_per_cu", [1, 2])
def test_keygen_batch_equals_single(fss, tile_mult, wg_per_cu):
    """Keygen batches equal the per-request calls at every keygen tile size
    (512 to 4096 rows, requests of 1 to 70,000 rows) and grid size."""
    reqs = _requests(fss)
    single, batch = [], []
    for rq in reqs:
        kb = fss.KeyBatch(rq["kind"], rq["nbits"], rq["n"])
        fss.fss_keygen(rq["seed"], rq["q"], rq["p"], rq["a"], rq["hi"], rq["r"], kb)
        single.append(kb)
        batch.append(fss.KeyBatch(rq["kind"], rq["nbits"], rq["n"]))
    queue = fss.Queue(len(reqs))
    fss.set_keygen_tuning(tile_mult)
    fss.set_tuning(1, wg_per_cu)
    fss.fss_keygen_batch([(rq["seed"], rq["q"], rq["p"], rq["a"], rq["hi"], rq["r"], kb)
                          for rq, kb in zip(reqs, batch)], queue)
    torch.cuda.synchronize()
    fss.set_keygen_tuning(1)
    fss.set_tuning(1, 2)
    # compare the rows' keys (pad rows up to the next multiple of 64 are never written)
    from keylayout import from_device
    for rq, kb1, kb2 in zip(reqs, single, batch):
        nb = kb1.bytes_per_party
        for b in range(2):
            k1 = from_device(rq["kind"], rq["nbits"], rq["n"], B(kb1.key[b], nb))
            k2 = from_device(rq["kind"], rq["nbits"], rq["n"], B(kb2.key[b], nb))
            assert k1.tobytes() == k2.tobytes()


def test_keygen_and_eval_batch_equal_oracle(fss):
    """The batch calls against the oracle directly (not only through the
    single calls): keys of every request, in row chunks with row offsets (the
    serving runner's form), byte for byte equal to the oracle's keygen of the
    same table rows, and each party's evaluation words equal to the oracle's."""
    from keylayout import from_device
    reqs = _requests(fss)
    kg, ev, checks = [], [], []
    for rq in reqs:
        n = rq["n"]
        cut = n // 2 // 64 * 64 if n > 128 else 0     # two chunks where the table allows (offsets keep 64-row pads)
        for c0, c1 in ((0, cut), (cut, n)) if cut else ((0, n),):
            kb = fss.KeyBatch(rq["kind"], rq["nbits"], c1 - c0)
            kg.append((rq["seed"], rq["q"], rq["p"], rq["a"], rq["hi"], rq["r"][c0:c1], kb, c0))
            outs = [torch.full(((c1 - c0 + 31) // 32,), -1, dtype=torch.int32, device=DEV) for _ in range(2)]
            for b in range(2):
                ev.append((b, kb, rq["xhat"][c0:c1], outs[b]))
            checks.append((rq, c0, c1, kb, outs))
    fss.fss_keygen_batch(kg, fss.Queue(len(kg)))
    fss.fss_eval_batch(ev, fss.Queue(len(ev)))
    torch.cuda.synchronize()
    for rq, c0, c1, kb, outs in checks:
        r = U(rq["r"])[c0:c1]
        xh = U(rq["xhat"])[c0:c1]
        rows = np.arange(c0, c1, dtype=np.uint32)
        if rq["kind"] == 0:
            want = ofss.keygen_eq(rq["nbits"], rq["seed"], rq["q"], rq["p"], rq["a"], r, rows=rows)
            ev_fn = ofss.eval_eq
        else:
            want = ofss.keygen_range(rq["nbits"], rq["seed"], rq["q"], rq["p"], rq["a"], rq["hi"], r, rows=rows)
            ev_fn = ofss.eval_range
        for b in range(2):
            got = from_device(rq["kind"], rq["nbits"], c1 - c0, B(kb.key[b], kb.bytes_per_party))
            assert got.tobytes() == want[b].tobytes(), f"request {rq['p']} rows {c0}..{c1} party {b} keys"
            np.testing.assert_array_equal(U(outs[b]), ofss.pack_bits(ev_fn(rq["nbits"], b, want[b], xh)))


@pytest.mark.parametrize("tuning", TUNINGS)
def test_eval_batch_equals_single(fss, tuning):
    reqs = _requests(fss)
    evs = []
    for rq in reqs:
        kb = fss.KeyBatch(rq["kind"], rq["nbits"], rq["n"])
        fss.fss_keygen(rq["seed"], rq["q"], rq["p"], rq["a"], rq["hi"], rq["r"], kb)
        nw = (rq["n"] + 31) // 32
        for b in range(2):
            o1 = torch.full((nw,), 7, dtype=torch.int32, device=DEV)
            o2 = torch.full((nw,), 9, dtype=torch.int32, device=DEV)
            (fss.fss_eval_eq if rq["kind"] == 0 else fss.fss_eval_lt)(b, kb, rq["xhat"], o1)
            evs.append((b, kb, rq, o1, o2))
    fss.set_tuning(*tuning)
    queue = fss.Queue(len(evs))
    fss.fss_eval_batch([(b, kb, rq["xhat"], o2) for b, kb, rq, o1, o2 in evs], queue)
    torch.cuda.synchronize()
    fss.set_tuning(1, 2)
    for b, kb, rq, o1, o2 in evs:
        assert np.array_equal(U(o1), U(o2))
    # reconstruction is the plaintext predicate
    for i in range(0, len(evs), 2):
        _, _, rq, s0, _ = evs[i]
        s1 = evs[i + 1][3]
        rec = ofss.unpack_bits(U(s0) ^ U(s1), rq["n"])
        x = rq["x"].astype(np.uint64)
        truth = (x == rq["a"]) if rq["kind"] == 0 else ((x >= rq["a"]) & (x < rq["hi"]))
        np.testing.assert_array_equal(rec, truth.astype(np.uint8))


def _setup_query(fss, graph, q, shares, masks, seed):
    preds, kg = [], []
    for k, p in enumerate(q.preds):
        on_edge = p.target >= q.n_qv
        x0, x1 = shares[("e:" if on_edge else "") + p.column]
        rows = graph.n_edges if on_edge else graph.n_vertices
        r = T(masks[k]) if rows else torch.zeros(1, dtype=torch.int32, device=DEV)
        xhat = torch.empty(max(rows, 1), dtype=torch.int32, device=DEV)
        if rows:
            fss.fss_mask_open(T(x0), T(x1), r, xhat)
        kb = fss.KeyBatch(fss.EQ if p.kind == "eq" else fss.RANGE, 32, rows)
        kg.append((seed, q.query_id, k, p.a if p.kind == "eq" else p.lo, p.hi, r, kb))
        preds.append((p.target, kb, xhat))
    src = T(graph.src) if graph.n_edges else None
    dst = T(graph.dst) if graph.n_edges else None
    plan = fss.Plan(seed, q.query_id, q.n_qv, graph.n_vertices, graph.n_edges, preds, src, dst,
                    q.edges).allocate()
    return plan, kg


def test_uneven_query_batch(fss):
    """Uneven queries (1-5 predicates, 1-4 query vertices, candidate tables of
    2^8..2^16 rows) over a Chung-Lu graph: one keygen launch and one eval
    launch for all of them equal 16 sequential per-query pipelines."""
    g = synth.Graph(1 << 16, *synth.chung_lu_graph(5, 1 << 16, 1 << 19),
                    synth.vertex_table(5, 1 << 16), {})
    rng = np.random.default_rng(5)
    g.ecols = {"label": rng.integers(0, 4, g.n_edges, dtype=np.uint32),
               "weight": rng.integers(0, 1 << 16, g.n_edges, dtype=np.uint32)}
    shares = column_shares(g, 55)
    mix = synth.batch_queries(7, g, count=16, min_log_rows=8, max_log_rows=16)
    seed = 9090
    views, seq_out, plans, kgs = [], [], [], []
    for q, rows in mix:
        view, erows = synth.candidate_view(g, rows)
        vsh = synth.view_shares(shares, g, view, erows)
        masks = synth.pred_masks(seed, q, view)
        views.append((view, vsh, masks))
        plan, kg = _setup_query(fss, view, q, vsh, masks, seed)
        for args in kg:
            fss.fss_keygen(*args)
        fss.match_query(plan)
        torch.cuda.synchronize()
        seq_out.append(plan_outputs(plan, q, view))
        plan2, kg2 = _setup_query(fss, view, q, vsh, masks, seed)
        plans.append(plan2)
        kgs.extend(kg2)
    fss.fss_keygen_batch(kgs, fss.Queue(len(kgs)))
    fss.match_query_batch(plans, fss.Queue(sum(2 * p.c.n_pred for p in plans)))
    torch.cuda.synchronize()
    checked = 0
    for i, ((q, rows), (view, vsh, masks), plan) in enumerate(zip(mix, views, plans)):
        got = plan_outputs(plan, q, view)
        for j, (a, b) in enumerate(zip(got, seq_out[i])):
            np.testing.assert_array_equal(a[0], b[0], err_msg=f"query {i} output {j}")
            np.testing.assert_array_equal(a[1], b[1], err_msg=f"query {i} output {j}")
        if i % 5 == 0:
            nrows = view.n_vertices if q.n_qv == 1 else view.n_edges
            if nrows:
                rows_s = np.unique(np.random.default_rng(i).integers(0, nrows, 24))
                want = omatch.sampled_outputs(32, seed, view, q, vsh, masks, rows_s)
                for j, o in enumerate(got):
                    for b in range(2):
                        np.testing.assert_array_equal(ofss.unpack_bits(o[b], nrows)[rows_s], want[j, b])
                checked += 1
    assert checked >= 2


def test_chunked_runner_matches_whole_table(fss):
    """Waves of 4,096-row chunks under a key budget smaller than the jobs' keys
    give the same shares as whole-table calls (dealer randomness is addressed by
    table row)."""
    from paper_2209_03526_amd.runner import ChunkedRunner
    g, q = synth.config1(1)
    seed = 4242
    shares = column_shares(g, seed)
    masks = synth.pred_masks(seed, q, g)
    want = omatch.run_plan(32, seed, g, q, shares, masks)
    tiny = synth.tiny_graph(2, n_vertices=12, n_edges=30)
    tq = synth.Query(5, 3, [synth.Pred(0, "range", "attr", lo=2, hi=14), synth.Pred(1, "eq", "label", a=1),
                            synth.Pred(3, "range", "weight", lo=0, hi=12), synth.Pred(2, "range", "attr", lo=4, hi=16)])
    tsh = column_shares(tiny, 7)
    tm = synth.pred_masks(7, tq, tiny)
    twant = omatch.run_plan(32, 7, tiny, tq, tsh, tm)
    jobs = [job_inputs(fss, g, q, shares, masks, seed), job_inputs(fss, tiny, tq, tsh, tm, 7)]
    # the budget holds the largest chunk's keys (both parties) but well under
    # half of all keys, so the run needs several waves
    chunk_keys = [2 * fss.fss_keybatch_bytes(p["kind"], 32, min(4096, p["rows"] - c0))
                  for job in jobs for p in job.preds for c0 in range(0, p["rows"], 4096)]
    budget = max(max(chunk_keys) + 4096, sum(chunk_keys) // 3)
    assert budget < sum(chunk_keys) // 2
    runner = ChunkedRunner(budget_bytes=budget, chunk_rows=4096)
    runner.run(jobs)
    torch.cuda.synchronize()
    assert runner.waves >= 2
    for job, qq, gg, ww in ((jobs[0], q, g, want), (jobs[1], tq, tiny, twant)):
        got = plan_outputs(job.plan, qq, gg)
        for j, (a, b) in enumerate(zip(got, ww)):
            np.testing.assert_array_equal(a[0], b[0])
            np.testing.assert_array_equal(a[1], b[1])


def test_shutdown_releases_and_library_stays_usable(fss):
    """fss_shutdown frees the staging ring; the next batch call re-creates it
    and gives the same keys (the rows' keys: pad rows are never written)."""
    from keylayout import from_device
    n = 3000
    r = T(np.random.default_rng(5).integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32))
    q = fss.Queue(8, DEV)
    outs = []
    for i in range(2):
        kb = fss.KeyBatch(fss.RANGE, 32, n, DEV)
        fss.fss_keygen_batch([(11, 1, 0, 5, 7000, r, kb, 0)], q)
        torch.cuda.synchronize()
        outs.append(from_device(1, 32, n, B(kb.key[0], kb.bytes_per_party)).tobytes())
        fss.shutdown()
    assert outs[0] == outs[1]
