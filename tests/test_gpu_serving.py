"""The serving loop: continuous batching with admission by device memory
gives, request by request, the same result shares as the plain one-at-a-time
path, whether a request is served alone or in the mix; sampled rows match the
oracle."""
import copy
import time

import numpy as np
import pytest
import torch

import synth
from gpu_util import DEV, column_shares
from oracle import fss as ofss
from oracle import match as omatch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_03526_amd import serving
    torch.cuda.set_device(0)
    nv, ne = 1 << 14, 1 << 17
    src, dst = synth.chung_lu_graph(9, nv, ne)
    g = synth.Graph(nv, src, dst, synth.vertex_table(9, nv), {})
    rng = np.random.default_rng(9)
    g.ecols = {"label": rng.integers(0, 4, ne, dtype=np.uint32),
               "weight": rng.integers(0, 1 << 16, ne, dtype=np.uint32)}
    sh = column_shares(g, 99)
    vsh = {k: v for k, v in sh.items() if not k.startswith("e:")}
    esh = {k[2:]: v for k, v in sh.items() if k.startswith("e:")}
    rg = serving.resident_graph(nv, ne, src, dst, vsh, esh, DEV)
    mix = synth.batch_queries(11, g, count=12, min_log_rows=8, max_log_rows=14)
    return serving, g, sh, rg, mix


def _requests(serving, mix, arrivals, seed=777):
    reqs = []
    for i, t in enumerate(arrivals):
        q, rows = mix[i % len(mix)]
        q = copy.deepcopy(q)
        q.query_id = 50000 + i
        reqs.append(serving.Request(i, float(t), q, rows, seed))
    return reqs


def _run(serving, path, reqs):
    start = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    path.run(reqs, start, t0)
    return [serving.outputs(r) for r in reqs]


def test_served_equals_plain_and_alone(env):
    serving, g, sh, rg, mix = env
    n = 24
    arrivals = serving.poisson_arrivals(400.0, n, 3)
    served = serving.ServedPath(rg, budget_bytes=3 << 30, key_arena_bytes=1 << 30, chunk_rows=4096, device=DEV)
    out_mix = _run(serving, served, _requests(serving, mix, arrivals))
    assert served.waves >= 2
    out_plain = _run(serving, serving.PlainPath(rg, device=DEV), _requests(serving, mix, arrivals))
    # alone: requests far apart, so each wave holds one request only
    alone = serving.ServedPath(rg, budget_bytes=3 << 30, key_arena_bytes=1 << 30, chunk_rows=1 << 20, device=DEV)
    out_alone = _run(serving, alone, _requests(serving, mix, np.arange(n) * 0.01))
    for i in range(n):
        for b in range(2):
            np.testing.assert_array_equal(out_mix[i][b], out_plain[i][b], err_msg=f"request {i}")
            np.testing.assert_array_equal(out_mix[i][b], out_alone[i][b], err_msg=f"request {i}")


def test_served_matches_oracle_on_sampled_rows(env):
    serving, g, sh, rg, mix = env
    reqs = _requests(serving, mix, serving.poisson_arrivals(300.0, 6, 4), seed=4242)
    served = serving.ServedPath(rg, budget_bytes=2 << 30, key_arena_bytes=512 << 20, chunk_rows=2048, device=DEV)
    outs = _run(serving, served, reqs)
    for req, out in zip(reqs, outs):
        view, erows = synth.candidate_view(g, req.rows)
        vsh = synth.view_shares(sh, g, view, erows)
        q = req.query
        masks = [ofss.masks(req.seed, q.query_id, k, synth.rows_of_target(view, q, p.target))
                 for k, p in enumerate(q.preds)]
        nrows = view.n_vertices if q.n_qv == 1 else view.n_edges
        if nrows == 0:
            continue
        rows = np.unique(np.random.default_rng(req.rid).integers(0, nrows, 16))
        want = omatch.sampled_outputs(32, req.seed, view, q, vsh, masks, rows)
        w = (nrows + 31) // 32
        for j in range(want.shape[0]):
            for b in range(2):
                got = ofss.unpack_bits(out[b][j * w:(j + 1) * w], nrows)[rows]
                np.testing.assert_array_equal(got, want[j, b])


def test_admission_respects_memory(env):
    """With a budget that fits the largest request but not two of them, the
    admitted bytes never exceed it, requests wait (fewer in flight than
    requests), and all complete in arrival order."""
    serving, g, sh, rg, mix = env
    reqs = _requests(serving, mix, np.zeros(8))
    for r in reqs:
        r.mem = serving.memory_bound(r)
    big = max(r.mem for r in reqs)
    arena = 64 << 20
    served = serving.ServedPath(rg, budget_bytes=arena + big, key_arena_bytes=arena, chunk_rows=4096, device=DEV)
    _run(serving, served, reqs)
    assert served.max_used <= big
    assert served.max_in_flight < len(reqs)
    assert all(r.done_event is not None for r in reqs)
    done = [r.latency_ms + 1e3 * r.arrival for r in reqs]
    assert all(a <= b for a, b in zip(done, done[1:]))


# --------------------------------------------------------------------------- token given

@pytest.fixture(scope="module")
def pool(env):
    serving, g, sh, rg, mix = env
    for i, (q, rows) in enumerate(mix):
        q.query_id = 60000 + i
    return serving.TokenPool(rg, mix, 2024, DEV)


def _given(serving, arrivals, n_entries, seed=5):
    entries = np.random.default_rng(seed).integers(0, n_entries, len(arrivals))
    return [serving.GivenRequest(i, float(t), int(e)) for i, (t, e) in enumerate(zip(arrivals, entries))]


def _run_given(serving, path, reqs, pool):
    start = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    path.run(reqs, start, t0)
    return [serving.given_outputs(r, pool) for r in reqs]


def test_given_served_equals_plain_and_alone(env, pool):
    """Token given: continuous batching gives, request by request, the shares
    of the one-at-a-time path and of the same request served alone."""
    serving, g, sh, rg, mix = env
    n = 40
    arrivals = serving.poisson_arrivals(2000.0, n, 6)
    served = serving.GivenServedPath(rg, pool, budget_bytes=2 << 30, device=DEV)
    out_mix = _run_given(serving, served, _given(serving, arrivals, len(mix)), pool)
    assert served.waves >= 2 and served.max_wave >= 2
    out_plain = _run_given(serving, serving.GivenPlainPath(rg, pool, device=DEV), _given(serving, arrivals, len(mix)),
                           pool)
    out_alone = _run_given(serving, serving.GivenServedPath(rg, pool, budget_bytes=2 << 30, device=DEV),
                           _given(serving, np.arange(n) * 0.01, len(mix)), pool)
    for i in range(n):
        for b in range(2):
            np.testing.assert_array_equal(out_mix[i][b], out_plain[i][b], err_msg=f"request {i}")
            np.testing.assert_array_equal(out_mix[i][b], out_alone[i][b], err_msg=f"request {i}")


def _oracle_rows(g, sh, q, rows, seed, out, rid, k=16):
    view, erows = synth.candidate_view(g, rows)
    vsh = synth.view_shares(sh, g, view, erows)
    masks = [ofss.masks(seed, q.query_id, j, synth.rows_of_target(view, q, p.target)) for j, p in enumerate(q.preds)]
    nrows = view.n_vertices if q.n_qv == 1 else view.n_edges
    if nrows == 0:
        return
    rows_ = np.unique(np.random.default_rng(rid).integers(0, nrows, k))
    want = omatch.sampled_outputs(32, seed, view, q, vsh, masks, rows_)
    w = (nrows + 31) // 32
    for j in range(want.shape[0]):
        for b in range(2):
            got = ofss.unpack_bits(out[b][j * w:(j + 1) * w], nrows)[rows_]
            np.testing.assert_array_equal(got, want[j, b], err_msg=f"request {rid} output {j} party {b}")


def test_given_served_matches_oracle(env, pool):
    serving, g, sh, rg, mix = env
    reqs = _given(serving, serving.poisson_arrivals(1000.0, 12, 8), len(mix), seed=9)
    served = serving.GivenServedPath(rg, pool, budget_bytes=2 << 30, device=DEV)
    outs = _run_given(serving, served, reqs, pool)
    for req, out in zip(reqs, outs):
        q, rows = mix[req.entry]
        _oracle_rows(g, sh, q, rows, 2024, out, req.rid)


def test_given_admission_respects_memory(env, pool):
    serving, g, sh, rg, mix = env
    reqs = _given(serving, np.zeros(10), len(mix), seed=10)
    big = max(serving.given_memory(pool.tokens[r.entry]) for r in reqs)
    served = serving.GivenServedPath(rg, pool, budget_bytes=big, device=DEV)
    _run_given(serving, served, reqs, pool)
    assert served.max_used <= big
    assert served.max_in_flight < len(reqs)
    done = [r.latency_ms for r in reqs]         # all arrived at 0: completion order = latency order
    assert all(a <= b for a, b in zip(done, done[1:]))


# --------------------------------------------------------------------------- full size

def test_given_served_full_size_matches_oracle():
    """The served path over the resident 2^22-vertex / 2^25-edge Chung-Lu graph:
    ten requests of the 64-shape mix (tokens of eight mix entries, two of them
    repeated), each checked against the oracle on sampled rows."""
    from paper_2209_03526_amd import serving
    g, _ = synth.config3(3)
    seed = 31
    vsh = synth.share_columns(seed, g.vcols)
    esh = synth.share_columns(seed + 1, g.ecols)
    rg = serving.resident_graph(g.n_vertices, g.n_edges, g.src, g.dst, vsh, esh, DEV)
    mix = synth.batch_queries(4, g, count=64)
    entries = [0, 5, 17, 23, 31, 42, 50, 63]
    sub = [mix[e] for e in entries]
    tokens = serving.TokenPool(rg, sub, seed, DEV)
    order = [0, 1, 2, 3, 4, 5, 6, 7, 2, 5]
    reqs = [serving.GivenRequest(i, 0.002 * i, e) for i, e in enumerate(order)]
    served = serving.GivenServedPath(rg, tokens, budget_bytes=64 * 10**9, device=DEV)
    outs = _run_given(serving, served, reqs, tokens)
    sh = dict(vsh)
    sh.update({"e:" + k: v for k, v in esh.items()})
    for req, out in zip(reqs, outs):
        q, rows = sub[req.entry]
        _oracle_rows(g, sh, q, rows, seed, out, req.rid, k=24)
    for i, j in ((2, 8), (5, 9)):             # a repeated token gives the same shares
        for b in range(2):
            np.testing.assert_array_equal(outs[i][b], outs[j][b])
