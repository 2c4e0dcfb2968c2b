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
    """With a budget that fits about one request at a time, requests queue in
    arrival order and all complete."""
    serving, g, sh, rg, mix = env
    reqs = _requests(serving, mix, np.zeros(8))
    big = max(serving.memory_bound(r) for r in reqs)
    served = serving.ServedPath(rg, budget_bytes=(64 << 20) + big, key_arena_bytes=64 << 20, chunk_rows=4096,
                                device=DEV)
    _run(serving, served, reqs)
    assert served.max_in_flight <= 8
    assert all(r.done_event is not None for r in reqs)
