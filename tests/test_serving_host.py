"""Host logic of the serving loop (admission, waves, memory release), run on
the CPU with the library calls and HIP events replaced by recorders: every
request completes, in arrival order, also when the memory budget admits one
request at a time (a request blocked on memory must see earlier requests'
memory returned)."""
import time
import types

import pytest
import torch

from paper_2209_03526_amd import serving


class FakeEvent:
    """Completes a fixed delay after it is recorded, like work on a stream."""
    delay = 0.003

    def __init__(self, enable_timing=True):
        self.t = None

    def record(self, stream=None):
        self.t = time.perf_counter() + self.delay

    def query(self):
        return self.t is not None and time.perf_counter() >= self.t

    def synchronize(self):
        while not self.query():
            time.sleep(0.0005)

    def elapsed_time(self, other):
        return 1e3 * (other.t - (self.t or other.t))


class FakeArena:
    def __init__(self, nbytes, device):
        self.nbytes, self.used = nbytes, 0

    def reset(self):
        self.used = 0

    def take(self, nbytes):
        nbytes = (nbytes + 255) // 256 * 256
        assert self.used + nbytes <= self.nbytes
        self.used += nbytes
        return self.used


def _fake_fss(log):
    f = types.SimpleNamespace(EQ=0, RANGE=1)
    f.fss_keybatch_bytes = lambda kind, nb, n: n * (432 if kind == 0 else 872)
    f.KeyBatch = types.SimpleNamespace(view=lambda kind, nb, n, p0, p1: (kind, n))
    f.Queue = lambda cap, dev: types.SimpleNamespace(capacity=cap)
    f.fss_keygen_batch = lambda kg, q, s: log.append(("keygen", [k[1] for k in kg]))
    f.fss_eval_batch = lambda ev, q, s: log.append(("eval", len(ev)))
    f.match_query_batch = lambda plans, q, w, s: log.append(("match", len(plans)))
    return f


def _prepare(req, g, device, stream=None):
    req.view = dict(n_vertices=req.rows, n_edges=0, src=None, dst=None)
    req.preds = [dict(target=0, kind=k % 2, rows=req.rows, a_or_lo=1, hi=5, r=torch.zeros(req.rows),
                      xhat=torch.zeros(req.rows)) for k in range(2)]
    return req


@pytest.fixture
def fake(monkeypatch):
    log = []
    monkeypatch.setattr(serving, "fss", _fake_fss(log))
    monkeypatch.setattr(serving, "KeyArena", FakeArena)
    monkeypatch.setattr(serving, "prepare", _prepare)
    monkeypatch.setattr(serving, "_plan", lambda req, given, dev: types.SimpleNamespace(release_inputs=lambda: None))
    monkeypatch.setattr(torch.cuda, "Event", FakeEvent)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a: None)
    return log


def _reqs(arrivals, rows=1000):
    return [serving.Request(i, float(t), types.SimpleNamespace(query_id=100 + i, n_qv=1, n_qe=0, edges=None, preds=[None, None]),
                            rows, 7) for i, t in enumerate(arrivals)]


def _run(path, reqs):
    start = FakeEvent()
    start.record()
    start.t -= FakeEvent.delay
    return path.run(reqs, start, time.perf_counter())


@pytest.mark.timeout(30)
def test_memory_bound_admission_completes_in_order(fake):
    reqs = _reqs([0.0] * 8)
    one = serving.memory_bound(reqs[0])
    arena = 4 << 20
    path = serving.ServedPath(None, budget_bytes=arena + one, key_arena_bytes=arena, chunk_rows=512,
                              device="cpu", stream=object())
    _run(path, reqs)
    assert all(r.done_event is not None for r in reqs)
    assert path.max_in_flight == 1
    # one request in memory at a time: its waves all come before the next one's
    order = [qid for kind, ids in fake if kind == "keygen" for qid in ids]
    assert order == sorted(order)
    assert [e for e in fake if e[0] == "match"] == [("match", 1)] * 8


@pytest.mark.timeout(30)
def test_continuous_batching_mixes_arrivals(fake):
    reqs = _reqs([0.0, 0.0, 0.0, 0.02, 0.02, 0.05])
    arena = 8 * 1000 * 872     # both parties' keys of about four chunks
    path = serving.ServedPath(None, budget_bytes=1 << 30, key_arena_bytes=arena, chunk_rows=512,
                              device="cpu", stream=object())
    _run(path, reqs)
    assert all(r.done_event is not None for r in reqs)
    assert all(r.latency_ms >= 0 for r in reqs)
    waves = [ids for kind, ids in fake if kind == "keygen"]
    assert any(len(set(ids)) > 1 for ids in waves)      # a wave holds chunks of several requests
    assert sum(len(ids) for ids in waves) == 6 * 2 * 2  # every (request, predicate, chunk) once


def test_chunk_larger_than_key_arena_is_rejected(fake):
    path = serving.ServedPath(None, budget_bytes=1 << 30, key_arena_bytes=1 << 19, chunk_rows=512, device="cpu",
                              stream=object())
    with pytest.raises(ValueError, match="key arena"):
        _run(path, _reqs([0.0]))


def test_resident_edge_prefix_is_the_candidate_view(monkeypatch):
    """A request's edge tables on the served path (prefix slices of the
    resident graph) are the candidate view's edges, in the same order, with
    the same shares; the prefix length is found without converting the key
    array (a search bound of another dtype would copy all of it per request)."""
    import numpy as np
    import synth
    calls = []
    f = _fake_fss(calls)
    f.fss_dealer_masks = lambda *a, **k: None
    f.fss_mask_open = lambda x0, x1, r, xh, s=None: calls.append(("open", x0.clone(), x1.clone()))
    monkeypatch.setattr(serving, "fss", f)
    real_search = np.searchsorted

    def search(a, v, side="left"):
        # a Python int bound makes numpy convert the whole key array first
        assert isinstance(v, np.generic) and v.dtype == a.dtype, "bound must be in the keys' dtype"
        return real_search(a, v, side=side)

    nv, ne = 1 << 12, 1 << 20
    src, dst = synth.chung_lu_graph(5, nv, ne)
    g = synth.Graph(nv, src, dst, {}, {"w": np.arange(ne, dtype=np.uint32)})
    esh = {"w": (np.arange(ne, dtype=np.uint32), np.zeros(ne, np.uint32))}
    rg = serving.resident_graph(nv, ne, src, dst, {}, esh, "cpu")
    monkeypatch.setattr(np, "searchsorted", search)
    for rows in (0, 1, 100, 3000, 1 << 12, 1 << 16):
        q = types.SimpleNamespace(query_id=1, n_qv=2, preds=[synth.Pred(2, "eq", "w", a=3)])
        req = serving.Request(0, 0.0, q, rows, 7)
        calls.clear()
        serving.prepare(req, rg, "cpu")
        view, erows = synth.candidate_view(g, rows)
        assert req.view["n_edges"] == view.n_edges
        if view.n_edges:
            assert np.array_equal(req.view["src"].numpy().view(np.uint32), view.src)
            assert np.array_equal(req.view["dst"].numpy().view(np.uint32), view.dst)
            assert np.array_equal(calls[0][1].numpy().view(np.uint32), erows.astype(np.uint32))


@pytest.mark.timeout(30)
def test_wave_cap_splits_work(fake):
    """A wave never holds more keys than wave_bytes (beyond its first chunk)."""
    reqs = _reqs([0.0] * 4, rows=4096)
    chunk_keys = 2 * 512 * 872
    path = serving.ServedPath(None, budget_bytes=1 << 30, key_arena_bytes=64 << 20, chunk_rows=512,
                              device="cpu", stream=object(), wave_bytes=3 * chunk_keys)
    sizes = []
    f = serving.fss
    keygen = f.fss_keygen_batch
    f.fss_keygen_batch = lambda kg, q, st: (sizes.append([2 * f.fss_keybatch_bytes(k[6][0], 32, k[6][1]) for k in kg]),
                                            keygen(kg, q, st))
    _run(path, reqs)
    assert sum(len(w) for w in sizes) == 4 * 2 * 8          # every chunk exactly once
    assert all(sum(w) <= 3 * chunk_keys or len(w) == 1 for w in sizes)
    assert len(sizes) >= 8
    assert all(r.done_event is not None for r in reqs)
