"""Serving loop over a graph resident in HBM.

Requests (path queries over candidate tables of the resident graph) arrive
over time.  Two protocols:

* token given (the primary one; the paper measures query latency from a
  query token the client has already made, Sec. VII): the tokens of the
  query mix -- the dealer's masks and both parties' keys of every predicate --
  are dealt before the run and stay resident; a request names its mix entry,
  and serving it is the servers' whole work: the masked opens, both parties'
  evaluation of every row of every predicate, the ANDs and the joins.
  GivenServedPath runs continuous batching: while the GPU runs a wave, the
  requests that arrive are admitted (in arrival order, while the device memory
  of their intermediates fits the budget) and form the next wave -- one
  persistent evaluation launch over all their predicates and parties, then one
  match_query_batch for their tails; at most two waves are in flight.
  GivenPlainPath serves one request at a time.
* keygen included: each request's token is dealt on arrival, inside its
  latency (ServedPath and PlainPath): the served path cuts every request's
  rows into chunks and runs each wave as one persistent dealer launch and one
  persistent evaluation launch over a key arena.

Latency is arrival -> result shares in device memory, timed by HIP events on
the serving stream against an event recorded when the clock starts.  Results
are bit-identical on every path (every kernel is a pure function of its
rows), which the tests check request by request.  Every allocation of a path
is made on its own stream (the caching allocator then reuses freed memory in
that stream's order).
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import fss
from .runner import KeyArena


@dataclass
class ResidentGraph:
    """Both servers' shares of every column plus the public endpoints, on the
    device.  Edge rows are stored sorted by (larger endpoint, row): the
    candidate edges of a request over r vertices are then a prefix, whose
    length comes from the host copy of the sorted larger endpoints, so a
    request's edge tables are slices -- no gather and no device round trip."""
    n_vertices: int
    n_edges: int
    src: torch.Tensor        # in edge order
    dst: torch.Tensor
    vshares: dict            # column -> (x0, x1) int32 tensors
    eshares: dict            # column -> (x0, x1), in edge order
    edge_keys: np.ndarray = None    # host: sorted larger endpoints


@dataclass
class Request:
    rid: int
    arrival: float           # seconds after the start
    query: object            # synth.Query (query_id unique per request)
    rows: int                # candidate table size
    seed: int
    # filled while served
    view: dict = field(default_factory=dict)
    preds: list = field(default_factory=list)
    bits: list = field(default_factory=list)
    plan: object = None
    mem: int = 0
    done_event: object = None
    latency_ms: float = 0.0


def _words(rows):
    return max(1, (rows + 31) // 32)


def prepare(req: Request, g: ResidentGraph, device, stream=None):
    """Candidate view, fresh dealer masks and opened values on the device."""
    q = req.query
    r_v = min(req.rows, g.n_vertices)
    if q.n_qv > 1:
        # the bound in the keys' own dtype: a Python int would make numpy
        # convert the whole key array before searching
        n_e = min(req.rows, int(np.searchsorted(g.edge_keys, g.edge_keys.dtype.type(r_v), side="left")))
        src, dst = g.src[:n_e], g.dst[:n_e]
    else:
        n_e, src, dst = 0, None, None
    req.view = dict(n_vertices=r_v, n_edges=n_e, src=src, dst=dst)
    req.preds = []
    for k, p in enumerate(q.preds):
        on_edge = p.target >= q.n_qv
        rows = n_e if on_edge else r_v
        if on_edge:
            x0, x1 = (t[:n_e] for t in g.eshares[p.column])
        else:
            x0, x1 = (t[:r_v] for t in g.vshares[p.column])
        r = torch.empty(max(rows, 1), dtype=torch.int32, device=device)
        xhat = torch.empty(max(rows, 1), dtype=torch.int32, device=device)
        if rows:
            fss.fss_dealer_masks(req.seed, q.query_id, k, rows, r, stream=stream)
            fss.fss_mask_open(x0.contiguous(), x1.contiguous(), r, xhat, stream)
        req.preds.append(dict(target=p.target, kind=fss.EQ if p.kind == "eq" else fss.RANGE, rows=rows,
                              a_or_lo=p.a if p.kind == "eq" else p.lo, hi=p.hi, r=r, xhat=xhat))
    return req


def memory_bound(req: Request) -> int:
    """Device bytes a request holds while admitted (keys excluded: they live
    in the wave arena): masks, opened values, share bits and the plan
    workspace, bounded with every table at ``rows`` rows (plus a margin for
    edge tables, which are slices of the resident graph)."""
    rows = req.rows
    npred = len(req.query.preds)
    per_table = 8 * rows + 16 * _words(rows)
    width = max(req.query.n_qv, req.query.n_qe + 1)     # n_qv for a path
    return 16 * rows + npred * (per_table + 16 * rows) + 32 * _words(rows) * (2 * npred + 8 * width)


def request_key_bytes(req: Request) -> int:
    return sum(2 * fss.fss_keybatch_bytes(p["kind"], 32, p["rows"]) for p in req.preds)


def _plan(req: Request, bits_given: bool, device):
    q, v = req.query, req.view
    if bits_given:
        preds = [(p["target"], None, None, req.bits[k]) for k, p in enumerate(req.preds)]
    else:
        preds = [(p["target"], p["kb"], p["xhat"]) for p in req.preds]
    return fss.Plan(req.seed, q.query_id, q.n_qv, v["n_vertices"], v["n_edges"], preds, v["src"],
                    v["dst"], q.edges).allocate(device)


class ServedPath:
    """Keygen included: continuous batching over a key arena (see the module notes)."""

    def __init__(self, graph: ResidentGraph, budget_bytes: int, key_arena_bytes: int, chunk_rows: int = 1 << 20,
                 device=None, stream=None, wave_bytes: int = None):
        """wave_bytes caps the keys (both parties) of one wave, i.e. its work:
        shorter waves let a request that arrives behind a large one finish one
        short wave later.  None: a wave may fill the whole key arena."""
        assert key_arena_bytes < budget_bytes and chunk_rows % 64 == 0
        self.g = graph
        self.device = device or torch.device("cuda")
        self.stream = stream or torch.cuda.current_stream()
        self.budget = budget_bytes
        self.arena = KeyArena(key_arena_bytes, self.device)
        self.wave_cap = min(key_arena_bytes, wave_bytes) if wave_bytes else key_arena_bytes
        self.chunk_rows = chunk_rows
        self.queue = fss.Queue(2048, self.device)
        self.waves = 0
        self.max_in_flight = 0
        self.max_used = 0           # peak admitted bytes (outside the key arena)

    def run(self, requests, clock_start_event, t0):
        """Serve `requests` (sorted by arrival) in real time from host time t0."""
        with torch.cuda.stream(self.stream):
            return self._run(requests, clock_start_event, t0)

    def _run(self, requests, clock_start_event, t0):
        pending = deque(requests)
        admitted = []           # requests with chunks left: (req, deque of chunk items)
        in_mem = []             # admitted, not released
        used = 0
        free_at = self.budget - self.arena.nbytes
        while pending or admitted:
            # the admission budget is returned once a request's results are in device memory
            keep = []
            for req in in_mem:
                if req.done_event is not None and req.done_event.query():
                    used -= req.mem
                else:
                    keep.append(req)
            in_mem = keep
            now = time.perf_counter() - t0
            # admission, in arrival order, while memory allows
            while pending and pending[0].arrival <= now:
                req = pending[0]
                req.mem = memory_bound(req)
                if in_mem and used + req.mem > free_at:
                    break          # admitted once memory frees up (arrival order is kept)
                pending.popleft()
                prepare(req, self.g, self.device, self.stream)
                req.bits = [tuple(torch.empty(_words(p["rows"]), dtype=torch.int32, device=self.device)
                                  for _ in range(2)) for p in req.preds]
                items = deque()
                for k, p in enumerate(req.preds):
                    for c0 in range(0, p["rows"], self.chunk_rows):
                        items.append((k, c0, min(self.chunk_rows, p["rows"] - c0)))
                admitted.append((req, items))
                in_mem.append(req)
                used += req.mem
                self.max_used = max(self.max_used, used)
            self.max_in_flight = max(self.max_in_flight, len(admitted))
            if not admitted:
                wait = pending[0].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.002))
                elif in_mem:
                    # the head request waits for memory: every admitted request is
                    # finished and enqueued, so the oldest one's results free it
                    in_mem[0].done_event.synchronize()
                continue
            # one wave over the admitted requests' chunks, oldest first
            self.arena.reset()
            kg, ev, finished = [], [], []
            for req, items in admitted:
                while items:
                    k, c0, n = items[0]
                    p = req.preds[k]
                    half = fss.fss_keybatch_bytes(p["kind"], 32, n)
                    if self.arena.used + 2 * half > self.arena.nbytes:
                        if not kg:
                            raise ValueError(f"a {n}-row chunk needs {2 * half} key bytes; the key arena "
                                             f"holds {self.arena.nbytes}")
                        break
                    if kg and self.arena.used + 2 * half > self.wave_cap:
                        break
                    items.popleft()
                    kb = fss.KeyBatch.view(p["kind"], 32, n, self.arena.take(half), self.arena.take(half))
                    kg.append((req.seed, req.query.query_id, k, p["a_or_lo"], p["hi"], p["r"][c0:c0 + n], kb, c0))
                    for b in range(2):
                        ev.append((b, kb, p["xhat"][c0:c0 + n], req.bits[k][b][c0 // 32:]))
                if not items:
                    finished.append(req)
                if kg and self.arena.used >= self.wave_cap:
                    break
            if kg:
                if len(ev) > self.queue.capacity:
                    self.queue = fss.Queue(2 * len(ev), self.device)
                fss.fss_keygen_batch(kg, self.queue, self.stream)
                fss.fss_eval_batch(ev, self.queue, self.stream)
                self.waves += 1
            if finished:
                plans = []
                for req in finished:
                    req.plan = _plan(req, True, self.device)
                    plans.append(req.plan)
                fss.match_query_batch(plans, self.queue, 3, self.stream)
                for req in finished:
                    req.done_event = torch.cuda.Event(enable_timing=True)
                    req.done_event.record(self.stream)
                    _drop_intermediates(req)   # stream-ordered allocator: safe once enqueued
                admitted = [(r, it) for r, it in admitted if r not in finished]
        torch.cuda.synchronize()
        for req in requests:
            req.latency_ms = clock_start_event.elapsed_time(req.done_event) - 1e3 * req.arrival
        return requests


class PlainPath:
    """Keygen included, one request at a time: masks, open, per-predicate keygen, match_query.

    sync=True waits for each request's results before taking the next (a
    server that answers one query before it starts another); sync=False only
    enqueues, so the host prepares request i+1 while the GPU runs request i."""

    def __init__(self, graph: ResidentGraph, device=None, stream=None, sync: bool = False):
        self.g = graph
        self.device = device or torch.device("cuda")
        self.stream = stream or torch.cuda.current_stream()
        self.sync = sync

    def run(self, requests, clock_start_event, t0):
        with torch.cuda.stream(self.stream):
            return self._run(requests, clock_start_event, t0)

    def _run(self, requests, clock_start_event, t0):
        for req in requests:
            wait = req.arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            prepare(req, self.g, self.device, self.stream)
            for k, p in enumerate(req.preds):
                p["kb"] = fss.KeyBatch(p["kind"], 32, p["rows"], self.device)
                if p["rows"]:
                    fss.fss_keygen(req.seed, req.query.query_id, k, p["a_or_lo"], p["hi"], p["r"], p["kb"],
                                   self.stream)
            req.plan = _plan(req, False, self.device)
            fss.match_query(req.plan, 3, self.stream)
            req.done_event = torch.cuda.Event(enable_timing=True)
            req.done_event.record(self.stream)
            _drop_intermediates(req)
            if self.sync:
                req.done_event.synchronize()
        torch.cuda.synchronize()
        for req in requests:
            req.latency_ms = clock_start_event.elapsed_time(req.done_event) - 1e3 * req.arrival
        return requests


# --------------------------------------------------------------------------- token given

@dataclass
class Token:
    """One mix entry's query token as the servers hold it: the candidate view
    and, per predicate, the dealer's masks and both parties' keys."""
    query: object
    rows: int
    seed: int
    view: dict
    preds: list             # dicts: target, kind, rows, r, kb
    key_bytes: int = 0


class TokenPool:
    """The tokens of a query mix, dealt before the run (dealer masks with
    fss_dealer_masks, keys with fss_keygen) and kept in device memory."""

    def __init__(self, graph: ResidentGraph, mix, seed: int, device=None, stream=None):
        self.device = device or torch.device("cuda")
        s = stream or torch.cuda.current_stream()
        self.tokens = []
        with torch.cuda.stream(s):
            for q, rows in mix:
                req = Request(-1, 0.0, q, rows, seed)
                view = _view(req, graph)
                preds = []
                for k, p in enumerate(q.preds):
                    n = view["n_edges"] if p.target >= q.n_qv else view["n_vertices"]
                    kind = fss.EQ if p.kind == "eq" else fss.RANGE
                    r = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
                    kb = fss.KeyBatch(kind, 32, n, self.device)
                    if n:
                        fss.fss_dealer_masks(seed, q.query_id, k, n, r, stream=s)
                        fss.fss_keygen(seed, q.query_id, k, p.a if p.kind == "eq" else p.lo, p.hi, r, kb, s)
                    preds.append(dict(target=p.target, kind=kind, rows=n, r=r, kb=kb))
                self.tokens.append(Token(q, rows, seed, view, preds,
                                         sum(2 * d["kb"].bytes_per_party for d in preds)))
        s.synchronize()

    @property
    def key_bytes(self) -> int:
        return sum(t.key_bytes for t in self.tokens)


@dataclass
class GivenRequest:
    rid: int
    arrival: float          # seconds after the start
    entry: int              # mix entry whose token the request carries
    keep: bool = True       # keep the result shares after completion (else they are dropped)
    # filled while served
    xhat: list = field(default_factory=list)
    bits: list = field(default_factory=list)
    plan: object = None
    mem: int = 0
    done_event: object = None
    latency_ms: float = 0.0


def _view(req, g: ResidentGraph) -> dict:
    """Candidate vertices [0, rows) and the edges among them (a prefix of the
    resident edge order)."""
    q = req.query
    r_v = min(req.rows, g.n_vertices)
    if q.n_qv > 1:
        # the bound in the keys' own dtype: a Python int would make numpy
        # convert the whole key array before searching
        n_e = min(req.rows, int(np.searchsorted(g.edge_keys, g.edge_keys.dtype.type(r_v), side="left")))
        return dict(n_vertices=r_v, n_edges=n_e, src=g.src[:n_e], dst=g.dst[:n_e])
    return dict(n_vertices=r_v, n_edges=0, src=None, dst=None)


def token_walks(tok: Token) -> int:
    """Tree walks of a token's evaluation (both parties; a range is two)."""
    return sum(2 * d["rows"] * (1 if d["kind"] == fss.EQ else 2) for d in tok.preds)


def given_memory(tok: Token) -> int:
    """Device bytes a token-given request allocates while admitted: opened
    values, both parties' share bits, the plan's workspace and outputs
    (bounded with every table at the token's largest row count)."""
    rows = max([d["rows"] for d in tok.preds] + [tok.view["n_vertices"], tok.view["n_edges"], 1])
    npred = len(tok.preds)
    width = max(tok.query.n_qv, tok.query.n_qe + 1)     # n_qv for a path
    return 4 * rows * npred + 8 * _words(rows) * (2 * npred + 4 * width + 4) + 4096 * (npred + 2)


def _open_given(req: GivenRequest, tok: Token, g: ResidentGraph, device, stream):
    """The request's masked opens: x0 + x1 + r per predicate, with the token's masks."""
    q = tok.query
    req.xhat = []
    for k, p in enumerate(q.preds):
        d = tok.preds[k]
        n = d["rows"]
        xhat = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        if n:
            cols = g.eshares if p.target >= q.n_qv else g.vshares
            x0, x1 = (t[:n] for t in cols[p.column])
            fss.fss_mask_open(x0, x1, d["r"], xhat, stream)
        req.xhat.append(xhat)


def _given_plan_with_keys(req: GivenRequest, tok: Token, device):
    q, v = tok.query, tok.view
    preds = [(d["target"], d["kb"], req.xhat[k]) for k, d in enumerate(tok.preds)]
    return fss.Plan(tok.seed, q.query_id, q.n_qv, v["n_vertices"], v["n_edges"], preds, v["src"],
                    v["dst"], q.edges).allocate(device)


def _given_plan_with_bits(req: GivenRequest, tok: Token, device):
    q, v = tok.query, tok.view
    req.bits = [tuple(torch.empty(max(1, _words(d["rows"])), dtype=torch.int32, device=device) for _ in range(2))
                for d in tok.preds]
    preds = [(d["target"], None, None, req.bits[k]) for k, d in enumerate(tok.preds)]
    return fss.Plan(tok.seed, q.query_id, q.n_qv, v["n_vertices"], v["n_edges"], preds, v["src"],
                    v["dst"], q.edges).allocate(device)


class GivenServedPath:
    """Token given, continuous batching (see the module notes)."""

    def __init__(self, graph: ResidentGraph, pool: TokenPool, budget_bytes: int, device=None, stream=None,
                 max_waves_in_flight: int = 2, batch_walks: int = 4 << 20):
        """batch_walks: a wave is cut, in arrival order, into batches of at most
        this many tree walks (a request larger than that is a batch of its
        own); each batch is one evaluation launch and one match_query_batch
        with its own completion event, so a request completes no later than
        the requests that arrived after it."""
        self.g, self.pool = graph, pool
        self.batch_walks = batch_walks
        self.device = device or torch.device("cuda")
        self.stream = stream or torch.cuda.current_stream()
        self.budget = budget_bytes
        self.max_waves = max_waves_in_flight
        self.queue = fss.Queue(4096, self.device)
        self.waves = 0
        self.batches = 0
        self.max_in_flight = 0
        self.max_used = 0
        self.max_wave = 0

    def run(self, requests, clock_start_event, t0, deadline_s: float = None):
        with torch.cuda.stream(self.stream):
            return self._run(requests, clock_start_event, t0, deadline_s)

    def _run(self, requests, clock_start_event, t0, deadline_s):
        pending = deque(requests)
        in_mem = []             # admitted, results not yet in device memory
        waves = deque()         # completion events of the waves in flight
        used = 0
        while pending:
            if deadline_s is not None and time.perf_counter() - t0 > deadline_s:
                break           # overloaded: the rest is never served (reported as missing)
            keep = []
            for req in in_mem:
                if req.done_event.query():
                    used -= req.mem
                else:
                    keep.append(req)
            in_mem = keep
            while waves and waves[0].query():
                waves.popleft()
            now = time.perf_counter() - t0
            if len(waves) >= self.max_waves or not pending or pending[0].arrival > now:
                # nothing to start: wait for a wave to end or the next arrival
                if waves and len(waves) >= self.max_waves:
                    time.sleep(0.0002)
                elif pending and pending[0].arrival > now:
                    time.sleep(min(pending[0].arrival - now, 0.001))
                continue
            wave = []
            while pending and pending[0].arrival <= now:
                req = pending[0]
                tok = self.pool.tokens[req.entry]
                req.mem = given_memory(tok)
                if (in_mem or wave) and used + req.mem > self.budget:
                    break      # admitted once memory frees up (arrival order is kept)
                pending.popleft()
                wave.append(req)
                used += req.mem
                self.max_used = max(self.max_used, used)
            if not wave:
                in_mem[0].done_event.synchronize()      # the head request waits for memory
                continue
            batches, cur, walks = [], [], 0
            for req in wave:
                w = token_walks(self.pool.tokens[req.entry])
                if cur and walks + w > self.batch_walks:
                    batches.append(cur)
                    cur, walks = [], 0
                cur.append(req)
                walks += w
            batches.append(cur)
            for batch in batches:
                ev, plans = [], []
                for req in batch:
                    tok = self.pool.tokens[req.entry]
                    _open_given(req, tok, self.g, self.device, self.stream)
                    req.plan = _given_plan_with_bits(req, tok, self.device)
                    for k, d in enumerate(tok.preds):
                        if d["rows"]:
                            for b in range(2):
                                ev.append((b, d["kb"], req.xhat[k], req.bits[k][b]))
                    plans.append(req.plan)
                self.queue.reserve(fss.fss_queue_workspace_bytes(len(ev)))
                if ev:
                    fss.fss_eval_batch(ev, self.queue, self.stream)
                fss.match_query_batch(plans, self.queue, 3, self.stream)
                done = torch.cuda.Event(enable_timing=True)
                done.record(self.stream)
                for req in batch:
                    req.done_event = done
                    req.xhat, req.bits = [], []
                    req.plan.release_inputs()
                    if not req.keep:
                        req.plan = None
                self.batches += 1
            in_mem.extend(wave)
            waves.append(done)
            self.waves += 1
            self.max_wave = max(self.max_wave, len(wave))
            self.max_in_flight = max(self.max_in_flight, len(in_mem))
        torch.cuda.synchronize()
        for req in requests:
            req.latency_ms = (clock_start_event.elapsed_time(req.done_event) - 1e3 * req.arrival
                              if req.done_event is not None else float("inf"))
        return requests


class GivenPlainPath:
    """Token given, one request at a time: the opens, then match_query (both
    parties' evaluation, the ANDs, the joins).  sync=True waits for each
    request's results before taking the next; sync=False only enqueues."""

    def __init__(self, graph: ResidentGraph, pool: TokenPool, device=None, stream=None, sync: bool = True):
        self.g, self.pool = graph, pool
        self.device = device or torch.device("cuda")
        self.stream = stream or torch.cuda.current_stream()
        self.sync = sync

    def run(self, requests, clock_start_event, t0, deadline_s: float = None):
        with torch.cuda.stream(self.stream):
            for req in requests:
                if deadline_s is not None and time.perf_counter() - t0 > deadline_s:
                    break
                wait = req.arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
                tok = self.pool.tokens[req.entry]
                _open_given(req, tok, self.g, self.device, self.stream)
                req.plan = _given_plan_with_keys(req, tok, self.device)
                fss.match_query(req.plan, 3, self.stream)
                req.done_event = torch.cuda.Event(enable_timing=True)
                req.done_event.record(self.stream)
                req.xhat = []
                req.plan.release_inputs()
                if not req.keep:
                    req.plan = None
                if self.sync:
                    req.done_event.synchronize()
        torch.cuda.synchronize()
        for req in requests:
            req.latency_ms = (clock_start_event.elapsed_time(req.done_event) - 1e3 * req.arrival
                              if req.done_event is not None else float("inf"))
        return requests


def given_outputs(req: GivenRequest, pool: TokenPool):
    tok = pool.tokens[req.entry]
    v = tok.view
    w = _words(v["n_vertices"]) if tok.query.n_qv == 1 else tok.query.n_qe * _words(v["n_edges"])
    return [req.plan.out[b][:w].cpu().numpy().copy() for b in range(2)]


def _drop_intermediates(req: Request):
    """Release everything but the result shares (their last use is enqueued)."""
    req.preds = [dict(target=p["target"], rows=p["rows"], kind=p["kind"]) for p in req.preds]
    req.bits = []
    req.view = dict(n_vertices=req.view["n_vertices"], n_edges=req.view["n_edges"], src=None, dst=None)
    if req.plan is not None:
        req.plan.release_inputs()


def outputs(req: Request):
    v = req.view
    w = _words(v["n_vertices"]) if req.query.n_qv == 1 else req.query.n_qe * _words(v["n_edges"])
    return [req.plan.out[b][:w].cpu().numpy().copy() for b in range(2)]


def poisson_arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, count))


def summarize(requests, wall_s: float) -> dict:
    """Requests served per second of wall time and latency percentiles; a
    request never served (run cut at its deadline) counts as infinitely late."""
    lat = np.array([r.latency_ms for r in requests])
    done = np.isfinite(lat)
    return {"requests": len(requests), "served": int(done.sum()), "qps": float(done.sum()) / wall_s,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat[done].mean()) if done.any() else float("inf"), "wall_s": wall_s}


def resident_graph(n_vertices, n_edges, src, dst, vshares, eshares, device) -> ResidentGraph:
    """Upload both servers' column shares and the public endpoints (numpy
    uint32), edge rows sorted by (larger endpoint, row) -- the order of
    ``synth.Graph.edge_order``."""
    def T(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(device)
    key = np.maximum(src, dst)
    order = np.argsort(key, kind="stable")
    return ResidentGraph(n_vertices, n_edges, T(src[order]), T(dst[order]),
                         {k: (T(v[0]), T(v[1])) for k, v in vshares.items()},
                         {k: (T(v[0][order]), T(v[1][order])) for k, v in eshares.items()},
                         np.ascontiguousarray(key[order]))
