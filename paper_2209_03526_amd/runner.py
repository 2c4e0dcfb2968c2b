"""Batched execution of many queries under a device-memory budget.

Every predicate of every query is cut into row chunks.  Chunks are grouped
into waves whose keys (both parties) fit ``budget_bytes``; each wave is one
persistent dealer launch (``fss_keygen_batch``) and one persistent evaluation
launch (``fss_eval_batch``) over all its chunks, and its key memory is reused
by the next wave.  A query whose predicate bits are complete is finished --
its ANDs and edge joins -- by ``match_query_batch`` with the bits supplied.
Chunk boundaries are multiples of 64 rows, and the dealer's randomness is
addressed by table row, so results are bit-identical to whole-table calls.

All work is enqueued on one stream; the only host synchronisation is the
wait for a staging buffer inside the library.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import fss


@dataclass
class QueryJob:
    """One query over its candidate tables, inputs already on the device.

    preds: list of dicts with keys target, kind (fss.EQ / fss.RANGE), rows,
    a_or_lo, hi, r (mask tensor), xhat (opened values), in plan order."""
    seed: int
    query_id: int
    n_qv: int
    n_vertices: int
    n_edges: int
    preds: list
    src: object = None
    dst: object = None
    nbits: int = 32
    bits: list = field(default_factory=list)      # per predicate: (bits0, bits1) tensors
    plan: object = None
    edges: list = None                            # query edges; None: the path


def _key_bytes(kind, nbits, rows):
    return fss.fss_keybatch_bytes(kind, nbits, rows)


class KeyArena:
    """One device buffer carved into key batches, wave by wave."""

    def __init__(self, nbytes: int, device):
        self.nbytes = nbytes
        self.buf = torch.empty(max(nbytes, 512), dtype=torch.uint8, device=device)
        self.base = self.buf.data_ptr()
        assert self.base % 256 == 0
        self.used = 0

    def reset(self):
        self.used = 0

    def take(self, nbytes: int) -> int:
        nbytes = (nbytes + 255) // 256 * 256
        if self.used + nbytes > self.nbytes:
            raise MemoryError("key arena exhausted")
        p = self.base + self.used
        self.used += nbytes
        return p


class ChunkedRunner:
    def __init__(self, budget_bytes: int, chunk_rows: int = 1 << 20, device=None, stream=None):
        assert chunk_rows % 64 == 0
        self.device = device or torch.device("cuda")
        self.chunk_rows = chunk_rows
        self.arena = KeyArena(budget_bytes, self.device)
        self.stream = stream
        self.queue = fss.Queue(1024, self.device)
        self.waves = 0

    def _chunks(self, jobs):
        items = []
        for qi, job in enumerate(jobs):
            for k, p in enumerate(job.preds):
                rows = p["rows"]
                for c0 in range(0, rows, self.chunk_rows):
                    n = min(self.chunk_rows, rows - c0)
                    items.append((qi, k, c0, n, 2 * _key_bytes(p["kind"], job.nbits, n)))
        return items

    def _ensure_queue(self, count):
        if count > self.queue.capacity:
            self.queue = fss.Queue(max(count, 2 * self.queue.capacity), self.device)

    def _event(self):
        e = torch.cuda.Event(enable_timing=True)
        e.record(self.stream if isinstance(self.stream, torch.cuda.Stream) else torch.cuda.current_stream())
        return e

    def run(self, jobs, timings=None):
        """Evaluate and finish every job; returns the jobs (outputs in job.plan.out).

        timings: optional list that receives ("keygen" | "eval", start event,
        end event) per wave (HIP events on the launch stream; the stream must
        be None or a torch stream)."""
        for job in jobs:
            job.bits = []
            for p in job.preds:
                nw = max(1, fss.words(p["rows"]))
                job.bits.append(tuple(torch.empty(nw, dtype=torch.int32, device=self.device) for _ in range(2)))
        items = self._chunks(jobs)
        remaining = [sum(1 for it in items if it[0] == qi) for qi in range(len(jobs))]
        finished = [False] * len(jobs)
        i = 0
        while i < len(items):
            self.arena.reset()
            wave, keep = [], []
            while i < len(items):
                qi, k, c0, n, nbytes = items[i]
                if wave and self.arena.used + nbytes > self.arena.nbytes:
                    break
                job, p = jobs[qi], jobs[qi].preds[k]
                half = _key_bytes(p["kind"], job.nbits, n)
                kb = fss.KeyBatch.view(p["kind"], job.nbits, n, self.arena.take(half), self.arena.take(half))
                wave.append((qi, k, c0, n, kb))
                i += 1
            self._ensure_queue(2 * len(wave))
            kg, ev = [], []
            for qi, k, c0, n, kb in wave:
                job, p = jobs[qi], jobs[qi].preds[k]
                r = p["r"][c0:c0 + n]
                kg.append((job.seed, job.query_id, k, p["a_or_lo"], p["hi"], r, kb, c0))
                xh = p["xhat"][c0:c0 + n]
                for b in range(2):
                    ev.append((b, kb, xh, job.bits[k][b][c0 // 32:]))
                keep.append(kb)
            if timings is not None:
                e0 = self._event()
            fss.fss_keygen_batch(kg, self.queue, self.stream)
            if timings is not None:
                e1 = self._event()
            fss.fss_eval_batch(ev, self.queue, self.stream)
            if timings is not None:
                timings += [("keygen", e0, e1), ("eval", e1, self._event())]
            self.waves += 1
            done = []
            for qi, k, c0, n, kb in wave:
                remaining[qi] -= 1
                if remaining[qi] == 0 and not finished[qi]:
                    done.append(qi)
            self._finish([jobs[qi] for qi in done])
            for qi in done:
                finished[qi] = True
            # the next wave overwrites this wave's keys; stream order keeps it safe
        self._finish([job for qi, job in enumerate(jobs) if not finished[qi]])
        return jobs

    def _finish(self, jobs):
        if not jobs:
            return
        plans = []
        for job in jobs:
            preds = [(p["target"], None, None, job.bits[k]) for k, p in enumerate(job.preds)]
            plan = fss.Plan(job.seed, job.query_id, job.n_qv, job.n_vertices, job.n_edges, preds, job.src,
                            job.dst, job.edges).allocate(self.device)
            job.plan = plan
            plans.append(plan)
        fss.match_query_batch(plans, self.queue, 3, self.stream)
        for job, plan in zip(jobs, plans):
            plan.release_inputs()
            job.bits = []
