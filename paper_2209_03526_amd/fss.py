"""Python binding of ``liboblivgm_fss.so``: the C ABI of include/oblivgm_fss.h,
same names, argument marshalling only.  Device buffers are torch tensors on a
HIP device; ``stream`` defaults to torch's current stream.  Every computation
runs in the library's HIP kernels; there is no host fallback: importing this
module without the built library raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

from . import build as _build

EQ, RANGE = 0, 1
SS_AND_OPEN, SS_AND_CLOSE = 0, 1
MAX_QV, MAX_QE, MAX_PREDS = 8, 16, 32

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED = 0, -1, -2, -3, -4


class FssError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class fss_keybatch(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nbits", ctypes.c_uint32), ("n", ctypes.c_uint64),
                ("key", ctypes.c_void_p * 2)]


class fss_pred(ctypes.Structure):
    _fields_ = [("target", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("keys", ctypes.POINTER(fss_keybatch)), ("d_xhat", ctypes.c_void_p),
                ("d_bits", ctypes.c_void_p * 2)]


class match_plan(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("query_id", ctypes.c_uint32), ("n_qv", ctypes.c_uint32),
                ("n_pred", ctypes.c_uint32), ("n_qe", ctypes.c_uint32),
                ("n_vertices", ctypes.c_uint64), ("n_edges", ctypes.c_uint64),
                ("d_src", ctypes.c_void_p), ("d_dst", ctypes.c_void_p),
                ("preds", ctypes.POINTER(fss_pred)), ("q_edges", ctypes.POINTER(ctypes.c_uint32)),
                ("d_out", ctypes.c_void_p * 2),
                ("d_workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_uint64),
                ("round", ctypes.c_uint32), ("reserved2", ctypes.c_uint32),
                ("d_peer_msg", ctypes.c_void_p), ("d_msg", ctypes.c_void_p)]


class fss_keygen_req(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("query_id", ctypes.c_uint32), ("pred_id", ctypes.c_uint32),
                ("a_or_lo", ctypes.c_uint32), ("hi", ctypes.c_uint32), ("d_r", ctypes.c_void_p),
                ("out", ctypes.POINTER(fss_keybatch)), ("row_offset", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class fss_eval_req(ctypes.Structure):
    _fields_ = [("party", ctypes.c_int32), ("reserved", ctypes.c_int32), ("keys", ctypes.POINTER(fss_keybatch)),
                ("d_xhat", ctypes.c_void_p), ("d_out_bits", ctypes.c_void_p)]


class fss_eval_all_req(ctypes.Structure):
    _fields_ = [("party", ctypes.c_int32), ("reserved", ctypes.c_int32), ("keys", ctypes.POINTER(fss_keybatch)),
                ("key_row", ctypes.c_uint64), ("npoints", ctypes.c_uint64), ("d_out_bits", ctypes.c_void_p)]


def _load():
    if not os.path.exists(_build.LIB):
        raise ImportError(f"HIP library not built: {_build.LIB} (build it: python paper_2209_03526_amd/build.py)")
    lib = ctypes.CDLL(_build.LIB)
    P, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
    sigs = {
        "fss_key_bytes": ([i32, u32], u64),
        "fss_keybatch_bytes": ([i32, u32, u64], u64),
        "fss_last_error": ([], ctypes.c_char_p),
        "fss_version": ([], ctypes.c_char_p),
        "fss_shutdown": ([], ctypes.c_int),
        "fss_mask_open": ([u64, P, P, P, P, P], ctypes.c_int),
        "fss_keygen": ([u64, u32, u32, u32, u32, P, ctypes.POINTER(fss_keybatch), P], ctypes.c_int),
        "fss_eval_eq": ([i32, ctypes.POINTER(fss_keybatch), P, P, P], ctypes.c_int),
        "fss_eval_lt": ([i32, ctypes.POINTER(fss_keybatch), P, P, P], ctypes.c_int),
        "ss_triples": ([u64, u32, u32, u64, P, P, P], ctypes.c_int),
        "ss_and": ([i32, i32, u64, P, P, P, P, P, P], ctypes.c_int),
        "match_workspace_bytes": ([ctypes.POINTER(match_plan)], u64),
        "match_query": ([ctypes.POINTER(match_plan), i32, P], ctypes.c_int),
        "match_rounds": ([ctypes.POINTER(match_plan), ctypes.POINTER(u32), ctypes.POINTER(u64), u32], ctypes.c_int),
        "match_batch_queue_bytes": ([ctypes.POINTER(match_plan), u32], u64),
        "fss_queue_workspace_bytes": ([u64], u64),
        "fss_keygen_batch": ([ctypes.POINTER(fss_keygen_req), u32, P, u64, P], ctypes.c_int),
        "fss_eval_batch": ([ctypes.POINTER(fss_eval_req), u32, P, u64, P], ctypes.c_int),
        "fss_eval_batch_noalloc": ([ctypes.POINTER(fss_eval_req), u32, P], ctypes.c_int),
        "match_query_batch": ([ctypes.POINTER(match_plan), u32, i32, P, u64, P], ctypes.c_int),
        "fss_set_tuning": ([u32, u32], ctypes.c_int),
        "fss_eval_all": ([i32, ctypes.POINTER(fss_keybatch), u64, u64, P, P], ctypes.c_int),
        "fss_eval_all_batch": ([ctypes.POINTER(fss_eval_all_req), u32, P], ctypes.c_int),
        "fss_dealer_masks": ([u64, u32, u32, u32, u64, P, P], ctypes.c_int),
        "rss_reshare": ([u64, P, P, u32, P, P], ctypes.c_int),
        "rss_from_fss": ([u64, P, P, u32, P, P], ctypes.c_int),
        "rss_and": ([u64, P, P, P, u32, P, P], ctypes.c_int),
        "rss_shuffle_workspace_bytes": ([u64, u32], u64),
        "rss_shuffle": ([u64, u32, P, P, P, P, u64, P], ctypes.c_int),
        "rss_shuffle_prepare_workspace_bytes": ([u64], u64),
        "rss_shuffle_prepare": ([u64, P, P, P, u64, P], ctypes.c_int),
        "rss_shuffle_prepared_workspace_bytes": ([u64, u32], u64),
        "rss_shuffle_prepared": ([u64, u32, P, P, P, P, P, u64, P], ctypes.c_int),
        "rss_fetch_unique": ([u64, u32, P, P, P, P], ctypes.c_int),
        "rss_fetch_many_workspace_bytes": ([u64, u32], u64),
        "rss_fetch_many": ([u64, u32, P, P, P, P, P, P, u64, P], ctypes.c_int),
        "rss_compact_valid": ([u64, u32, P, P, P, P, P, P, u64, P], ctypes.c_int),
        "rss_sec_eval": ([u64, u32, P, P, P, P, P, P], ctypes.c_int),
        "rss_sec_eval_records": ([u64, u32, P, P, P, P, P, P], ctypes.c_int),
        "rss_fetch_table": ([u64, P, u32, P, u32, P, P, P], ctypes.c_int),
        "fss_get_tuning": ([ctypes.POINTER(u32), ctypes.POINTER(u32)], ctypes.c_int),
        "fss_set_keygen_tuning": ([u32], ctypes.c_int),
        "fss_get_keygen_tuning": ([ctypes.POINTER(u32)], ctypes.c_int),
        "rss_set_shuffle_tuning": ([u32], ctypes.c_int),
        "rss_get_shuffle_tuning": ([ctypes.POINTER(u32)], ctypes.c_int),
        "rss_group_k": ([u64, P, P, u32, P, P], ctypes.c_int),
        "rss_group_k_lists": ([u64, u32, P, P, u32, P, P], ctypes.c_int),
        "rss_enc_posting_lists": ([u64, u32, P, P, P, P, u64, P, u32, P, P, u64, P], ctypes.c_int),
        "rss_sec_access_workspace_bytes": ([u32, u32, u32], u64),
        "rss_sec_access": ([u64, u32, P, P, u32, P, u32, P, P, u32, P, P, P, P, P, P, u64, P], ctypes.c_int),
        "rss_sec_access_batch": ([u32, u64, u32, P, P, u32, P, u32, P, P, P, P, P, P, P, P, P, u64, P],
                                 ctypes.c_int),
    }
    for name, (args, res) in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


LIB = _load()
EXPORTS = ("fss_key_bytes", "fss_keybatch_bytes", "fss_last_error", "fss_version", "fss_shutdown", "fss_mask_open",
           "fss_keygen", "fss_eval_eq", "fss_eval_lt", "ss_triples", "ss_and", "match_workspace_bytes",
           "match_query", "match_rounds", "match_batch_queue_bytes", "fss_queue_workspace_bytes", "fss_keygen_batch", "fss_eval_batch", "fss_eval_batch_noalloc", "match_query_batch",
           "fss_set_tuning", "fss_get_tuning", "fss_set_keygen_tuning", "fss_get_keygen_tuning",
           "rss_set_shuffle_tuning", "rss_get_shuffle_tuning", "fss_eval_all", "fss_eval_all_batch", "rss_sec_eval", "fss_dealer_masks", "rss_reshare", "rss_from_fss", "rss_and",
           "rss_shuffle_workspace_bytes", "rss_shuffle", "rss_shuffle_prepare_workspace_bytes", "rss_shuffle_prepare",
           "rss_shuffle_prepared_workspace_bytes", "rss_shuffle_prepared", "rss_fetch_unique",
           "rss_fetch_many_workspace_bytes",
           "rss_fetch_many", "rss_compact_valid", "rss_sec_eval_records", "rss_fetch_table", "rss_group_k", "rss_group_k_lists", "rss_enc_posting_lists",
           "rss_sec_access_workspace_bytes", "rss_sec_access", "rss_sec_access_batch")


def _check(rc: int):
    if rc != OK:
        raise FssError(rc, LIB.fss_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        # torch's current stream on the current device, read without the
        # Python-level device lookups of torch.cuda.current_stream() (which
        # cost several microseconds a call, most of a small call's host time)
        return torch._C._cuda_getCurrentRawStream(torch._C._cuda_getDevice())
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return stream


def words(rows: int) -> int:
    return (rows + 31) // 32


def version() -> str:
    return LIB.fss_version().decode()


def shutdown():
    """Release the library's own buffers (they are re-created on demand)."""
    _check(LIB.fss_shutdown())


def fss_key_bytes(kind: int, nbits: int) -> int:
    return int(LIB.fss_key_bytes(kind, nbits))


def fss_keybatch_bytes(kind: int, nbits: int, n: int) -> int:
    return int(LIB.fss_keybatch_bytes(kind, nbits, n))


class KeyBatch:
    """One predicate's keys for n rows, both parties, in device memory."""

    def __init__(self, kind: int, nbits: int, n: int, device=None):
        self.kind, self.nbits, self.n = kind, nbits, n
        nbytes = fss_keybatch_bytes(kind, nbits, n)
        if nbytes == 0 and n > 0:
            raise FssError(EINVAL, f"bad key kind {kind} / nbits {nbits}")
        dev = device or torch.device("cuda")
        # torch's caching allocator returns 256-byte aligned blocks of >= 512 bytes
        self.key = [torch.empty(max(nbytes, 512), dtype=torch.uint8, device=dev) for _ in range(2)]
        self.c = fss_keybatch(kind, nbits, n, (ctypes.c_void_p * 2)(self.key[0].data_ptr(), self.key[1].data_ptr()))

    @classmethod
    def view(cls, kind: int, nbits: int, n: int, ptr0: int, ptr1: int):
        """A batch over device memory owned elsewhere (256-byte aligned pointers)."""
        kb = cls.__new__(cls)
        kb.kind, kb.nbits, kb.n = kind, nbits, n
        kb.key = [None, None]
        kb.c = fss_keybatch(kind, nbits, n, (ctypes.c_void_p * 2)(ptr0, ptr1))
        return kb

    @property
    def bytes_per_party(self) -> int:
        return fss_keybatch_bytes(self.kind, self.nbits, self.n)


def fss_mask_open(x0, x1, r, xhat, stream=None):
    _check(LIB.fss_mask_open(x0.numel(), _ptr(x0), _ptr(x1), _ptr(r), _ptr(xhat), _stream(stream)))


def fss_keygen(seed: int, query_id: int, pred_id: int, a_or_lo: int, hi: int, r, out: KeyBatch, stream=None):
    _check(LIB.fss_keygen(seed, query_id, pred_id, a_or_lo, hi, _ptr(r), ctypes.byref(out.c), _stream(stream)))


def fss_dealer_masks(seed: int, query_id: int, pred_id: int, n: int, r, row_offset: int = 0, stream=None):
    _check(LIB.fss_dealer_masks(seed, query_id, pred_id, row_offset, n, _ptr(r), _stream(stream)))


def fss_eval_eq(party: int, keys: KeyBatch, xhat, out_bits, stream=None):
    _check(LIB.fss_eval_eq(party, ctypes.byref(keys.c), _ptr(xhat), _ptr(out_bits), _stream(stream)))


def fss_eval_lt(party: int, keys: KeyBatch, xhat, out_bits, stream=None):
    _check(LIB.fss_eval_lt(party, ctypes.byref(keys.c), _ptr(xhat), _ptr(out_bits), _stream(stream)))


def ss_triples(seed: int, query_id: int, and_id: int, nwords: int, trip0, trip1, stream=None):
    _check(LIB.ss_triples(seed, query_id, and_id, nwords, _ptr(trip0), _ptr(trip1), _stream(stream)))


def ss_and(phase: int, party: int, nrows: int, x, y, triple, de_open, out, stream=None):
    _check(LIB.ss_and(phase, party, nrows, _ptr(x), _ptr(y), _ptr(triple), _ptr(de_open), _ptr(out),
                      _stream(stream)))


class Plan:
    """A match_plan with its ctypes storage kept alive."""

    def __init__(self, seed, query_id, n_qv, n_vertices, n_edges, preds, src=None, dst=None, edges=None):
        """preds: list of (target, KeyBatch, xhat tensor) -- evaluated by match_query --
        or (target, None, None, (bits0, bits1)) -- share bits already evaluated.
        edges: the query edges [(a, b), ...]; None: the path (j, j + 1)."""
        self._preds = (fss_pred * max(1, len(preds)))()
        self._keep = []
        for i, pr in enumerate(preds):
            target, kb, xhat = pr[:3]
            bits = pr[3] if len(pr) > 3 else (None, None)
            self._preds[i] = fss_pred(target, 0, ctypes.pointer(kb.c) if kb is not None else None, _ptr(xhat),
                                      (ctypes.c_void_p * 2)(_ptr(bits[0]), _ptr(bits[1])))
            self._keep.append((kb, xhat, bits))
        self.c = match_plan()
        self.c.seed = seed
        self.c.query_id = query_id
        self.c.n_qv = n_qv
        self.c.n_pred = len(preds)
        self.c.n_vertices = n_vertices
        self.c.n_edges = n_edges
        self.c.d_src = _ptr(src)
        self.c.d_dst = _ptr(dst)
        self.c.preds = ctypes.cast(self._preds, ctypes.POINTER(fss_pred))
        self._keep.append((src, dst))
        flat = [int(v) for e in (edges or []) for v in e]
        self._qedges = (ctypes.c_uint32 * max(1, len(flat)))(*flat)    # read on every call: kept
        self.c.n_qe = len(flat) // 2
        self.c.q_edges = ctypes.cast(self._qedges, ctypes.POINTER(ctypes.c_uint32)) if flat else None
        self.out = None
        self.workspace = None

    def out_words(self) -> int:
        if self.c.n_qv == 1:
            return words(self.c.n_vertices)
        n_qe = self.c.n_qe or self.c.n_qv - 1
        return n_qe * words(self.c.n_edges)

    def allocate(self, device=None):
        dev = device or torch.device("cuda")
        self.out = [torch.empty(max(1, self.out_words()), dtype=torch.int32, device=dev) for _ in range(2)]
        nbytes = int(LIB.match_workspace_bytes(ctypes.byref(self.c)))
        self.workspace = torch.empty(max(nbytes, 512), dtype=torch.uint8, device=dev)
        self.c.d_out[0] = self.out[0].data_ptr()
        self.c.d_out[1] = self.out[1].data_ptr()
        self.c.d_workspace = self.workspace.data_ptr()
        self.c.workspace_bytes = self.workspace.numel()
        return self

    def release_inputs(self):
        """Drop the references to keys, opened values, share bits and the
        workspace once the plan's work is enqueued (the caching allocator
        reuses the memory in stream order); only the result shares stay."""
        self._keep = []
        self.workspace = None


def match_workspace_bytes(plan: Plan) -> int:
    return int(LIB.match_workspace_bytes(ctypes.byref(plan.c)))


def match_rounds(plan: Plan) -> list:
    """Message words of each exchange round of a single-party run (its length is R)."""
    n = ctypes.c_uint32()
    _check(LIB.match_rounds(ctypes.byref(plan.c), ctypes.byref(n), None, 0))
    words_ = (ctypes.c_uint64 * max(1, n.value))()
    _check(LIB.match_rounds(ctypes.byref(plan.c), ctypes.byref(n), words_, n.value))
    return [int(words_[r]) for r in range(n.value)]


def match_query(plan: Plan, party_mask: int = 3, stream=None, round: int = 0, peer_msg=None, msg=None):
    """party_mask 3: both parties.  1 / 2: party 0 / 1, round `round`, with the
    peer's message of round - 1 (peer_msg) and this party's message (msg)."""
    plan.c.round = round
    plan.c.d_peer_msg = _ptr(peer_msg)
    plan.c.d_msg = _ptr(msg)
    _check(LIB.match_query(ctypes.byref(plan.c), party_mask, _stream(stream)))


# --------------------------------------------------------------------------- batches

def fss_queue_workspace_bytes(count: int) -> int:
    return int(LIB.fss_queue_workspace_bytes(count))


class Queue:
    """Device memory for the work queue of batch calls (counter + descriptors)."""

    def __init__(self, capacity: int, device=None):
        self.capacity = capacity
        nbytes = fss_queue_workspace_bytes(max(1, capacity))
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device or torch.device("cuda"))

    def reserve(self, nbytes: int):
        """Grow to at least nbytes (the old buffer's uses are all enqueued on
        the stream that allocated it, which the caching allocator respects)."""
        if nbytes > self.buf.numel():
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.buf.device)

    def ptr(self):
        return self.buf.data_ptr(), self.buf.numel()


def fss_keygen_batch(reqs, queue: Queue, stream=None):
    """reqs: list of (seed, query_id, pred_id, a_or_lo, hi, r tensor, KeyBatch[, row_offset])."""
    arr = (fss_keygen_req * max(1, len(reqs)))()
    for i, rq in enumerate(reqs):
        seed, qid, pid, a, hi, r, kb = rq[:7]
        off = rq[7] if len(rq) > 7 else 0
        arr[i] = fss_keygen_req(seed, qid, pid, a, hi, _ptr(r), ctypes.pointer(kb.c), off, 0)
    d, nbytes = queue.ptr()
    _check(LIB.fss_keygen_batch(arr, len(reqs), d, nbytes, _stream(stream)))


def fss_eval_batch(reqs, queue: Queue, stream=None):
    """reqs: list of (party, KeyBatch, xhat tensor, out tensor)."""
    arr = (fss_eval_req * max(1, len(reqs)))()
    for i, (party, kb, xhat, out) in enumerate(reqs):
        arr[i] = fss_eval_req(party, 0, ctypes.pointer(kb.c), _ptr(xhat), _ptr(out))
    d, nbytes = queue.ptr()
    _check(LIB.fss_eval_batch(arr, len(reqs), d, nbytes, _stream(stream)))


def _plan_array(plans):
    arr = (match_plan * max(1, len(plans)))()
    for i, p in enumerate(plans):
        arr[i] = p.c
    return arr


def match_batch_queue_bytes(plans) -> int:
    return int(LIB.match_batch_queue_bytes(_plan_array(plans), len(plans)))


NOALLOC_EVAL_MAX = 1360


def _eval_reqs(reqs):
    arr = (fss_eval_req * max(1, len(reqs)))()
    for i, (party, kb, xhat, out) in enumerate(reqs):
        arr[i] = fss_eval_req(party, 0, ctypes.pointer(kb.c), _ptr(xhat), _ptr(out))
    return arr


def fss_eval_batch_noalloc(reqs, stream=None):
    """fss_eval_batch with the library's own per-GPU queue (no allocation)."""
    _check(LIB.fss_eval_batch_noalloc(_eval_reqs(reqs), len(reqs), _stream(stream)))


def match_query_batch(plans, queue: Queue, party_mask: int = 3, stream=None):
    """party_mask 1 / 2: each plan runs its own round (plan.c.round, messages set
    beforehand, e.g. with set_round)."""
    arr = _plan_array(plans)
    queue.reserve(int(LIB.match_batch_queue_bytes(arr, len(plans))))
    d, nbytes = queue.ptr()
    _check(LIB.match_query_batch(arr, len(plans), party_mask, d, nbytes, _stream(stream)))


def set_round(plan: Plan, round: int, peer_msg=None, msg=None):
    plan.c.round = round
    plan.c.d_peer_msg = _ptr(peer_msg)
    plan.c.d_msg = _ptr(msg)


def set_tuning(rows_per_thread: int, wg_per_cu: int):
    _check(LIB.fss_set_tuning(rows_per_thread, wg_per_cu))


def get_tuning():
    a, b = ctypes.c_uint32(), ctypes.c_uint32()
    LIB.fss_get_tuning(ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def set_keygen_tuning(tile_mult: int):
    _check(LIB.fss_set_keygen_tuning(tile_mult))


def get_keygen_tuning() -> int:
    a = ctypes.c_uint32()
    LIB.fss_get_keygen_tuning(ctypes.byref(a))
    return a.value


def set_shuffle_tuning(perm_method: int):
    _check(LIB.rss_set_shuffle_tuning(perm_method))


def get_shuffle_tuning() -> int:
    a = ctypes.c_uint32()
    LIB.rss_get_shuffle_tuning(ctypes.byref(a))
    return a.value


# --------------------------------------------------------------------------- one-hot RSS secEval

def fss_eval_all(party: int, keys: KeyBatch, key_row: int, npoints: int, out_bits, stream=None):
    _check(LIB.fss_eval_all(party, ctypes.byref(keys.c), key_row, npoints, _ptr(out_bits), _stream(stream)))


def fss_eval_all_batch(reqs, stream=None):
    """reqs: list of (party, KeyBatch, key_row, npoints, out_bits tensor)."""
    arr = (fss_eval_all_req * max(1, len(reqs)))()
    for i, (party, kb, row, npoints, out) in enumerate(reqs):
        arr[i] = fss_eval_all_req(party, 0, ctypes.pointer(kb.c), row, npoints, _ptr(out))
    _check(LIB.fss_eval_all_batch(arr, len(reqs), _stream(stream)))


def rss_sec_eval(ncand: int, npos: int, eval_a, eval_b, share_a, share_b, out_bits, stream=None):
    _check(LIB.rss_sec_eval(ncand, npos, _ptr(eval_a), _ptr(eval_b), _ptr(share_a), _ptr(share_b), _ptr(out_bits),
                            _stream(stream)))


def _ptr3(ts):
    return (ctypes.c_void_p * 3)(*[_ptr(t) for t in ts])


def rss_sec_eval_records(ncand: int, npos: int, eval_a, eval_b, share_a, share_b, out_bits, stream=None):
    _check(LIB.rss_sec_eval_records(ncand, npos, _ptr(eval_a), _ptr(eval_b), _ptr(share_a), _ptr(share_b),
                                    _ptr(out_bits), _stream(stream)))


def rss_fetch_table(ncand: int, bits3, id_words: int, ids3, val_words: int, vals3, out3, stream=None):
    _check(LIB.rss_fetch_table(ncand, _ptr3(bits3), id_words, _ptr3(ids3) if ids3 is not None else None, val_words,
                               _ptr3(vals3) if vals3 is not None else None, _ptr3(out3), _stream(stream)))


def rss_reshare(nrows: int, x3, prf_keys, counter: int, z3, stream=None):
    keys = (ctypes.c_uint64 * 3)(*prf_keys)
    _check(LIB.rss_reshare(nrows, _ptr3(x3), keys, counter, _ptr3(z3), _stream(stream)))


def rss_from_fss(nrows: int, y2, prf_keys, counter: int, z3, stream=None):
    """y2: (party 0 bits, party 1 bits) of the masked-input path -> RSS z3."""
    keys = (ctypes.c_uint64 * 3)(*prf_keys)
    _check(LIB.rss_from_fss(nrows, (ctypes.c_void_p * 2)(*[_ptr(t) for t in y2]), keys, counter, _ptr3(z3),
                            _stream(stream)))


def rss_and(nrows: int, x3, y3, prf_keys, counter: int, z3, stream=None):
    keys = (ctypes.c_uint64 * 3)(*prf_keys)
    _check(LIB.rss_and(nrows, _ptr3(x3), _ptr3(y3), keys, counter, _ptr3(z3), _stream(stream)))


def rss_shuffle(nrows: int, nwords: int, d3, seeds, out3, stream=None):
    nbytes = int(LIB.rss_shuffle_workspace_bytes(nrows, nwords))
    work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=d3[0].device)
    _check(LIB.rss_shuffle(nrows, nwords, _ptr3(d3), (ctypes.c_uint64 * 3)(*seeds), _ptr3(out3), _ptr(work),
                           work.numel(), _stream(stream)))
    return work


def rss_shuffle_prepare(nrows: int, seeds, perms, stream=None):
    """perms: device int32 tensor of 3 * nrows entries, filled with
    [inverse of pi12 | inverse of pi31 | pi23]."""
    nbytes = int(LIB.rss_shuffle_prepare_workspace_bytes(nrows))
    work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=perms.device)
    _check(LIB.rss_shuffle_prepare(nrows, (ctypes.c_uint64 * 3)(*seeds), _ptr(perms), _ptr(work), work.numel(),
                                   _stream(stream)))
    return work


def rss_shuffle_prepared(nrows: int, nwords: int, d3, seeds, perms, out3, stream=None):
    nbytes = int(LIB.rss_shuffle_prepared_workspace_bytes(nrows, nwords))
    work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=d3[0].device)
    _check(LIB.rss_shuffle_prepared(nrows, nwords, _ptr3(d3), (ctypes.c_uint64 * 3)(*seeds), _ptr(perms),
                                    _ptr3(out3), _ptr(work), work.numel(), _stream(stream)))
    return work


def rss_fetch_unique(ncand: int, nwords: int, x3, rows3, out3, stream=None):
    _check(LIB.rss_fetch_unique(ncand, nwords, _ptr3(x3), _ptr3(rows3), _ptr3(out3), _stream(stream)))


def rss_fetch_many(ncand: int, nwords: int, table3, seeds, out3, rows_out, count, stream=None):
    nbytes = int(LIB.rss_fetch_many_workspace_bytes(ncand, nwords))
    work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=table3[0].device)
    _check(LIB.rss_fetch_many(ncand, nwords, _ptr3(table3), (ctypes.c_uint64 * 3)(*seeds), _ptr3(out3),
                              _ptr(rows_out), _ptr(count), _ptr(work), work.numel(), _stream(stream)))
    return work


def rss_compact_valid(nrec: int, nwords: int, table3, seeds, out3, rows_out, count, stream=None):
    nbytes = int(LIB.rss_fetch_many_workspace_bytes(nrec, nwords))
    work = torch.empty(max(nbytes, 256), dtype=torch.int8, device=table3[0].device)
    _check(LIB.rss_compact_valid(nrec, nwords, _ptr3(table3), (ctypes.c_uint64 * 3)(*seeds), _ptr3(out3),
                                 _ptr(rows_out), _ptr(count), _ptr(work), work.numel(), _stream(stream)))
    return work


# --------------------------------------------------------------------------- Alg. 1 / Alg. 6

def rss_group_k(lengths, types, k: int):
    """Host arrays in, (padded lengths, group numbers) out (numpy uint32)."""
    import numpy as np
    lengths = np.ascontiguousarray(lengths, np.uint32)
    types = np.ascontiguousarray(types, np.uint32)
    padded = np.zeros(lengths.size, np.uint32)
    group = np.zeros(lengths.size, np.uint32)
    _check(LIB.rss_group_k(lengths.size, lengths.ctypes.data, types.ctypes.data, k, padded.ctypes.data,
                           group.ctypes.data))
    return padded, group


def rss_group_k_lists(lengths, types, k: int):
    """Host arrays in: lengths (nlists, n), types (n,); out: (padded lengths
    (nlists, n), group numbers (n,)), numpy uint32."""
    import numpy as np
    lengths = np.ascontiguousarray(np.atleast_2d(lengths), np.uint32)
    types = np.ascontiguousarray(types, np.uint32)
    nl, n = lengths.shape
    padded = np.zeros((nl, n), np.uint32)
    group = np.zeros(n, np.uint32)
    _check(LIB.rss_group_k_lists(n, nl, lengths.ctypes.data, types.ctypes.data, k, padded.ctypes.data,
                                 group.ctypes.data))
    return padded, group


def rss_enc_posting_lists(n: int, x_bits: int, adj_off, adj, slot, off, nrec: int, split_keys, counter: int, out3,
                          stream=None):
    work = torch.empty(max(4 * nrec, 256), dtype=torch.uint8, device=out3[0].device)
    _check(LIB.rss_enc_posting_lists(n, x_bits, _ptr(adj_off), _ptr(adj), _ptr(slot), _ptr(off), nrec,
                                     (ctypes.c_uint64 * 2)(*split_keys), counter, _ptr3(out3), _ptr(work),
                                     work.numel(), _stream(stream)))
    return work


def rss_sec_access_batch(ncand: int, x_bits: int, idm_ptrs, off, lmax: int, post3, attr_words: int, attr3,
                         prf_keys, counters, seeds, ids3, attrs3, rows_out, count, stream=None):
    """len(counters) secAccess calls in one library call: idm_ptrs holds the
    3 device addresses of each call's matched-ID shares, seeds 3 values per
    call; call c's outputs sit at offset c times one call's capacity."""
    n = len(counters)
    nbytes = int(LIB.rss_sec_access_workspace_bytes(lmax, x_bits, attr_words))
    work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=ids3[0].device)
    _check(LIB.rss_sec_access_batch(n, ncand, x_bits, (ctypes.c_void_p * (3 * n))(*idm_ptrs), _ptr(off), lmax,
                                    _ptr3(post3), attr_words, _ptr3(attr3), (ctypes.c_uint64 * 3)(*prf_keys),
                                    (ctypes.c_uint32 * n)(*counters), (ctypes.c_uint64 * (3 * n))(*seeds),
                                    _ptr3(ids3), _ptr3(attrs3), _ptr(rows_out), _ptr(count), _ptr(work),
                                    work.numel(), _stream(stream)))
    return work


def rss_sec_access(ncand: int, x_bits: int, idm3, off, lmax: int, post3, attr_words: int, attr3, prf_keys,
                   counter: int, seeds, ids3, attrs3, rows_out, count, stream=None):
    nbytes = int(LIB.rss_sec_access_workspace_bytes(lmax, x_bits, attr_words))
    work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=ids3[0].device)
    _check(LIB.rss_sec_access(ncand, x_bits, _ptr3(idm3), _ptr(off), lmax, _ptr3(post3), attr_words, _ptr3(attr3),
                              (ctypes.c_uint64 * 3)(*prf_keys), counter, (ctypes.c_uint64 * 3)(*seeds), _ptr3(ids3),
                              _ptr3(attrs3), _ptr(rows_out), _ptr(count), _ptr(work), work.numel(), _stream(stream)))
    return work
