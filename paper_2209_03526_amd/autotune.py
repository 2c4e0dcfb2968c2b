"""Autotuner for the tile / occupancy shape of the persistent launches.

The shape (rows per thread of an evaluation tile, workgroups per CU of the
persistent grids, rows of a keygen tile) never changes results, only speed.
``tune`` times each evaluation shape on the caller's own batch with HIP
events on the launch stream and keeps the fastest per size bucket (log2 of the
batch's total rows); ``tune_keygen`` then does the same for the keygen tile
(512, 1024, 2048 or 4096 rows) with that shape set.  Later batches in the same
bucket reuse the choices.
"""
from __future__ import annotations

import math

import torch

from . import fss

CANDIDATES = [(1, 2), (2, 2), (4, 2), (1, 1), (2, 1)]
KEYGEN_CANDIDATES = [1, 2, 4, 8]
_cache: dict = {}
_keygen_cache: dict = {}


def bucket(total_rows: int) -> int:
    return int(math.log2(max(1, total_rows)))


def _time(run, reps, s) -> float:
    run()                                       # warm
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        run()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(run, total_rows: int, reps: int = 2, stream=None):
    """run(): enqueue the batch once on `stream` (it must be idempotent).
    Returns the chosen (rows_per_thread, wg_per_cu) and leaves it set."""
    key = bucket(total_rows)
    if key in _cache:
        fss.set_tuning(*_cache[key])
        return _cache[key]
    s = stream or torch.cuda.current_stream()
    best, best_ms = None, float("inf")
    for cand in CANDIDATES:
        fss.set_tuning(*cand)
        ms = _time(run, reps, s)
        if ms < best_ms:
            best, best_ms = cand, ms
    _cache[key] = best
    fss.set_tuning(*best)
    return best


def tune_keygen(run, total_rows: int, reps: int = 2, stream=None) -> int:
    """run(): enqueue a batch that makes keys (it must be idempotent).
    Returns the chosen keygen tile multiplier and leaves it set."""
    key = bucket(total_rows)
    if key in _keygen_cache:
        fss.set_keygen_tuning(_keygen_cache[key])
        return _keygen_cache[key]
    s = stream or torch.cuda.current_stream()
    best, best_ms = None, float("inf")
    for cand in KEYGEN_CANDIDATES:
        fss.set_keygen_tuning(cand)
        ms = _time(run, reps, s)
        if ms < best_ms:
            best, best_ms = cand, ms
    _keygen_cache[key] = best
    fss.set_keygen_tuning(best)
    return best


def chosen() -> dict:
    return dict(_cache)


def chosen_keygen() -> dict:
    return dict(_keygen_cache)
