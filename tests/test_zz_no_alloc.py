"""The allocation-free batch evaluation (fss_eval_batch_noalloc) against the
existing entry point it varies (fss_eval_batch), bit for bit, on two calls in
a row -- the second with fewer and smaller requests, so that what the first
call left in the library's per-GPU queue must not leak into it."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, T, U

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fss():
    from paper_2209_03526_amd import fss as f
    return f


def _requests(fss, rows_kinds, seed):
    rng = np.random.default_rng(seed)
    reqs, outs = [], []
    for k, (rows, kind) in enumerate(rows_kinds):
        r = T(rng.integers(0, 2**32, rows, dtype=np.uint64).astype(np.uint32))
        xhat = T(rng.integers(0, 2**32, rows, dtype=np.uint64).astype(np.uint32))
        kb = fss.KeyBatch(kind, 32, rows)
        if rows and kind == fss.EQ:
            fss.fss_keygen(seed, 5, k, 12345, 0, r, kb)
        elif rows:
            fss.fss_keygen(seed, 5, k, 1000, 3_000_000_000, r, kb)
        for b in range(2):
            a = torch.full((fss.words(rows),), -1, dtype=torch.int32, device=DEV)
            n = torch.full((fss.words(rows),), -1, dtype=torch.int32, device=DEV)
            reqs.append(((b, kb, xhat), a, n))
            outs.append((a, n))
    return reqs, outs


def test_eval_batch_noalloc_equals_queue_path(fss):
    queue = fss.Queue(64)
    calls = [
        [(70001, fss.RANGE), (5000, fss.EQ), (1, fss.RANGE), (4099, fss.EQ), (130, fss.RANGE)],
        [(300, fss.EQ), (64, fss.RANGE)],
    ]
    for call, rows_kinds in enumerate(calls):
        reqs, outs = _requests(fss, rows_kinds, 900 + call)
        fss.fss_eval_batch([(*q, a) for q, a, _ in reqs], queue)
        fss.fss_eval_batch_noalloc([(*q, n) for q, _, n in reqs])
        torch.cuda.synchronize()
        for i, (a, n) in enumerate(outs):
            np.testing.assert_array_equal(U(n), U(a), err_msg=f"call {call} request {i}")


def test_eval_batch_noalloc_many_requests(fss):
    """Several argument chunks of descriptors (42 to a chunk), empty requests
    among them, equal row counts whose order must stay stable, then a smaller
    call."""
    queue = fss.Queue(64)
    rng = np.random.default_rng(77)
    big = [(int(rng.choice([0, 1, 64, 1000, 2049, 3000])), fss.RANGE if rng.random() < 0.5 else fss.EQ)
           for _ in range(70)]
    calls = [big, [(2049, fss.EQ), (0, fss.RANGE), (17, fss.RANGE)]]
    for call, rows_kinds in enumerate(calls):
        reqs, outs = _requests(fss, rows_kinds, 950 + call)
        fss.fss_eval_batch([(*q, a) for q, a, _ in reqs], queue)
        fss.fss_eval_batch_noalloc([(*q, n) for q, _, n in reqs])
        torch.cuda.synchronize()
        for i, (a, n) in enumerate(outs):
            np.testing.assert_array_equal(U(n), U(a), err_msg=f"call {call} request {i}")


def test_eval_batch_noalloc_rejects_too_many(fss):
    kb = fss.KeyBatch(fss.EQ, 32, 1)
    x = torch.zeros(1, dtype=torch.int32, device=DEV)
    o = torch.zeros(1, dtype=torch.int32, device=DEV)
    with pytest.raises(fss.FssError) as e:
        fss.fss_eval_batch_noalloc([(0, kb, x, o)] * (fss.NOALLOC_EVAL_MAX + 1))
    assert e.value.code == fss.EINVAL
