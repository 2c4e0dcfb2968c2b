"""hipGraph capture of one query's per-call pipeline -- the open and dealer
keygen of every predicate, then match_query (both parties' evaluation and
the ANDs) -- and its replay.  The pipeline holds no memset, no host copy and
no host wait, so it can be captured whole; a replay redoes the same work
(same seeds, so the same keys) and must give the eager result bit for bit,
every time, with eager work and synchronisations between the replays."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import DEV

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
