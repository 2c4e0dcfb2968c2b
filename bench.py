"""Benchmark of the FSS hot path on one MI355X.

Default workload (the headline line): the full path query over a power-law
graph -- Chung-Lu (exponent 2.1), 2^22 vertices x 4 uint32 attributes (two
labels uniform in [0,64), two Zipf(1.1) integers over [0,2^32)), 2^25 edges
with a label uniform in [0,4) and a weight uniform in [0,2^16).  Query a->b->c
with 4 vertex predicates (2 equality, 2 range) and 2 edge predicates (1 and 1),
evaluated by both simulated parties: filter -> shared edge join -> shared
result bits over every edge.

One step is the whole path over that graph: for each predicate the masked
open and the dealer's key generation, then one persistent evaluation launch
over all predicates and both parties, then match_query on the share bits (the
ANDs of each vertex and edge fold and both hop joins).  The reported value
counts DPF and DCF tree walks of both parties (a range is two DCF walks) per
second of step time, keygen included.

Extra fields: per-kernel durations (HIP events on the launch stream), the
roofline of the dominant kernel, the oracle timed on a bounded sample of edge
rows (checked bit for bit against the GPU shares at those rows), the vertex
filter over 2^22 rows, and a bounded served-vs-plain block.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

LOG_ROWS = 22
NBITS = 32
SEED = 20220907
# Issue floor of the T-table AES on one CDNA4 CU: 4 SIMDs x 16 lanes of VALU
# (64 lane-ops per clock) and one LDS pipe serving 32 random 32-bit reads per
# clock (128 B), at 2.4 GHz on 256 CUs.
CUS, CLOCK_HZ = 256, 2.4e9
HBM_BYTES_PER_S = 8e12                  # MI355X HBM3E, published
VALU_PER_CLK, LDS_PER_CLK = 64, 32
PEAK_INT_TOPS = CUS * VALU_PER_CLK * CLOCK_HZ / 1e12
# (VALU lane-ops, LDS table reads) of one tree hash H(s) = AES(sigma(s)) ^
# sigma(s) in this design: 9 full rounds of 4 columns x (4 byte-select perms,
# 4 reads, 2 xor3, 1 rotate), a last round of 4 x (4 perms, 4 reads, 2 perms,
# 1 xor3), 4 XORs of the first round key, 4 of the feed-forward and 2 for sigma.
AES_SINGLE = (9 * 4 * 7 + 4 * 7 + 4 + 4 + 2, 10 * 16)
# VALU lane-ops of one ChaCha12 block (64 bytes): 12 rounds of 4 quarter rounds
# of 4 adds, 4 xors and 4 rotates, and the 16 adds of the feed-forward.  The
# shuffle's tables and permutation keys are ChaCha12 output.
CHACHA_OPS = 12 * 4 * 12 + 16
NU = NBITS - 7                          # tree levels above the 128-bit leaf
# AES blocks per table row, both parties.  Eval: one hash per level and one
# leaf hash per walk (a range is two walks).  Dealer (one lane per party):
# roots (one block per lane per tree, one more for the range's wrap share),
# one hash per level and one leaf hash per tree.
AES_WORK = {
    "eval_eq": 2 * (NU + 1),
    "eval_range": 2 * 2 * (NU + 1),
    "keygen_eq": 2 * (1 + NU + 1),
    "keygen_range": 2 * (3 + 2 * (NU + 1)),
}


def aes_floor(blocks: float) -> dict:
    """Issue-bound time of that many AES blocks on the whole chip."""
    valu = blocks * AES_SINGLE[0]
    lds = blocks * AES_SINGLE[1]
    t_valu = valu / VALU_PER_CLK / CUS / CLOCK_HZ
    t_lds = lds / LDS_PER_CLK / CUS / CLOCK_HZ
    return {"blocks": blocks, "valu_ops": valu, "lds_reads": lds, "t_valu": t_valu, "t_lds": t_lds,
            "t_floor": max(t_valu, t_lds), "binding": "lds" if t_lds >= t_valu else "valu"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of every source and header the library is built from."""
    import hashlib

    from paper_2209_03526_amd import build as hip_build
    h = hashlib.sha256()
    for f in [*hip_build.SRCS, *hip_build.HEADERS]:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_record(kernel: str) -> dict:
    """The committed rocprofv3 counter summary of `kernel`
    (profiles/<kernel>.traffic.txt: HBM bytes per launch from FETCH_SIZE and
    WRITE_SIZE scaled by a plain copy's reading, and the clock and pipe busy
    fractions of the same launch from the SQ counters), or {} if there is none
    or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}.traffic.txt")
    if not os.path.exists(path):
        return {}
    vals = {}
    with open(path) as fh:
        for ln in fh:
            if ":" in ln and not ln.startswith("#"):
                k, v = ln.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256_16") != kernel_source_hash():
        return {}
    out = {}
    for key in ("traffic_bytes_per_launch", "clock_ghz", "valu_busy_pct", "lds_busy_pct"):
        try:
            out[key] = float(vals[key])
        except (KeyError, ValueError):
            pass
    return out


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from measured_record, or None."""
    return measured_record(kernel).get("traffic_bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample-rows", type=int, default=262144,
                    help="full: edge rows the oracle computes for the CPU baseline (bit-checked vs the GPU)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-vertex-filter", action="store_true", help="full: skip the 2^22-row vertex filter key")
    ap.add_argument("--no-serve", action="store_true", help="full: skip the bounded served-vs-plain block")
    ap.add_argument("--graph", action="store_true", help="full: also replay the step as one hipGraph")
    ap.add_argument("--log-rows", type=int, default=LOG_ROWS, help="vertex-filter: rows (log2)")
    ap.add_argument("--workload", default="full", choices=["full", "vertex-filter", "batch64", "serve", "next",
                                                           "secmatch"])
    ap.add_argument("--sweep-rates", default="50,100,200,250,300,350,400,450",
                    help="serve: offered rates (queries/s) of the token-given sweep")
    ap.add_argument("--keygen-rates", default="50,200", help="serve: rates of the keygen-included runs ('' = none)")
    ap.add_argument("--serve-seconds", type=float, default=30.0, help="serve: arrival window per rate")
    ap.add_argument("--slo-ms", default="50,100,250",
                    help="serve: p99 latency objectives (ms); the sweep of a path stops past the largest")
    ap.add_argument("--block-rates", default="100,400", help="full: rates of the bounded serving block")
    ap.add_argument("--block-seconds", type=float, default=15.0, help="full: arrival window per rate of the block")
    ap.add_argument("--budget-gb", type=float, default=0.0,
                    help="batch64: key memory budget of the batched runner (0: 96 GB); serve: admission budget "
                         "(0: 64 GB)")
    ap.add_argument("--chunk-log-rows", type=int, default=20, help="batch64: rows per keygen/eval chunk (log2)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 1 GiB device-to-device copy (reference dispatch for HBM byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus above 1 is not supported "
                                   "(a multi-GPU run would shard the rows of each table)"}))
        sys.exit(2)
    import torch
    from paper_2209_03526_amd import fss

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("calibration copy of 1 GiB done")
    if args.workload == "batch64":
        return run_batch64(args, torch, fss, dev)
    if args.workload == "serve":
        return run_serve(args, torch, fss, dev)
    if args.workload == "next":
        return run_next(args, torch, fss, dev)
    if args.workload == "secmatch":
        return run_secmatch_sweep(args, torch, dev)
    if args.workload == "vertex-filter":
        out = run_vertex_filter(args, torch, fss, dev, args.steps, args.warmup)
        print(json.dumps(out), flush=True)
        return
    log("generating the 2^22 / 2^25 Chung-Lu graph")
    graph3, query3 = synth.config3(3)
    out = run_full(args, torch, fss, dev, graph3, query3)
    if not args.no_vertex_filter:
        vf = run_vertex_filter(args, torch, fss, dev, 3, 1)
        out["vertex_filter_2p22"] = {k: vf[k] for k in ("value", "unit", "ms_per_step", "eval_only_evals_per_s",
                                                         "kernels", "config")}
    if not args.no_serve:
        out["serving"] = serve_block(args, torch, fss, dev, graph3)
    print(json.dumps(out), flush=True)


class Timer:
    """HIP events around launches on one stream, grouped by name."""

    def __init__(self, torch, stream):
        self.torch, self.stream, self.ev = torch, stream, {}

    def __call__(self, name, fn, record=True):
        if not record:
            return fn()
        e0 = self.torch.cuda.Event(enable_timing=True)
        e1 = self.torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        r = fn()
        e1.record(self.stream)
        self.ev.setdefault(name, []).append((e0, e1))
        return r

    def ms(self, name):
        """Mean duration of one call of `name` and the number of calls per step."""
        return float(np.mean([a.elapsed_time(b) for a, b in self.ev[name]]))


def kernel_row(ms: float, launches: int, blocks: float, hbm_bytes: float) -> dict:
    """One AES kernel's figures: `ms` per launch, `blocks` and `hbm_bytes` per launch."""
    f = aes_floor(blocks)
    t = ms / 1e3
    return {"ms": round(ms, 4), "launches_per_step": launches, "aes_blocks": int(blocks),
            "aes_gblocks_per_s": round(blocks / t / 1e9, 3), "floor_gblocks_per_s": round(blocks / f["t_floor"] / 1e9, 3),
            "binding_unit": f["binding"], "frac_of_floor": round(f["t_floor"] / t, 4),
            "valu_frac": round(f["t_valu"] / t, 4), "lds_frac": round(f["t_lds"] / t, 4),
            "hbm_bytes": int(hbm_bytes), "hbm_gb_per_s": round(hbm_bytes / t / 1e9, 1)}


def roofline_of(name: str, k: dict) -> dict:
    rec = measured_record(name)
    out = {"bound": "alu", "kernel": name, "achieved": k["aes_gblocks_per_s"], "peak": k["floor_gblocks_per_s"],
           "unit": "G AES-128 blocks/s (peak: the LDS-read issue floor of the T-table AES, 32 reads per clock "
                   "per CU, 160 per block, 256 CUs at 2.4 GHz)",
           "frac": k["frac_of_floor"], "traffic": rec.get("traffic_bytes_per_launch"),
           "binding_unit": k["binding_unit"], "valu_frac": k["valu_frac"], "lds_frac": k["lds_frac"],
           "aes_blocks_per_launch": k["aes_blocks"], "ms_per_launch": k["ms"]}
    if "clock_ghz" in rec:
        # the same floor at the clock the counters measured for this kernel
        clk = rec["clock_ghz"]
        out.update(measured_clock_ghz=clk, frac_at_measured_clock=round(k["frac_of_floor"] * 2.4 / clk, 4),
                   valu_busy_pct=rec.get("valu_busy_pct"), lds_busy_pct=rec.get("lds_busy_pct"))
    return out


def run_full(args, torch, fss, dev, graph, query):
    """The full path query a -> b -> c over the Chung-Lu graph (2^22 vertices,
    2^25 edges), 4 vertex and 2 edge predicates, both parties (Alg. 2)."""
    from paper_2209_03526_amd import autotune

    shares = synth.share_columns(SEED, graph.vcols)
    shares.update({"e:" + k: v for k, v in synth.share_columns(SEED + 1, graph.ecols).items()})
    masks = synth.pred_masks(SEED, query, graph)

    def T(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(dev)

    preds, walks = [], 0
    for k, p in enumerate(query.preds):
        on_edge = p.target >= query.n_qv
        x0, x1 = shares[("e:" if on_edge else "") + p.column]
        rows = graph.n_edges if on_edge else graph.n_vertices
        kind = fss.EQ if p.kind == "eq" else fss.RANGE
        preds.append({"p": p, "k": k, "kind": kind, "rows": rows, "table": "edges" if on_edge else "vertices",
                      "x0": T(x0), "x1": T(x1), "r": T(masks[k]),
                      "xhat": torch.empty(rows, dtype=torch.int32, device=dev),
                      "kb": fss.KeyBatch(kind, NBITS, rows, dev),
                      "bits": [torch.empty(fss.words(rows), dtype=torch.int32, device=dev) for _ in range(2)]})
        walks += 2 * rows * (1 if p.kind == "eq" else 2)
    evreqs = [(b, d["kb"], d["xhat"], d["bits"][b]) for d in preds for b in (0, 1)]
    queue = fss.Queue(len(evreqs), dev)
    plan = fss.Plan(SEED, query.query_id, query.n_qv, graph.n_vertices, graph.n_edges,
                    [(d["p"].target, None, None, tuple(d["bits"])) for d in preds],
                    T(graph.src), T(graph.dst), query.edges).allocate(dev)
    key_gb = sum(2 * d["kb"].bytes_per_party for d in preds) / 1e9
    log(f"inputs resident; keys {key_gb:.1f} GB for both parties")
    stream = torch.cuda.current_stream()
    tm = Timer(torch, stream)

    def step(record=True):
        for d in preds:
            p = d["p"]
            tm("open", lambda: fss.fss_mask_open(d["x0"], d["x1"], d["r"], d["xhat"], stream), record)
            tm(("keygen", p.kind, d["table"]),
               lambda: fss.fss_keygen(SEED, query.query_id, d["k"], p.a if p.kind == "eq" else p.lo, p.hi, d["r"],
                                      d["kb"], stream), record)
        tm("eval", lambda: fss.fss_eval_batch(evreqs, queue, stream), record)
        tm("tail", lambda: fss.match_query(plan, 3, stream), record)

    step(False)
    torch.cuda.synchronize()
    tuning = autotune.tune(lambda: fss.fss_eval_batch(evreqs, queue, stream), sum(d["rows"] for d in preds))
    log(f"evaluation shape chosen: {tuning}")
    for i in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    step_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        s0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - s0) * 1e3)
        log(f"step {i + 1}/{args.steps}: {step_ms[-1]:.2f} ms")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps

    kb_eq, kb_rg = fss.fss_key_bytes(fss.EQ, NBITS), fss.fss_key_bytes(fss.RANGE, NBITS)
    kernels = {}
    # dealer launches: one per predicate; blocks and bytes (keys of both parties
    # written, the mask read) per launch
    for d in preds:
        p = d["p"]
        name = f"k_keygen_{p.kind}[{d['table']} 2^{int(np.log2(d['rows']))}]"
        if name in kernels:
            kernels[name]["launches_per_step"] += 1
            continue
        kb = kb_eq if p.kind == "eq" else kb_rg
        kernels[name] = kernel_row(tm.ms(("keygen", p.kind, d["table"])), 1, AES_WORK["keygen_" + p.kind] * d["rows"],
                                   d["rows"] * (2 * kb + 4))
    ev_blocks = sum(AES_WORK["eval_" + d["p"].kind] * d["rows"] for d in preds)
    ev_bytes = sum(2 * d["rows"] * ((kb_eq if d["p"].kind == "eq" else kb_rg) + 4) + 8 * fss.words(d["rows"])
                   for d in preds)
    kernels["k_eval_queue"] = kernel_row(tm.ms("eval"), 1, ev_blocks, ev_bytes)
    share = {k: v["ms"] * v["launches_per_step"] for k, v in kernels.items()}
    dom = max(share, key=share.get)
    tail_ms = tm.ms("tail")
    open_ms = tm.ms("open")
    open_bytes = 16 * float(np.mean([d["rows"] for d in preds]))
    out = {
        "metric": "32-bit DCF/DPF evals/sec + query p50/p99 latency, served vs plain, 1 GPU",
        "value": walks / (ms / 1e3), "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "p50_step_ms": float(np.percentile(step_ms, 50)),
        "p99_step_ms": float(np.percentile(step_ms, 99)), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "full path query a->b->c: Chung-Lu (gamma 2.1) 2^22 vertices / 2^25 edges, "
                               "4 vertex + 2 edge predicates, 2 parties, 32-bit domain",
                   "step": "dealer keygen + open + evaluation of both parties + ANDs + hop joins; value = tree "
                           "walks per second, served vs plain p50/p99 in 'serving'",
                   "evals_per_step": walks, "key_gb_both_parties": round(key_gb, 2),
                   "eval_tuning": list(tuning)},
        "eval_only_evals_per_s": walks / (kernels["k_eval_queue"]["ms"] / 1e3),
        "kernels": kernels,
        "tail": {"ms": round(tail_ms, 4), "what": "match_query on evaluated bits: 3 fold ANDs, 2 hop joins "
                                                  "(gathers of both endpoints and 2 ANDs each)"},
        "hbm_kernels": {"k_mask_open": {"ms": round(open_ms, 4), "launches_per_step": len(preds),
                                        "hbm_gb_per_s": round(open_bytes / (open_ms / 1e3) / 1e9, 1),
                                        "frac_of_hbm_peak": round(open_bytes / (open_ms / 1e3) / HBM_BYTES_PER_S, 4)}},
        "roofline": roofline_of(dom if dom == "k_eval_queue" else dom.split("[")[0], kernels[dom]),
        "cpu_baseline": None,
    }
    out["roofline"]["kernel_launch"] = dom
    log(f"{out['value'] / 1e9:.3f} G evals/s, {ms:.2f} ms per step; dominant {dom}: {kernels[dom]}")
    if args.graph:
        out["graph_replay"] = graph_replay(torch, step, args.steps, walks)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_full(graph, query, shares, masks, plan, args.cpu_sample_rows)
    del preds, evreqs, plan, queue
    torch.cuda.empty_cache()
    return out


def graph_replay(torch, step, steps, walks):
    """The step captured once into a hipGraph and replayed: the per-call
    pipeline holds no memset, host copy or host wait, and a replay redoes the
    same work.  A failure is reported, not raised."""
    try:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step(False)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step(False)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        g_ms = (time.perf_counter() - t1) * 1e3 / steps
        del g
        log(f"graph replay: {g_ms:.2f} ms per step")
        return {"ms_per_step": g_ms, "value": walks / (g_ms / 1e3)}
    except Exception as exc:      # noqa: BLE001 -- the eager result stands
        log(f"graph replay failed: {exc}")
        return {"error": f"{type(exc).__name__}: {exc}"}


def run_vertex_filter(args, torch, fss, dev, steps, warmup):
    """Vertex filtering: 2^log_rows rows x 4 attributes, 2 equality and 2
    range predicates over all rows, both parties, the 4 bits ANDed into one."""
    n = 1 << args.log_rows
    log(f"vertex filter: generating {n} rows")
    graph, query = synth.config2(2, n=n)
    shares = synth.share_columns(SEED, graph.vcols)
    masks = synth.pred_masks(SEED, query, graph)

    def T(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(dev)

    preds = []
    for k, p in enumerate(query.preds):
        x0, x1 = shares[p.column]
        kind = fss.EQ if p.kind == "eq" else fss.RANGE
        preds.append({"p": p, "k": k, "kind": kind, "x0": T(x0), "x1": T(x1), "r": T(masks[k]),
                      "xhat": torch.empty(n, dtype=torch.int32, device=dev),
                      "kb": fss.KeyBatch(kind, NBITS, n, dev)})
    plan = fss.Plan(SEED, query.query_id, 1, n, 0, [(0, d["kb"], d["xhat"]) for d in preds]).allocate(dev)
    stream = torch.cuda.current_stream()
    tm = Timer(torch, stream)
    n_eq = sum(1 for d in preds if d["p"].kind == "eq")
    n_rg = len(preds) - n_eq
    walks = 2 * n * (n_eq + 2 * n_rg)

    def step(record=True):
        for d in preds:
            p = d["p"]
            tm("open", lambda: fss.fss_mask_open(d["x0"], d["x1"], d["r"], d["xhat"], stream), record)
            tm(("keygen", p.kind), lambda: fss.fss_keygen(SEED, query.query_id, d["k"], p.a if p.kind == "eq" else p.lo,
                                                          p.hi, d["r"], d["kb"], stream), record)
        tm("match", lambda: fss.match_query(plan, 3, stream), record)

    for _ in range(warmup):
        step(False)
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    kb_eq, kb_rg = fss.fss_key_bytes(fss.EQ, NBITS), fss.fss_key_bytes(fss.RANGE, NBITS)
    kernels = {
        "k_keygen_range": kernel_row(tm.ms(("keygen", "range")), n_rg, AES_WORK["keygen_range"] * n, n * (2 * kb_rg + 4)),
        "k_keygen_eq": kernel_row(tm.ms(("keygen", "eq")), n_eq, AES_WORK["keygen_eq"] * n, n * (2 * kb_eq + 4)),
        "match_query(k_eval+ands)": kernel_row(tm.ms("match"), 1,
                                               n * (n_eq * AES_WORK["eval_eq"] + n_rg * AES_WORK["eval_range"]),
                                               2 * n * (n_eq * (kb_eq + 4) + n_rg * (kb_rg + 4))),
    }
    share = {k: v["ms"] * v["launches_per_step"] for k, v in kernels.items()}
    dom = max(share, key=share.get)
    out = {"metric": "32-bit DCF/DPF evals/sec (vertex filter: dealer keygen + open + eval of both parties + AND)",
           "value": walks / (ms / 1e3), "unit": "evals/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
           "data": "synthetic",
           "config": {"workload": f"vertex filtering: 2^{args.log_rows} rows x 4 uint32 attrs, 2 eq + 2 range "
                                  "predicates, 2 parties, 32-bit domain", "rows": n, "evals_per_step": walks},
           "eval_only_evals_per_s": walks / (kernels["match_query(k_eval+ands)"]["ms"] / 1e3),
           "kernels": kernels, "roofline": roofline_of(dom, kernels[dom]), "cpu_baseline": None}
    log(f"vertex filter: {out['value'] / 1e9:.3f} G evals/s, {ms:.2f} ms per step")
    del preds, plan
    torch.cuda.empty_cache()
    return out


def batch_graph_replay(torch, runner, jobs, plain_out, outputs):
    """The whole batched pass (every wave's keygen and evaluation launches,
    the finishing match_query_batch calls and their descriptor uploads)
    captured into one hipGraph and replayed: time per replay and bit-exactness
    of every replay against the plain path.  A replay redoes the same batch
    (same seeds, so the same keys)."""
    try:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            runner.run(jobs)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            runner.run(jobs)
        torch.cuda.synchronize()
        ms, exact = [], True
        for _ in range(3):
            for j in jobs:
                for o in j.plan.out:
                    o.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.replay()
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
            exact = exact and all(np.array_equal(a[b], outputs(j.plan, j)[b])
                                  for a, j in zip(plain_out, jobs) for b in range(2))
        del g
        torch.cuda.synchronize()
        res = {"ms": round(float(np.median(ms)), 3), "replays": len(ms), "bit_exact_vs_plain": bool(exact),
               "queries_per_s": round(64 / (float(np.median(ms)) / 1e3), 1)}
    except Exception as e:     # the figure is optional; the batched pass above stands
        res = {"error": f"{type(e).__name__}: {e}"}
    log(f"graph replay of the batched pass: {res}")
    return res


def run_batch64(args, torch, fss, dev):
    """64 uneven queries over the power-law graph (2^22 vertices, 2^25 edges):
    plain = one query after another (per-predicate keygen launches, then
    match_query); batched = chunked waves of one persistent keygen launch and
    one persistent eval launch, then the queries' ANDs and joins."""
    from paper_2209_03526_amd import autotune
    from paper_2209_03526_amd.runner import ChunkedRunner, QueryJob

    log("generating the 2^22 / 2^25 power-law graph")
    g, _ = synth.config3(3)
    shares = synth.share_columns(SEED, g.vcols)
    shares.update({"e:" + k: v for k, v in synth.share_columns(SEED + 1, g.ecols).items()})
    mix = synth.batch_queries(4, g, count=64)

    def T(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(dev)

    jobs, walks = [], 0
    for q, rows in mix:
        view, erows = synth.candidate_view(g, rows)
        vsh = synth.view_shares(shares, g, view, erows)
        masks = synth.pred_masks(SEED, q, view)
        preds = []
        for k, p in enumerate(q.preds):
            on_edge = p.target >= q.n_qv
            x0, x1 = vsh[("e:" if on_edge else "") + p.column]
            nrow = view.n_edges if on_edge else view.n_vertices
            r = T(masks[k]) if nrow else torch.zeros(1, dtype=torch.int32, device=dev)
            xhat = torch.empty(max(nrow, 1), dtype=torch.int32, device=dev)
            if nrow:
                fss.fss_mask_open(T(x0), T(x1), r, xhat)
            walks += 2 * nrow * (1 if p.kind == "eq" else 2)
            preds.append(dict(target=p.target, kind=fss.EQ if p.kind == "eq" else fss.RANGE, rows=nrow,
                              a_or_lo=p.a if p.kind == "eq" else p.lo, hi=p.hi, r=r, xhat=xhat))
        jobs.append(QueryJob(SEED, q.query_id, q.n_qv, view.n_vertices, view.n_edges, preds,
                             T(view.src) if view.n_edges else None, T(view.dst) if view.n_edges else None,
                             edges=q.edges))
    torch.cuda.synchronize()
    log(f"64 queries ready: {walks / 1e6:.1f} M tree walks (both parties)")

    def outputs(plan, job):
        n_qe = len(job.edges) if job.edges is not None else job.n_qv - 1
        w = (job.n_vertices + 31) // 32 if job.n_qv == 1 else n_qe * ((job.n_edges + 31) // 32)
        return [plan.out[b][:w].cpu().numpy().copy() for b in range(2)]

    # plain: one query at a time
    def plain():
        res = []
        for job in jobs:
            kbs = []
            for k, p in enumerate(job.preds):
                kb = fss.KeyBatch(p["kind"], job.nbits, p["rows"], dev)
                if p["rows"]:
                    fss.fss_keygen(job.seed, job.query_id, k, p["a_or_lo"], p["hi"], p["r"], kb)
                kbs.append((p["target"], kb, p["xhat"]))
            plan = fss.Plan(job.seed, job.query_id, job.n_qv, job.n_vertices, job.n_edges, kbs, job.src,
                            job.dst, job.edges).allocate(dev)
            fss.match_query(plan)
            plan.release_inputs()      # the keys are not needed once match_query is enqueued
            res.append(plan)
            del kbs
        return res

    budget_gb = args.budget_gb or 96.0
    runner = ChunkedRunner(int(budget_gb * 1e9), chunk_rows=1 << args.chunk_log_rows, device=dev)
    # autotune the persistent evaluation shape on one representative wave
    probe = [j for j in jobs if any(p["rows"] >= 1 << 20 for p in j.preds)][:1] or jobs[:1]
    probe_rows = sum(p["rows"] for j in probe for p in j.preds)
    autotune.tune(lambda: runner.run(probe), probe_rows)
    autotune.tune_keygen(lambda: runner.run(probe), probe_rows)
    log(f"tuning chosen: {autotune.chosen()}, keygen tile x{autotune.chosen_keygen()}")

    times = {}
    for name in ("plain", "batched"):
        for rep in range(1 + args.warmup):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "plain":
                plans = plain()
            else:
                runner.waves = 0
                runner.run(jobs)
                waves_per_pass = runner.waves
                plans = [j.plan for j in jobs]
            torch.cuda.synchronize()
            times[name] = time.perf_counter() - t0
            log(f"{name} pass {rep + 1}: {times[name] * 1e3:.1f} ms")
        if name == "plain":
            plain_out = [outputs(p, j) for p, j in zip(plans, jobs)]
            del plans
            torch.cuda.empty_cache()
    exact = all(np.array_equal(a[b], outputs(j.plan, j)[b]) for a, j in zip(plain_out, jobs) for b in range(2))

    # one more batched pass with the persistent launches timed on the stream
    timings = []
    runner.run(jobs, timings)
    torch.cuda.synchronize()
    t_kind = {k: sum(a.elapsed_time(b) for kk, a, b in timings if kk == k) / 1e3 for k in ("keygen", "eval")}
    blocks = {"keygen": 0, "eval": 0}
    for j in jobs:
        for p in j.preds:
            kind = "eq" if p["kind"] == fss.EQ else "range"
            blocks["keygen"] += AES_WORK["keygen_" + kind] * p["rows"]
            blocks["eval"] += AES_WORK["eval_" + kind] * p["rows"]
    persistent = {}
    for k in ("keygen", "eval"):
        f = aes_floor(blocks[k])
        persistent["k_" + k + "_queue"] = {
            "ms_total": round(t_kind[k] * 1e3, 3), "aes_gblocks_per_s": round(f["blocks"] / t_kind[k] / 1e9, 3),
            "floor_gblocks_per_s": round(f["blocks"] / f["t_floor"] / 1e9, 3),
            "frac_of_floor": round(f["t_floor"] / t_kind[k], 4), "binding_unit": f["binding"]}
    log(f"persistent launches: {persistent}")
    graph_replay = batch_graph_replay(torch, runner, jobs, plain_out, outputs)
    out = {
        "metric": "queries/s, 64 uneven queries (1-5 predicates, 1-4 query vertices, 2^12..2^22 candidate rows)",
        "value": 64 / times["batched"], "unit": "queries/s", "n_gpus": 1, "higher_is_better": True,
        "plain_qps": 64 / times["plain"], "speedup_vs_plain": times["plain"] / times["batched"],
        "batched_ms": times["batched"] * 1e3, "plain_ms": times["plain"] * 1e3,
        "walks": walks, "batched_evals_per_s_incl_keygen": walks / times["batched"],
        "waves": waves_per_pass, "budget_gb": budget_gb, "chunk_rows": 1 << args.chunk_log_rows,
        "tuning": {str(k): v for k, v in autotune.chosen().items()},
        "keygen_tile_mult": {str(k): v for k, v in autotune.chosen_keygen().items()},
        "bit_exact_batched_vs_plain": bool(exact), "graph_replay": graph_replay, "dtype": "u32", "data": "synthetic",
        "persistent_kernels": persistent,
        "config": {"workload": "batch64: Chung-Lu 2^22 vertices / 2^25 edges, 64 queries"},
    }
    print(json.dumps(out), flush=True)


class ServeEnv:
    """The resident Chung-Lu graph (2^22 vertices, 2^25 edges), the 64-shape
    query mix and, for the token-given protocol, every mix entry's token dealt
    before the run."""

    def __init__(self, torch, fss, dev, graph=None, pool=True):
        from paper_2209_03526_amd import serving
        self.torch, self.fss, self.dev, self.serving = torch, fss, dev, serving
        if graph is None:
            log("generating the 2^22 / 2^25 Chung-Lu graph")
            graph, _ = synth.config3(3)
        self.g = graph
        self.vsh = synth.share_columns(SEED, graph.vcols)
        self.esh = synth.share_columns(SEED + 1, graph.ecols)
        self.rg = serving.resident_graph(graph.n_vertices, graph.n_edges, graph.src, graph.dst, self.vsh, self.esh,
                                         dev)
        self.mix = synth.batch_queries(4, graph, count=64)
        self.pool = None
        if pool:
            t0 = time.perf_counter()
            self.pool = serving.TokenPool(self.rg, self.mix, SEED, dev)
            log(f"tokens of the 64 mix entries dealt: {self.pool.key_bytes / 1e9:.1f} GB of keys in "
                f"{time.perf_counter() - t0:.1f} s")

    def free(self):
        self.pool = None
        self.rg = None
        self.torch.cuda.empty_cache()

    def requests(self, rate, seconds, seed):
        n = max(8, int(round(rate * seconds)))
        arrivals = self.serving.poisson_arrivals(rate, n, seed)
        entries = np.random.default_rng([seed, 1]).integers(0, len(self.mix), n)
        return [self.serving.GivenRequest(i, float(t), int(e)) for i, (t, e) in enumerate(zip(arrivals, entries))]

    def make(self, name, budget):
        s = self.serving
        if name == "served":
            return s.GivenServedPath(self.rg, self.pool, budget, device=self.dev)
        return s.GivenPlainPath(self.rg, self.pool, device=self.dev, sync=(name == "plain"))

    def run(self, name, rate, seconds, seed, budget, keep=None):
        """One path at one offered rate; `keep` (dict) receives the first output
        of each mix entry.  The run is cut (the rest counted as never served)
        once it is twice its arrival window plus 10 s old."""
        torch = self.torch
        reqs = self.requests(rate, seconds, seed)
        path = self.make(name, budget)
        seen = set()
        for r in reqs:
            r.keep = r.entry not in seen
            seen.add(r.entry)
        start = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        start.record()
        path.run(reqs, start, t0, deadline_s=2 * seconds + 10)
        wall = time.perf_counter() - t0
        res = self.serving.summarize(reqs, wall)
        res["offered_qps"] = rate
        if name == "served":
            res.update(waves=path.waves, batches=path.batches, max_wave=path.max_wave, max_in_flight=path.max_in_flight,
                       peak_admitted_gb=round(path.max_used / 1e9, 3))
        if keep is not None:
            for r in reqs:
                if r.keep and r.done_event is not None and r.entry not in keep:
                    keep[r.entry] = self.serving.given_outputs(r, self.pool)
        log(f"{name} at {rate:g} q/s: {res}")
        return res

    def oracle_check(self, outs, rows_per_entry=8):
        """Sampled rows of each kept output against the oracle (same tokens:
        same seeds, masks from the dealer's generator)."""
        from oracle import fss as ofss
        from oracle import match as omatch
        ok = True
        for e, out in sorted(outs.items()):
            q, rows = self.mix[e]
            view, erows = synth.candidate_view(self.g, rows)
            sh = {k: v for k, v in self.vsh.items()}
            sh.update({"e:" + k: v for k, v in self.esh.items()})
            vsh = synth.view_shares(sh, self.g, view, erows)
            masks = [ofss.masks(SEED, q.query_id, k, synth.rows_of_target(view, q, p.target))
                     for k, p in enumerate(q.preds)]
            nrows = view.n_vertices if q.n_qv == 1 else view.n_edges
            if nrows == 0:
                continue
            sample = np.unique(np.random.default_rng([SEED, e]).integers(0, nrows, rows_per_entry))
            want = omatch.sampled_outputs(NBITS, SEED, view, q, vsh, masks, sample)
            w = (nrows + 31) // 32
            for j in range(want.shape[0]):
                for b in range(2):
                    got = ofss.unpack_bits(out[b][j * w:(j + 1) * w], nrows)[sample]
                    ok &= bool(np.array_equal(got, want[j, b]))
        return ok


def max_rate_within(results, slo_ms):
    """Highest offered rate whose p99 meets the SLO (and all requests served)."""
    best = None
    for r in results:
        if r["p99_ms"] <= slo_ms and r["served"] == r["requests"]:
            best = r if best is None or r["offered_qps"] > best["offered_qps"] else best
    return best


def serve_sweep(env, names, rates, seconds, slos, budget, keep):
    """Each path at increasing offered rates until its p99 misses the largest
    SLO; per SLO, the highest rate within it."""
    out = {}
    for name in names:
        res = []
        for i, rate in enumerate(rates):
            res.append(env.run(name, rate, seconds, 1000 + i, budget, keep.setdefault(name, {})))
            env.torch.cuda.empty_cache()
            if res[-1]["p99_ms"] > max(slos) or res[-1]["served"] < res[-1]["requests"]:
                break
        out[name] = {"sweep": res, "at_slo": {}}
        for slo in slos:
            best = max_rate_within(res, slo)
            out[name]["at_slo"][str(int(slo))] = {
                "max_qps": best["qps"] if best else 0.0, "offered_qps": best["offered_qps"] if best else None,
                "p50_ms": best["p50_ms"] if best else None, "p99_ms": best["p99_ms"] if best else None}
    return out


def compare_outputs(keep):
    """Every path's kept output of a mix entry equals the served path's."""
    ref = keep.get("served", {})
    same = True
    for name, outs in keep.items():
        for e, o in outs.items():
            if e in ref:
                same &= all(np.array_equal(o[b], ref[e][b]) for b in range(2))
    return same


def run_serve(args, torch, fss, dev):
    """Serving over the resident 2^22 / 2^25 Chung-Lu graph, Poisson arrivals
    of the 64-shape mix.  Token given (primary): each path swept over offered
    rates (args.serve_seconds of arrivals each) up to the first whose p99
    misses the SLO; the ratio of the served path's highest rate within the SLO
    to the plain path's.  Then the keygen-inclusive protocol at the configured
    rates."""
    env = ServeEnv(torch, fss, dev)
    rates = [float(r) for r in args.sweep_rates.split(",")]
    budget = int(args.budget_gb * 1e9) if args.budget_gb else 64 * 10**9
    for name in ("plain", "served"):           # warm-up (allocator pools, first launches)
        env.run(name, 200.0, 1.0, 999, budget)
    keep = {}
    slos = [float(x) for x in args.slo_ms.split(",")]
    sweep = serve_sweep(env, ["plain", "served", "plain_pipelined"], rates, args.serve_seconds, slos, budget, keep)
    exact = compare_outputs(keep)
    oracle_ok = env.oracle_check(keep.get("served", {}))
    ratios = {}
    for slo in sweep["plain"]["at_slo"]:
        p = sweep["plain"]["at_slo"][slo]["max_qps"]
        pp = sweep["plain_pipelined"]["at_slo"][slo]["max_qps"]
        sv = sweep["served"]["at_slo"][slo]["max_qps"]
        ratios[slo] = {"served_qps": sv, "plain_qps": p, "plain_pipelined_qps": pp,
                       "served_vs_plain": (sv / p) if p else None, "served_vs_plain_pipelined": (sv / pp) if pp else None}
    main_slo = str(int(slos[len(slos) // 2]))
    out = {"metric": "served vs plain queries/s at equal p99 (token given), Poisson arrivals",
           "value": ratios[main_slo]["served_qps"], "unit": "queries/s", "n_gpus": 1, "higher_is_better": True,
           "slo_p99_ms": float(main_slo), "seconds_per_rate": args.serve_seconds, "at_equal_p99": ratios,
           "token_given": sweep, "bit_exact_across_paths": bool(exact), "oracle_sampled_rows_ok": bool(oracle_ok),
           "token_pool_gb": round(env.pool.key_bytes / 1e9, 1), "budget_gb": budget / 1e9,
           "dtype": "u32", "data": "synthetic",
           "config": {"workload": "serve: Chung-Lu 2^22 vertices / 2^25 edges resident, 64-shape query mix "
                                  "(1-5 predicates, 1-4 query vertices, 2^12..2^22 candidate rows)"},
           "paths": {"served": "continuous batching: the requests that arrive while <= 2 waves run form the next "
                               "wave (one persistent evaluation launch + one match_query_batch)",
                     "plain": "one request at a time, results awaited before the next request starts",
                     "plain_pipelined": "one request at a time on one stream, host runs ahead (no wait)"}}
    if args.keygen_rates:
        env.free()
        out["keygen_included"] = serve_keygen_included(args, torch, fss, dev, env.g)
    print(json.dumps(out), flush=True)


def serve_keygen_included(args, torch, fss, dev, graph):
    """Each request's token dealt on arrival, inside its latency: served
    (chunked waves over a 48 GB key arena) vs plain, at the given rates."""
    import copy

    from paper_2209_03526_amd import serving
    vsh = synth.share_columns(SEED, graph.vcols)
    esh = synth.share_columns(SEED + 1, graph.ecols)
    rg = serving.resident_graph(graph.n_vertices, graph.n_edges, graph.src, graph.dst, vsh, esh, dev)
    mix = synth.batch_queries(4, graph, count=64)

    def requests(arrivals, base):
        out = []
        for i, t in enumerate(arrivals):
            q, rows = mix[i % len(mix)]
            q = copy.deepcopy(q)
            q.query_id = base + i
            out.append(serving.Request(i, float(t), q, rows, SEED))
        return out

    def run(path, reqs):
        start = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        start.record()
        path.run(reqs, start, t0)
        return serving.summarize(reqs, time.perf_counter() - t0)

    paths = {"served": lambda: serving.ServedPath(rg, 64 * 10**9, key_arena_bytes=48 * 10**9, chunk_rows=1 << 20,
                                                  device=dev),
             "plain": lambda: serving.PlainPath(rg, device=dev, sync=True)}
    for name, make in paths.items():
        run(make(), requests(np.zeros(8), 90000))
        torch.cuda.empty_cache()
    res = {}
    for rate in [float(r) for r in args.keygen_rates.split(",")]:
        arrivals = serving.poisson_arrivals(rate, max(8, int(rate * args.serve_seconds)), int(rate))
        res[str(int(rate))] = {name: run(make(), requests(arrivals, 100000)) for name, make in paths.items()}
        log(f"keygen included, {rate:g} q/s: {res[str(int(rate))]}")
        torch.cuda.empty_cache()
    return res


def serve_block(args, torch, fss, dev, graph=None):
    """Bounded served-vs-plain block for the headline line (token given): both
    paths at one offered rate below the plain path's saturation and one at it,
    args.block_seconds of arrivals each."""
    env = ServeEnv(torch, fss, dev, graph)
    budget = 64 * 10**9
    for name in ("plain", "served"):
        env.run(name, 200.0, 1.0, 999, budget)
    keep, res = {}, {}
    for rate in [float(r) for r in args.block_rates.split(",")]:
        res[str(int(rate))] = {name: env.run(name, rate, args.block_seconds, 2000 + int(rate), budget,
                                             keep.setdefault(name, {})) for name in ("plain", "served")}
        res[str(int(rate))]["qps_ratio"] = res[str(int(rate))]["served"]["qps"] / res[str(int(rate))]["plain"]["qps"]
    out = {"protocol": "token given (keys dealt before arrival; latency from arrival to result shares)",
           "rates": res, "bit_exact_across_paths": bool(compare_outputs(keep)),
           "oracle_sampled_rows_ok": bool(env.oracle_check(keep.get("served", {}), 4)),
           "seconds_per_rate": args.block_seconds, "token_pool_gb": round(env.pool.key_bytes / 1e9, 1)}
    env.free()
    return out


def run_next(args, torch, fss, dev):
    """The rows built beyond the hot path, each timed alone with HIP events on
    the launch stream (median of 5 after one warm-up) against its floor: the
    larger of its algorithmic HBM bytes at 8 TB/s and its AES blocks at the
    single-block issue floor (160 LDS reads per block, 32 per clock per CU)."""
    stream = torch.cuda.current_stream()
    g = torch.Generator(device=dev)
    g.manual_seed(SEED)

    def rnd(*shape):
        return torch.randint(-2**31, 2**31 - 1, shape, dtype=torch.int32, device=dev, generator=g)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(5):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return float(np.median(ms))

    def row(name, ms, hbm_bytes, aes_blocks, what, chacha_blocks=0):
        t = ms / 1e3
        t_hbm = hbm_bytes / HBM_BYTES_PER_S
        t_aes = aes_floor(aes_blocks)["t_floor"]
        t_cc = chacha_blocks * CHACHA_OPS / (PEAK_INT_TOPS * 1e12)
        floors = {"hbm": t_hbm, "aes": t_aes, "chacha": t_cc}
        binding = max(floors, key=floors.get)
        out = {"ms": round(ms, 4), "hbm_gb": round(hbm_bytes / 1e9, 4), "hbm_gb_per_s": round(hbm_bytes / t / 1e9, 1)}
        if aes_blocks:
            out.update(aes_mblocks=round(aes_blocks / 1e6, 3), aes_gblocks_per_s=round(aes_blocks / t / 1e9, 2))
        if chacha_blocks:
            out.update(chacha_mblocks=round(chacha_blocks / 1e6, 3),
                       chacha_gblocks_per_s=round(chacha_blocks / t / 1e9, 2))
        out.update(binding=binding, frac_of_floor=round(floors[binding] / t, 4), work=what)
        log(f"{name}: {out}")
        return out

    res = {}
    # secEval over one-hot RSS attributes: 2^20 candidates, a 12-bit attribute (4,096 positions)
    ncand, npos = 1 << 20, 4096
    nwp = npos // 32
    kb = fss.KeyBatch(fss.RANGE, 12, 3, dev)
    zero = torch.zeros(3, dtype=torch.int32, device=dev)
    fss.fss_keygen(SEED, 7, 0, 100, 3000, zero, kb)
    evals = [torch.empty(nwp, dtype=torch.int32, device=dev) for _ in range(6)]
    sh = [rnd(nwp * ncand) for _ in range(3)]
    outs = [torch.empty((ncand + 31) // 32, dtype=torch.int32, device=dev) for _ in range(3)]
    terms = [((0, 0), (0, 1)), ((1, 1), (0, 2)), ((1, 2), (1, 0))]     # (party, replica) of each server's two keys

    eval_reqs = [(p, kb, r, npos, evals[2 * i + j]) for i, t in enumerate(terms) for j, (p, r) in enumerate(t)]

    def sec_eval():
        fss.fss_eval_all_batch(eval_reqs, stream)     # the six full-domain evaluations, side by side
        for i in range(3):
            fss.rss_sec_eval(ncand, npos, evals[2 * i], evals[2 * i + 1], sh[i], sh[(i + 1) % 3], outs[i], stream)

    res["sec_eval"] = row("sec_eval", timed(sec_eval), 3 * (2 * 4 * nwp * ncand + ncand // 8),
                          6 * npos * 2 * (12 - 7 + 1), f"3 servers x (2 full-domain range evals over {npos} positions + "
                          f"AND-parity over {ncand} candidates x {npos}-bit one-hot shares)")
    del sh, outs
    # RSS AND and re-share of 2^30 shared bits (2^25 words per share)
    nrows = 1 << 30
    nw = nrows // 32
    x3, y3, z3 = [rnd(nw) for _ in range(3)], [rnd(nw) for _ in range(3)], [rnd(nw) for _ in range(3)]
    keys = [11, 22, 33]
    prf_blocks = 3 * ((nw + 15) // 16)              # one ChaCha12 block per 16 words per PRF key
    res["rss_and"] = row("rss_and", timed(lambda: fss.rss_and(nrows, x3, y3, keys, 5, z3, stream)),
                         9 * 4 * nw, 0, f"{nrows} bits: 6 shares read, 3 written, 3 PRF streams", prf_blocks)
    res["rss_reshare"] = row("rss_reshare", timed(lambda: fss.rss_reshare(nrows, x3, keys, 6, z3, stream)),
                             6 * 4 * nw, 0, f"{nrows} bits: 3 shares read, 3 written, 3 PRF streams", prf_blocks)
    del x3, y3, z3
    # secShuffle of 2^22 records of 64 B, and the fetches
    nrec, nwords = 1 << 22, 16
    tbytes = nrec * nwords * 4
    d3 = [rnd(nrec * nwords) for _ in range(3)]
    o3 = [torch.empty(nrec * nwords, dtype=torch.int32, device=dev) for _ in range(3)]
    seeds = [101, 202, 303]
    work = {}

    def shuffle():
        work["w"] = fss.rss_shuffle(nrec, nwords, d3, seeds, o3, stream)

    # algorithmic work: 3 shares in, the two tables the pi23 gather takes (X1
    # and pi31(Y1 ^ T31)) written and read, 3 shares out; one ChaCha12 block
    # per 16-word slice of each of the 5 mask tables and per 8 rows of each of
    # the 3 permutations' keys (their bucket placing and ranking not counted)
    slices = nrec * ((nwords + 15) // 16)
    cc_blocks = 5 * slices + 3 * ((nrec + 7) // 8)
    res["rss_shuffle"] = row("rss_shuffle", timed(shuffle), 10 * tbytes, 0,
                             f"{nrec} records x {nwords * 4} B: 3 shares in, X1 and pi31(Y1 ^ T31) written and "
                             "read, 3 shares out; ChaCha12 for 5 mask tables and 3 permutations' keys (their "
                             "placing and ranking not counted)", cc_blocks)
    # the same shuffle in two parts: the permutations made ahead of the data
    # (rss_shuffle_prepare, seeds only), then the data-dependent launches
    perms = torch.empty(3 * nrec, dtype=torch.int32, device=dev)
    res["rss_shuffle_prepare"] = row("rss_shuffle_prepare",
                                     timed(lambda: work.__setitem__("p", fss.rss_shuffle_prepare(nrec, seeds, perms,
                                                                                                 stream))),
                                     3 * nrec * 4, 0, f"3 permutations of {nrec} rows from the pair seeds (keys "
                                     "counted; their placing and ranking not)", 3 * ((nrec + 7) // 8))
    res["rss_shuffle_prepared"] = row("rss_shuffle_prepared",
                                      timed(lambda: work.__setitem__("w", fss.rss_shuffle_prepared(
                                          nrec, nwords, d3, seeds, perms, o3, stream))),
                                      10 * tbytes, 0, f"{nrec} records x {nwords * 4} B with the permutations made: "
                                      "3 shares in, X1 and pi31(Y1 ^ T31) written and read, 3 shares out; ChaCha12 "
                                      "for 5 mask tables", 5 * slices)
    del perms
    xb = [rnd((nrec + 31) // 32) for _ in range(3)]
    f3 = [torch.empty(nwords, dtype=torch.int32, device=dev) for _ in range(3)]
    res["rss_fetch_unique"] = row("rss_fetch_unique",
                                  timed(lambda: fss.rss_fetch_unique(nrec, nwords, xb, d3, f3, stream)),
                                  3 * tbytes + 3 * nrec // 8, 0,
                                  f"selection product over {nrec} candidates x {nwords * 4} B, 3 shares")
    rows_out = torch.empty(nrec, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)

    def fetch_many():
        work["w"] = fss.rss_fetch_many(nrec, nwords, d3, seeds, o3, rows_out, count, stream)

    res["rss_fetch_many"] = row("rss_fetch_many", timed(fetch_many), 10 * tbytes + 3 * tbytes // 2, 0,
                                f"shuffle of {nrec} records (bit column + {(nwords - 1) * 4} B), open, compact "
                                "(about half kept)", cc_blocks)

    def compact():
        work["w"] = fss.rss_compact_valid(nrec, nwords, d3, seeds, o3, rows_out, count, stream)

    res["rss_compact_valid"] = row("rss_compact_valid", timed(compact), 10 * tbytes + 3 * tbytes // 2, 0,
                                   f"secAccess filter: shuffle {nrec} records of {nwords * 4} B, open parity, compact",
                                   cc_blocks)
    del d3, o3, xb
    # two-party FSS bits -> RSS: 2^30 rows (2^25 words per share)
    y2 = [rnd(nw) for _ in range(2)]
    z3 = [torch.empty(nw, dtype=torch.int32, device=dev) for _ in range(3)]
    res["rss_from_fss"] = row("rss_from_fss", timed(lambda: fss.rss_from_fss(nrows, y2, keys, 3, z3, stream)),
                              5 * 4 * nw, 0, f"{nrows} bits: 2 shares read, 3 written, 3 PRF streams", prf_blocks)
    del y2, z3
    # Alg. 1 encoding and Alg. 6 over k-grouped posting lists: 65,536 candidates,
    # 16,384 neighbour IDs (2 KB one-hot records), lists of 0..24 IDs, k = 4
    nc, xbits = 1 << 16, 1 << 14
    wx = xbits // 32
    types, adj, attr = synth.posting_graph(SEED, nc, xbits, 24, n_types=2)
    lengths = np.array([len(a) for a in adj], np.uint32)
    padded, _ = fss.rss_group_k(lengths, types, 4)
    slots = synth.posting_slots(SEED, lengths, padded)
    off = np.concatenate([[0], np.cumsum(padded)]).astype(np.uint32)
    nrec, lmax = int(off[-1]), int(padded.max())
    adj_off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.uint32)

    def Tu(a):
        return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(dev)

    d_off, d_adj_off, d_adj, d_slot = Tu(off), Tu(adj_off), Tu(np.concatenate(adj)), Tu(slots)
    post = [torch.empty(nrec * wx, dtype=torch.int32, device=dev) for _ in range(3)]
    res["rss_enc_posting_lists"] = row(
        "rss_enc_posting_lists",
        timed(lambda: work.__setitem__("w", fss.rss_enc_posting_lists(nc, xbits, d_adj_off, d_adj, d_slot, d_off, nrec,
                                                                      (71, 72), 0, post, stream))),
        3 * 4 * nrec * wx + 4 * nrec, 0, f"{nrec} one-hot records of {4 * wx} B (k = 4 groups): 3 shares written",
        2 * nrec * wx // 16)
    m = int(np.argmax(lengths))
    idm = [rnd((nc + 31) // 32) for _ in range(2)]
    onehot = np.zeros((nc + 31) // 32, np.uint32)
    onehot[m // 32] = 1 << (m % 32)
    idm.append(torch.bitwise_xor(torch.bitwise_xor(idm[0], idm[1]), Tu(onehot)))
    attr3 = [rnd(xbits * 2) for _ in range(3)]
    ids3 = [torch.empty(lmax * wx, dtype=torch.int32, device=dev) for _ in range(3)]
    attrs3 = [torch.empty(lmax * 2, dtype=torch.int32, device=dev) for _ in range(3)]
    rows_o = torch.empty(lmax, dtype=torch.int32, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    res["rss_sec_access"] = row(
        "rss_sec_access",
        timed(lambda: work.__setitem__("w", fss.rss_sec_access(nc, xbits, idm, d_off, lmax, post, 2, attr3, keys, 5,
                                                               seeds, ids3, attrs3, rows_o, cnt, stream))),
        3 * 4 * nrec * wx + 3 * 12 * lmax * wx + 3 * 4 * xbits * 2 * lmax, 0,
        f"one matched vertex over {nc} candidates ({nrec} records of {4 * wx} B): selection over all 3 shares, "
        f"re-share, shuffle/open/compact of {lmax} records, attribute selection over {xbits} records per kept ID",
        2 * 3 * lmax * wx // 16)
    del post, ids3, attrs3
    res["sec_match"] = sec_match_row(args, torch, dev)
    if not args.no_cpu_baseline:
        gpu_rate = {"sec_eval": ncand, "rss_and": nrows, "rss_reshare": nrows, "rss_shuffle": 1 << 22,
                    "rss_fetch_unique": 1 << 22, "rss_fetch_many": 1 << 22, "rss_compact_valid": 1 << 22,
                    "rss_from_fss": nrows, "rss_enc_posting_lists": nrec, "rss_sec_access": nc}
        for name, base in next_cpu_baselines().items():
            res[name]["cpu_baseline"] = base
            res[name]["gpu_rate"] = round(gpu_rate[name] / (res[name]["ms"] / 1e3), 1)
            res[name]["gpu_over_cpu"] = round(res[name]["gpu_rate"] / base["value"], 1)
    out = {"metric": "next rows: time per call and fraction of the HBM / AES / ChaCha floor", "value": None, "unit": "ms",
           "n_gpus": 1, "rows": res, "dtype": "u32", "data": "synthetic",
           "config": {"workload": "next: secEval 2^20 x 4096, RSS 2^30 bits, shuffle/fetch 2^22 x 64 B"}}
    print(json.dumps(out), flush=True)


def sec_match_row(args, torch, dev):
    """The paper's whole secMatch (Alg. 2) for one path query U -> P -> C over a
    typed graph (200 U, 8,000 P, 1,000 C vertices; up to 40 P neighbours per U
    and 3 C neighbours per P, k = 2 groups), all three servers on the GPU:
    wall-clock time of the call (its opens synchronise the host twice per
    target: after its secFetch calls and after its secAccess calls), beside
    the oracle on the same instance on one core."""
    from oracle import secmatch as osm
    from paper_2209_03526_amd import fss as lib
    from paper_2209_03526_amd import secmatch

    T = synth.TypedTarget
    n = {"U": 200, "P": 8000, "C": 1000}
    domains = {"U": {"city": 40}, "P": {"age": 100}, "C": {"industry": 16}}
    tg = synth.typed_graph(SEED, n, domains, {("U", "P"): 40, ("P", "C"): 3})
    q = synth.TypedQuery(31, [T("U", "city", "range", lo=3, hi=8), T("P", "age", "range", lo=25, hi=60),
                              T("C", "industry", "eq", a=5)])
    shares = synth.typed_shares(SEED, tg)
    padded = secmatch.padded_lengths(tg.adj, 2)
    slots = {pair: synth.posting_slots(SEED + e, np.array([len(a) for a in tg.adj[pair]], np.uint32), padded[pair])
             for e, pair in enumerate(sorted(tg.adj))}
    dom = {(t, a): d for t, v in tg.attrs.items() for a, (_, d) in v.items()}
    eg = secmatch.encode_graph(tg.n, dom, shares, tg.adj, slots, 2, device=dev)
    prf, c0, s0 = (41, 42, 43), 3, 900

    def once():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch = secmatch.sec_match(eg, q, SEED, prf, c0, s0, device=dev)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, ch

    once()
    runs = [once() for _ in range(5)]
    ms = float(np.median([r[0] for r in runs])) * 1e3
    chains = runs[-1][1]
    found = osm.reconstruct(tg, q, chains)
    ok = found == osm.plaintext_match(tg, q)
    out = {"ms": round(ms, 3), "binding": "launch-bound steps: two synchronisations per target (after its secFetch and its secAccess calls)",
           "results": len(found), "plaintext_match": ok,
           "work": "one 3-hop path query (Alg. 2: secEval, re-share, secFetch, secAccess per kept vertex) over "
                   f"{n['U']} U / {n['P']} P / {n['C']} C typed vertices, one-hot IDs, k = 2 posting lists"}
    if not args.no_cpu_baseline:
        enc = osm.encode(tg, shares, 2, SEED)
        _omp_threads(1)                       # the oracle's OpenMP loops on one core, like its numpy steps
        t0 = time.perf_counter()
        want, _ = osm.sec_match(tg, enc, q, SEED, prf, c0, s0)
        dt = time.perf_counter() - t0
        _omp_threads(int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0)))))
        exact = len(want) == len(chains) and all(
            np.array_equal(a[j], b[j]) for x, y in zip(want, chains) for a, b in zip(x, y) for j in range(3))
        out["cpu_baseline"] = {"value": round(dt * 1e3, 1), "unit": "ms per query", "cores": 1, "kind": "oracle",
                               "sample": "the same query on the same typed graph", "cpu": _cpu_model()}
        out["gpu_over_cpu"] = round(dt * 1e3 / ms, 1)
        out["shares_bit_exact_vs_oracle"] = exact
    log(f"sec_match: {out}")
    return out


def run_secmatch_sweep(args, torch, dev):
    """The paper's whole secMatch (Alg. 2) in the shape of its query-latency
    table (Table III: latency against k and the number of target vertices
    |q|), all three servers on one GPU: a typed graph of 200 U, 8,000 P and
    1,000 C vertices (up to 40 P per U, 3 C per P, 3 P friends per P), encoded
    with k = 2, 4, 6; path queries U -> P (|q| = 2), U -> P -> C (3) and
    U -> P -> P -> C (4), and Fig. 1's two-branch tree U -> P -> C, U -> P -> C
    (5).  Wall-clock median of 3 after one warm-up; every run's
    reconstruction is checked against plaintext matching."""
    from oracle import secmatch as osm
    from paper_2209_03526_amd import secmatch

    T = synth.TypedTarget
    n = {"U": 200, "P": 8000, "C": 1000}
    domains = {"U": {"city": 40}, "P": {"age": 100}, "C": {"industry": 16}}
    tg = synth.typed_graph(SEED, n, domains, {("U", "P"): 40, ("P", "C"): 3, ("P", "P"): 3})
    shares = synth.typed_shares(SEED, tg)
    u, p_, c = T("U", "city", "range", lo=3, hi=8), T("P", "age", "range", lo=25, hi=60), T("C", "industry", "eq", a=5)
    queries = {2: synth.TypedQuery(51, [u, p_]), 3: synth.TypedQuery(52, [u, p_, c]),
               4: synth.TypedQuery(53, [u, p_, T("P", "age", "range", lo=20, hi=70), c]),
               5: synth.TypedQuery(54, [u, p_, c, T("P", "age", "range", lo=40, hi=90),
                                        T("C", "industry", "range", lo=0, hi=8)], parents=[None, 0, 1, 0, 3])}
    dom = {(t, a): d for t, v in tg.attrs.items() for a, (_, d) in v.items()}
    rows = []
    for k in (2, 4, 6):
        padded = secmatch.padded_lengths(tg.adj, k)
        slots = {pair: synth.posting_slots(SEED + e, np.array([len(a) for a in tg.adj[pair]], np.uint32),
                                           padded[pair]) for e, pair in enumerate(sorted(tg.adj))}
        eg = secmatch.encode_graph(tg.n, dom, shares, tg.adj, slots, k, device=dev)
        for nq, q in queries.items():
            def once():
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = secmatch.sec_match(eg, q, SEED, (41, 42, 43), 3, 900, device=dev)
                torch.cuda.synchronize()
                return time.perf_counter() - t0, res
            once()
            runs = [once() for _ in range(3)]
            found = osm.reconstruct(tg, q, runs[-1][1])
            row = {"k": k, "q": nq, "ms": round(float(np.median([r[0] for r in runs])) * 1e3, 2),
                   "results": len(found), "plaintext_match": found == osm.plaintext_match(tg, q)}
            log(f"secmatch k={k} |q|={nq}: {row}")
            rows.append(row)
        del eg
    out = {"metric": "secMatch (Alg. 2) query latency against k and |q|, all three servers on one GPU",
           "value": None, "unit": "ms", "n_gpus": 1, "rows": rows, "dtype": "u32", "data": "synthetic",
           "config": {"workload": "typed graph 200 U / 8,000 P / 1,000 C, one-hot IDs; paths of 2-4 targets and "
                                  "Fig. 1's two-branch tree (|q| = 5)"}}
    print(json.dumps(out), flush=True)


def next_cpu_baselines():
    """The oracle of each row beyond the hot path, as it stands, timed on a
    bounded sample of the same kind of input (a few seconds each, all of the
    host's threads for the oracle's OpenMP loops) and reported per unit of the
    row's work: candidates, shared bits or records per second."""
    from oracle import access, rss as orss, shuffle as osh

    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    _omp_threads(threads)
    rng = np.random.default_rng(SEED)
    out = {}

    def rec(name, n, unit, what, fn):
        t0 = time.perf_counter()
        fn()
        dt = time.perf_counter() - t0
        out[name] = {"value": round(n / dt, 1), "unit": unit, "cores": threads, "kind": "oracle",
                     "sample": what, "seconds": round(dt, 3), "cpu": _cpu_model()}
        log(f"cpu baseline {name}: {out[name]}")

    # secEval: 8,192 candidates x 4,096-position one-hot shares, a range token
    c, npos = 1 << 13, 4096
    keys, nb = orss.token("range", npos, SEED, 7, 0, lo=100, hi=3000)
    sh = rng.integers(0, 2, (3, c, npos), dtype=np.uint8)
    rec("sec_eval", c, "candidates/s", f"{c} candidates x {npos} positions, range token",
        lambda: orss.server_shares("range", npos, keys, nb, sh))
    # RSS AND / re-share: 2^26 shared bits
    nb_bits = 1 << 26
    x3 = [rng.integers(0, 2**32, nb_bits // 32, dtype=np.uint64).astype(np.uint32) for _ in range(3)]
    y3 = [rng.integers(0, 2**32, nb_bits // 32, dtype=np.uint64).astype(np.uint32) for _ in range(3)]
    rec("rss_and", nb_bits, "shared bits/s", f"{nb_bits} bits", lambda: orss.rss_and(x3, y3, [11, 22, 33], 5, nb_bits))
    rec("rss_reshare", nb_bits, "shared bits/s", f"{nb_bits} bits", lambda: orss.reshare(x3, [11, 22, 33], 6, nb_bits))
    # shuffle and fetches: 2^18 records of 64 B (the selection product: 2^20)
    n, w = 1 << 18, 16
    d3 = [rng.integers(0, 2**32, (n, w), dtype=np.uint64).astype(np.uint32) for _ in range(3)]
    xb = [rng.integers(0, 2, n, dtype=np.uint8) for _ in range(3)]
    rec("rss_shuffle", n, "records/s", f"{n} records x {4 * w} B", lambda: osh.sec_shuffle(d3, 101, 202, 303))
    nu = 1 << 20
    du = [rng.integers(0, 2**32, (nu, w), dtype=np.uint64).astype(np.uint32) for _ in range(3)]
    xu = [rng.integers(0, 2, nu, dtype=np.uint8) for _ in range(3)]
    rec("rss_fetch_unique", nu, "candidates/s", f"{nu} candidates x {4 * w} B", lambda: osh.fetch_case1(xu, du))
    del du, xu
    rec("rss_fetch_many", n, "records/s", f"{n} records x {4 * w} B",
        lambda: osh.fetch_case2(xb, [t[:, 1:] for t in d3], 101, 202, 303))
    rec("rss_compact_valid", n, "records/s", f"{n} records x {4 * w} B",
        lambda: access.compact_valid(d3, (101, 202, 303)))
    y0, y1 = x3[0], x3[1]
    rec("rss_from_fss", nb_bits, "shared bits/s", f"{nb_bits} bits", lambda: orss.from_two_party(y0, y1, [11, 22, 33], 3,
                                                                                                    nb_bits))
    # Alg. 1 encoding and Alg. 6 over 4,096 candidates, 2,048 neighbour IDs
    types, adj, attr = synth.posting_graph(SEED, 4096, 2048, 24, n_types=2)
    lengths = np.array([len(a) for a in adj])
    padded, _ = access.group_k(lengths, types, 4)
    slots = synth.posting_slots(SEED, lengths, padded)
    enc = {}
    rec("rss_enc_posting_lists", int(padded.sum()), "records/s", f"{int(padded.sum())} records of 256 B",
        lambda: enc.update(r=access.rss_split_prf(access.encode_posting_lists_k(adj, 2048, padded, slots)[0], 71, 72, 0)))
    off = access.csr_offsets(padded)
    m = int(np.argmax(lengths))
    idm = np.zeros(4096, np.uint8)
    idm[m] = 1
    s1 = rng.integers(0, 2, 4096, dtype=np.uint8)
    s2 = rng.integers(0, 2, 4096, dtype=np.uint8)
    attr_sh = access.rss_split(attr, 5)
    rec("rss_sec_access", 4096, "candidates/s", "one matched vertex over 4,096 candidates, 2,048 IDs",
        lambda: access.sec_access_csr([s1, s2, idm ^ s1 ^ s2], enc["r"], off, attr_sh, 2048, [3, 4, 5], (7, 8, 9)))
    return out


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(n: int):
    """Set the OpenMP thread count of this process (the oracle's loops)."""
    import ctypes
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def cpu_baseline_full(graph, query, shares, masks, plan, nsample):
    """The oracle, as it stands, on a seeded sample of edge rows of the same
    graph, query and seeds: per sampled row both parties' keys and walks of
    every predicate the row's two hops need (source and destination vertex
    folds, the edge fold), the triple words and the ANDs.  Its shares are
    compared bit for bit with the GPU's at those rows.  All the host's
    threads, then one thread on an eighth of the sample."""
    from oracle import fss as ofss
    from oracle import match as omatch

    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    rng = np.random.default_rng(SEED)
    ne = graph.n_edges
    rows = np.unique(np.concatenate([[0, 1, 31, 32, ne - 2, ne - 1], rng.integers(0, ne, nsample)])).astype(np.int64)
    w = {"eq": 1, "range": 2}
    per_target = [sum(w[p.kind] for p in query.preds if p.target == t) for t in range(query.n_qv + query.n_qe)]
    walks_per_row = 2 * sum(per_target[a] + per_target[b] + per_target[query.n_qv + j]
                            for j, (a, b) in enumerate(query.qedges))

    def timed(sample, nthreads):
        _omp_threads(nthreads)
        log(f"cpu baseline: oracle on {sample.size} edge rows with {nthreads} threads")
        t0 = time.perf_counter()
        want = omatch.sampled_outputs(NBITS, SEED, graph, query, shares, masks, sample)
        return time.perf_counter() - t0, want

    dt, want = timed(rows, threads)
    we = (ne + 31) // 32
    exact = True
    for j in range(query.n_qe):
        for b in range(2):
            got = plan.out[b][j * we:(j + 1) * we].cpu().numpy().view(np.uint32)
            exact &= bool(np.array_equal(ofss.unpack_bits(got, ne)[rows], want[j, b]))
    log(f"cpu baseline: {dt:.1f} s, sampled shares bit-exact vs GPU: {exact}")
    small = rows[: max(64, rows.size // 8)]
    dt1, _ = timed(small, 1)
    _omp_threads(threads)
    return {"value": walks_per_row * rows.size / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{rows.size} seeded edge rows of the same graph/query/seeds: per row the keygen, open and "
                      f"both parties' walks of every predicate its two hops need ({walks_per_row} walks), "
                      "triples and ANDs",
            "seconds": round(dt, 3), "sampled_bit_exact_vs_gpu": exact, "cpu": _cpu_model(),
            "one_core": {"value": walks_per_row * small.size / dt1, "rows": int(small.size), "seconds": round(dt1, 3)}}


if __name__ == "__main__":
    main()
