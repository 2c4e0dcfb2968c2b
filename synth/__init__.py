"""Seeded synthetic inputs: graphs, attribute tables, their additive shares,
per-row masks and path queries.

This module holds none of the FSS method's arithmetic.  It produces the inputs
both the HIP path and the CPU oracle consume: plaintext columns (for brute-force
checking), the two servers' additive shares of every column (the outsourced
tables of Sec. V-B: x = x0 + x1 mod 2^32), the dealer's per-row masks r of the
masked-input approach (Sec. V-C), the public edge endpoints, and queries.
Every generator draws from numpy's PCG64 seeded through a SeedSequence.
"""
from .workloads import (  # noqa: F401
    Graph, Pred, Query, er_graph, chung_lu_graph, zipf_column, vertex_table,
    share_column, share_columns, pred_masks, tiny_graph, config1, config2, config3,
    batch_queries, rows_of_target, candidate_view, view_shares, onehot_rss, pack_word_major,
    posting_slots, posting_graph, TypedGraph, TypedTarget, TypedQuery, typed_graph, typed_shares,
    pack_records,
)
