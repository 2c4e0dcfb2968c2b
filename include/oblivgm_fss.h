/*
 * oblivgm_fss.h -- C ABI of the MI355X (gfx950) FSS-evaluation library.
 *
 * Masked-input function secret sharing over secret-shared attribute tables,
 * after OblivGM (arXiv 2209.03526): DPF evaluation for equality predicates and
 * DCF evaluation for range predicates (Sec. V-C), shared AND of predicate bits
 * (Sec. III-B, Sec. V-D), and a path query joined along public edge endpoints
 * (Alg. 2).  Two parties; both may be simulated on one GPU.
 *
 * Conventions for every call:
 *   - Buffers named d_* are DEVICE pointers owned by the caller.  The library
 *     never allocates or frees caller memory; it holds no device memory of its
 *     own except constant tables (batch calls stage their descriptors through
 *     a ring of eight pinned host buffers it owns; a buffer is reused once the
 *     copy that last read it has executed, which may make a batch call wait).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls validate
 *     their arguments synchronously, enqueue kernels on `stream` and return
 *     without waiting.  A negative return means nothing was enqueued;
 *     fss_last_error() (thread-local) then says why.  Device faults surface at
 *     the caller's next synchronisation.
 *   - Packed bits: row i is bit (i % 32) of 32-bit word i / 32; bits of rows
 *     beyond the table (pad bits of the last word) are 0 in every output share.
 *   - nbits (the FSS input domain) is 8..32.  Masked values are uint32; only
 *     their low nbits bits are evaluated.  Production inputs use nbits = 32.
 *   - Results are a pure function of the inputs: no atomics whose order matters.
 *
 * Key batch layout (per party), rows padded to Np = round_up(n, 64):
 *   a batch is a sequence of planes; plane p holds one field for every row,
 *   row e at byte offset plane_offset + e * field_size.
 *   DPF (nu = nbits - 7):   root[16] | cw_0[16] .. cw_{nu-1}[16] | cwleaf[16]
 *   DCF (nu = nbits - 7):   root[16] | cw_0[16] .. cw_{nu-1}[16] | vcw[4] | cwleaf[16]
 *   RANGE key:              DCF at U = hi + r, then DCF at L = lo + r
 *   The trees are half-trees (one hash per node, one correction word per
 *   level, right child = left child xor parent); bit i of vcw is the value
 *   correction of level i (level 0 consumes the most significant input bit);
 *   both trees stop nu levels down and a 128-bit leaf (cwleaf corrects the
 *   leaf hash of the last seed) answers the low 7 input bits; bit 31 of the
 *   upper DCF's vcw is the party's wrap share c_b.  Per element and party:
 *   DPF 16*(nbits - 5) bytes (432 at 32 bits), RANGE 2 * (16*(nbits - 5) + 4)
 *   bytes (872 at 32 bits).
 */
#ifndef OBLIVGM_FSS_H
#define OBLIVGM_FSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FSS_OK = 0,
    FSS_EINVAL = -1,        /* bad argument (null pointer, size, bound, party ...) */
    FSS_ENOMEM = -2,        /* caller-provided workspace too small */
    FSS_EDEVICE = -3,       /* HIP runtime error while enqueuing */
    FSS_EUNSUPPORTED = -4   /* valid request the library does not serve */
} fss_status;

typedef enum {
    FSS_EQ = 0,             /* x == a                          (one DPF)          */
    FSS_RANGE = 1           /* lo <= x < hi, half-open         (two DCFs + wrap)  */
} fss_kind;

/* One predicate's keys for n rows.  key[b] is party b's batch (device memory,
 * fss_keybatch_bytes(kind, nbits, n) bytes, 256-byte aligned). */
typedef struct fss_keybatch {
    int32_t  kind;          /* fss_kind */
    uint32_t nbits;         /* 8..32 */
    uint64_t n;             /* rows */
    void*    key[2];
} fss_keybatch;

/* Bytes of one element's key for one party (DPF 432 / RANGE 872 at 32 bits);
 * 0 for an invalid kind or nbits. */
uint64_t fss_key_bytes(int32_t kind, uint32_t nbits);

/* Bytes of a whole batch for one party: fss_key_bytes * round_up(n, 64). */
uint64_t fss_keybatch_bytes(int32_t kind, uint32_t nbits, uint64_t n);

/* Thread-local description of the last failed call ("" if none). */
const char* fss_last_error(void);

/* Library version string. */
const char* fss_version(void);

/* Release what the library holds on its own: the pinned staging buffers of
 * the batch calls (waiting for their last copies first) and the two streams
 * per device on which the shuffle calls make their permutations (drained
 * first).  Call it when no call is in flight on any thread; the library stays
 * usable (buffers and streams are re-created on demand).  FSS_EDEVICE if the
 * runtime reports an error while releasing. */
int fss_shutdown(void);

/*
 * Open the masked value (Sec. V-B additive shares, Sec. V-C masked input):
 *   d_xhat[i] = d_x0[i] + d_x1[i] + d_r[i]  (mod 2^32),  i < n.
 * In a deployment party b publishes x_b + r_b; with both parties simulated
 * the sum is formed at once.  d_xhat may alias none of the inputs' other rows
 * (in-place on d_x0 is allowed).
 */
int fss_mask_open(uint64_t n, const uint32_t* d_x0, const uint32_t* d_x1, const uint32_t* d_r,
                  uint32_t* d_xhat, void* stream);

/*
 * Dealer key generation (Def. 3 Gen; Sec. V-C token generation in its
 * masked-input form).  For every row e < out->n, with mask d_r[e]:
 *   FSS_EQ:    DPF at alpha = (a_or_lo + r) mod 2^nbits          (hi ignored)
 *   FSS_RANGE: DCF at U = hi + r and at L = a_or_lo + r, wrap share c_b with
 *              c_1 = c_0 xor [L > U]                               (lo <= hi)
 * Randomness (root seeds, c_0) comes from the dealer's counter-mode AES
 * generator keyed by `seed`, addressed by (query_id, pred_id, row).
 * Writes out->key[0] and out->key[1] (both parties).
 * Errors: EINVAL if out, its key pointers or d_r is NULL, nbits is outside
 * 8..32, a_or_lo / hi do not fit nbits, lo > hi, or a key pointer is not
 * 256-byte aligned.
 */
int fss_keygen(uint64_t seed, uint32_t query_id, uint32_t pred_id, uint32_t a_or_lo, uint32_t hi,
               const uint32_t* d_r, const fss_keybatch* out, void* stream);

/*
 * Dealer masks -- the per-row masks r of the masked-input approach (Sec. V-C),
 * drawn from the dealer's counter-mode generator: d_r[i] = little-endian word 0
 * of AES_{LE64(seed)||"OBLIVGM1"}(LE16 2 || LE16 0 || LE32 query_id ||
 * LE32 pred_id || LE32 (row_offset + i)), i < n.  (Callers may also supply
 * masks of their own; fss_keygen only needs them to be fresh per row.)
 */
int fss_dealer_masks(uint64_t seed, uint32_t query_id, uint32_t pred_id, uint32_t row_offset, uint64_t n,
                     uint32_t* d_r, void* stream);

/*
 * DPF evaluation (Def. 3 Eval) by `party` (0 or 1) on the opened
 * values d_xhat[0..n): writes ceil(n/32) packed share words to d_out_bits.
 * XOR of both parties' words is [x == a] per row.  k->kind must be FSS_EQ.
 */
int fss_eval_eq(int32_t party, const fss_keybatch* k, const uint32_t* d_xhat, uint32_t* d_out_bits,
                void* stream);

/*
 * Range evaluation: two DCF walks and the wrap share (interval
 * containment from comparisons, Sec. V-C).  XOR of both parties' words is
 * [lo <= x < hi].  k->kind must be FSS_RANGE.
 */
int fss_eval_lt(int32_t party, const fss_keybatch* k, const uint32_t* d_xhat, uint32_t* d_out_bits,
                void* stream);

/*
 * Shared AND of packed bits by Beaver triples (two-party analogue of the
 * AND of Sec. III-B; aggregation of predicates by AND, Sec. V-D).
 *
 * ss_triples: dealer's triples for AND number `and_id` of query `query_id`:
 *   d_trip0 / d_trip1 receive 3*nwords words a_b | b_b | c_b (party 0 / 1),
 *   with (a0^a1) & (b0^b1) = c0^c1, from the counter-mode generator (domain 4);
 *   nwords at most 4 * floor(2^32 / 5) (the block counter is 32-bit), else
 *   EUNSUPPORTED.
 * ss_and, phase SS_AND_OPEN:  out = d_b | e_b (2*nwords words),
 *   d_b = x ^ a_b, e_b = y ^ b_b.
 * ss_and, phase SS_AND_CLOSE: de_open = d | e (2*nwords words, the XOR of the
 *   two parties' OPEN messages); out = z_b (nwords words)
 *   = c_b ^ (d & b_b) ^ (e & a_b) ^ [party == 0](d & e), pad bits beyond nrows
 *   cleared.  x, y are ignored in CLOSE; de_open is ignored in OPEN.
 */
enum { SS_AND_OPEN = 0, SS_AND_CLOSE = 1 };
int ss_triples(uint64_t seed, uint32_t query_id, uint32_t and_id, uint64_t nwords, uint32_t* d_trip0,
               uint32_t* d_trip1, void* stream);
int ss_and(int32_t phase, int32_t party, uint64_t nrows, const uint32_t* d_x, const uint32_t* d_y,
           const uint32_t* d_triple, const uint32_t* d_de_open, uint32_t* d_out, void* stream);

/*
 * Edge matching -- a whole query graph (Def. 2; Alg. 2, secMatch, with public
 * edge endpoints).  The query has vertices 0 .. n_qv-1 and n_qe directed query
 * edges j = (a_j, b_j) given in q_edges as a_0, b_0, a_1, b_1, ...; n_qe == 0
 * with n_qv > 1 means the path v_0 -> v_1 -> ... -> v_{n_qv-1} (edge j =
 * (j, j+1)).  Query edges join distinct query vertices, no ordered pair comes
 * twice, every query vertex of a query of several lies on an edge, and a
 * one-vertex query has none (else EINVAL).
 *
 * Predicate k targets query vertex `target` (< n_qv; rows = vertex table) or
 * query edge target - n_qv (rows = edge table).  Its keys must have been made
 * with pred_id = k, and d_xhat holds the target table's opened values.
 * Semantics:
 *   1. each party evaluates every predicate (DPF / range) on its rows;
 *   2. per query vertex, then per query edge, its predicate bits are ANDed as
 *      a left fold in plan order (none: the public constant 1);
 *   3. per query edge j: h_j = (m_{a_j}[src] AND m_{b_j}[dst]) AND q_j over
 *      edge rows, where m[src] gathers each party's own share bit at the
 *      public index;
 *   4. ANDs are numbered 0,1,... in execution order (step 2 vertex folds, then
 *      edge folds, then two per query edge) and AND i uses the Beaver triple
 *      stream (seed, query_id, i); an AND with a public-1 operand is skipped
 *      and takes no number.
 * Output d_out[b] (party b): n_qv == 1 -> m_0, ceil(n_vertices/32) words;
 * else h_0 .. h_{n_qe-1} (n_qv - 1 of them for the path), each
 * ceil(n_edges/32) words, query edge after query edge.  The client joins the
 * h_j on their shared query vertices to list the matched subgraphs.
 * Workspace: match_workspace_bytes(plan) bytes of device memory, 256-aligned;
 * the library lays it out the same way on every call with the same plan.
 *
 * party_mask 3: both simulated parties at once (every AND opens, exchanges
 * and closes in one pass).
 * party_mask 1 / 2: ONE server's half (party 0 / party 1), run in rounds with
 * the peer.  An AND of level L (step L of a fold; a query edge's ANDs come
 * after the folds they read) opens in round L - 1 and closes in round L.
 * match_rounds() gives the number of exchange rounds R and the size of each
 * round's message.  Round r (plan->round = r, r = 0 .. R):
 *   r == 0: evaluates this party's predicate bits (only key[party] is read);
 *   r  > 0: closes the ANDs of level r with the peer's message of round r - 1
 *           (plan->d_peer_msg: d' || e' of each AND, AND-number order);
 *   r  < R: writes this party's message of round r (plan->d_msg, msg_words[r]
 *           words: d_b || e_b of each AND of level r + 1, AND-number order);
 *   outputs are complete in d_out[party] after round R.
 * The caller carries each message to the peer between calls (both parties'
 * calls for round r may run in any order).  The result shares are
 * bit-identical to those of party_mask 3.  Errors: EINVAL for a round beyond
 * R, a missing d_peer_msg (r > 0) or d_msg (r < R).
 */
#define FSS_MAX_QV 8
#define FSS_MAX_QE 16
#define FSS_MAX_PREDS 32

typedef struct fss_pred {
    int32_t target;                 /* query vertex, or n_qv + query edge */
    int32_t reserved;
    const fss_keybatch* keys;       /* host pointer; device key buffers */
    const uint32_t* d_xhat;         /* opened values of the target table */
    const uint32_t* d_bits[2];      /* optional: both parties' packed share bits of this
                                       predicate, already evaluated (e.g. chunk by chunk
                                       with fss_eval_batch); then keys and d_xhat are
                                       ignored.  NULL, NULL: match_query evaluates. */
} fss_pred;

typedef struct match_plan {
    uint64_t seed;                  /* dealer seed of the Beaver triples */
    uint32_t query_id;
    uint32_t n_qv;                  /* 1 .. FSS_MAX_QV */
    uint32_t n_pred;                /* 0 .. FSS_MAX_PREDS */
    uint32_t n_qe;                  /* 0 (the path, or no edge for n_qv == 1) .. FSS_MAX_QE */
    uint64_t n_vertices;
    uint64_t n_edges;
    const uint32_t* d_src;          /* public endpoints (n_edges each); unused when n_qv == 1 */
    const uint32_t* d_dst;
    const fss_pred* preds;          /* host array of n_pred predicates */
    const uint32_t* q_edges;        /* host array of 2 * n_qe query-edge ends; NULL if n_qe == 0 */
    uint32_t* d_out[2];
    void* d_workspace;
    uint64_t workspace_bytes;
    /* single-party runs (party_mask 1 or 2) only: */
    uint32_t round;                 /* round to run, 0 .. R */
    uint32_t reserved2;
    const uint32_t* d_peer_msg;     /* the peer's message of round - 1 */
    uint32_t* d_msg;                /* this party's message of round */
} match_plan;

uint64_t match_workspace_bytes(const match_plan* plan);
/* Exchange rounds R of a single-party run and, for r < min(R, cap), the
 * 32-bit words of round r's message (msg_words may be NULL). */
int match_rounds(const match_plan* plan, uint32_t* n_rounds, uint64_t* msg_words, uint32_t cap);
int match_query(const match_plan* plan, int32_t party_mask, void* stream);

/*
 * Batches: many requests in ONE persistent launch each.  The work of all
 * requests is cut into tiles (512 rows for keygen, 1024 x rows_per_thread
 * rows for evaluation); at most wg_per_cu workgroups per CU pull tiles from
 * a device work queue, ranges and larger tables first.  Results are
 * bit-identical to the per-request calls above, whatever the tuning.
 *
 * d_queue: caller-provided device memory of fss_queue_workspace_bytes(count)
 * bytes (256-aligned) holding the queue counter and the descriptors.  The
 * descriptors are staged through the library's ring of pinned host buffers
 * (see the conventions above); on a stream that is being captured into a
 * graph they are written by small store kernels whose arguments carry them
 * (2 KiB per launch), so that a replay reads the descriptors of the captured
 * call: the batch calls can be captured and replayed (a replay redoes the
 * same requests).  Batch calls on one stream run in order;
 * batches that share a d_queue must be on one stream.  A keygen batch runs as
 * one launch per key kind present (ranges first), each over its own tiles.
 *
 * fss_keygen_batch (dealer keygen for many predicates / queries): each request is one
 * fss_keygen call (same meaning, same checks).
 * fss_eval_batch (DPF / range evaluation for many predicates, parties, queries): each request
 * is one fss_eval_eq / fss_eval_lt call, chosen by keys->kind.
 * match_query_batch (edge matching for many plans): every predicate of every plan (of the
 * parties in party_mask) in one persistent launch; then the plans' ANDs and
 * joins merged into a few launches -- party_mask 3: one per AND level of the
 * deepest fold and one for all hop joins; party_mask 1 / 2: the round
 * plans[i].round of every plan (closes, gathers, openings: three launches).
 * Each plan has its own outputs, workspace and messages as in match_query.
 * The tail's descriptors take match_batch_queue_bytes(plans, count) bytes of
 * d_queue (at least that many must be passed); they are uploaded once per
 * call after the evaluation launch, in stream order.
 */
typedef struct fss_keygen_req {
    uint64_t seed;
    uint32_t query_id;
    uint32_t pred_id;
    uint32_t a_or_lo;
    uint32_t hi;
    const uint32_t* d_r;            /* masks of the request's rows */
    const fss_keybatch* out;
    uint32_t row_offset;            /* table row of the request's first row: a chunk of
                                       rows [row_offset, row_offset + out->n) gets exactly
                                       the keys a whole-table request gives those rows */
    uint32_t reserved;
} fss_keygen_req;

typedef struct fss_eval_req {
    int32_t party;
    int32_t reserved;
    const fss_keybatch* keys;
    const uint32_t* d_xhat;
    uint32_t* d_out_bits;
} fss_eval_req;

uint64_t fss_queue_workspace_bytes(uint64_t count);
int fss_keygen_batch(const fss_keygen_req* reqs, uint32_t count, void* d_queue, uint64_t queue_bytes, void* stream);
int fss_eval_batch(const fss_eval_req* reqs, uint32_t count, void* d_queue, uint64_t queue_bytes, void* stream);

/*
 * fss_eval_batch for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * requests, checks and results, but no d_queue argument and no allocation of
 * any kind -- the queue (tile counter and descriptors) lives in a file-scope
 * device array of the library, 64 KiB per GPU, held until the process ends,
 * and the descriptors reach it as kernel arguments (no pinned staging).
 * At most FSS_NOALLOC_EVAL_MAX requests per call, else EINVAL.  The array is
 * the current device's; `stream` must belong to that device.  Every call on
 * one GPU shares the array: calls that overlap on one GPU (other streams,
 * other threads) race -- serialise them.
 */
#define FSS_NOALLOC_EVAL_MAX 1360
int fss_eval_batch_noalloc(const fss_eval_req* reqs, uint32_t count, void* stream);
int match_query_batch(const match_plan* plans, uint32_t count, int32_t party_mask, void* d_queue,
                      uint64_t queue_bytes, void* stream);
uint64_t match_batch_queue_bytes(const match_plan* plans, uint32_t count);

/*
 * The paper's own secure predicate evaluation over one-hot attributes in
 * three-party binary replicated secret sharing (Sec. V-B, Sec. V-C token of
 * three replicated key pairs, Eq. predEval, Alg. 3).
 *
 * fss_eval_all: full-domain evaluation of ONE key -- party `party`'s key in row
 *   key_row of batch k -- at every public position x in [0, npoints)
 *   (npoints <= 2^nbits); ceil(npoints/32) packed words.  With masks r = 0 and
 *   rows 0..2 of one fss_keygen call as the replicas j = 1..3, party 0 / 1 of
 *   row j-1 is k_1^j / k_2^j.
 * rss_sec_eval: one server's two terms of Eq. predEval for every candidate c:
 *   out bit c = XOR_l (E_a[l] & S_a[c][l])  XOR  XOR_l (E_b[l] & S_b[c][l]),
 *   where E_a, E_b are the full-domain evaluations of the server's two keys
 *   (ceil(npos/32) words each) and S_a, S_b its two shares of the one-hot
 *   attribute vectors, word-major: word w of candidate c at [w * ncand + c],
 *   position p in bit p % 32 of word p / 32 (positions >= npos must be 0).
 *   The three servers' outputs XOR to the predicate bit (a 3-out-of-3 share).
 */
int fss_eval_all(int32_t party, const fss_keybatch* k, uint64_t key_row, uint64_t npoints, uint32_t* d_out_bits,
                 void* stream);

/*
 * fss_eval_all_batch: `count` fss_eval_all requests (same meaning, same checks;
 *   all are validated before anything is enqueued) run side by side, eight per
 *   launch -- e.g. the six keys of one secEval predicate.
 */
typedef struct fss_eval_all_req {
    int32_t party;
    int32_t reserved;
    const fss_keybatch* keys;
    uint64_t key_row;
    uint64_t npoints;
    uint32_t* d_out_bits;
} fss_eval_all_req;

int fss_eval_all_batch(const fss_eval_all_req* reqs, uint32_t count, void* stream);
int rss_sec_eval(uint64_t ncand, uint32_t npos, const uint32_t* d_eval_a, const uint32_t* d_eval_b,
                 const uint32_t* d_share_a, const uint32_t* d_share_b, uint32_t* d_out_bits, void* stream);

/*
 * rss_sec_eval_records: rss_sec_eval with candidate-major shares -- word w of
 *   candidate c at [c * ceil(npos/32) + w] -- the one-hot records that
 *   rss_fetch_many and rss_sec_access return (Alg. 2 evaluates the next
 *   target's predicate on the neighbours secAccess fetched).  Same output and
 *   errors; at most 2^32 candidates (FSS_EUNSUPPORTED).
 */
int rss_sec_eval_records(uint64_t ncand, uint32_t npos, const uint32_t* d_eval_a, const uint32_t* d_eval_b,
                         const uint32_t* d_share_a, const uint32_t* d_share_b, uint32_t* d_out_bits, void* stream);

/*
 * Three-party binary RSS arithmetic (Sec. III-B), all three parties simulated.
 * Share vectors are packed words (ceil(nrows/32) each); party P_i holds shares
 * i and i+1 (indices mod 3).  Zero sharing: <alpha>_i = F(k_i, j) ^ F(k_{i-1}, j)
 * with F(k, j) word w = slice word (w mod 16) of the ChaCha12 block (RFC 8439's
 * block function, 12 rounds) under key words (k mod 2^32, k div 2^32, 5, 0, 0, 0,
 * 0, 0) with state words 12-15 = (w div 16, j, 0, 0), its words read column by
 * column (slice word 4c + k = state word 4k + c); j = `counter` (fresh per call),
 * k_i = prf_keys[i].  Pad bits are cleared.  At most 2^41 rows (FSS_EUNSUPPORTED).
 * rss_reshare: three-out-of-three XOR shares x_i -> RSS shares z_i = x_i ^ <alpha>_i
 *   (P_i keeps z_i and obtains z_{i+1} from P_{i+1}; the paper words this as a
 *   send to P_{i+1}, which under its own holding convention is the same ring
 *   taken the other way).
 * rss_and: z = x AND y on RSS shares: P_i forms x_i y_i ^ x_i y_{i+1} ^ x_{i+1} y_i,
 *   then re-shares as above.
 * The outputs d_z must not overlap the inputs.
 */
/*
 * rss_from_fss: the masked-input path's two-party XOR shares -> RSS (the
 *   re-share of Sec. III-B applied to (y0, y1, 0)): the two FSS parties are
 *   servers P_1 (d_y[0], party 0's packed bits) and P_2 (d_y[1]); P_3's
 *   three-out-of-three share is zero, so z_1 = y0 ^ <alpha>_1,
 *   z_2 = y1 ^ <alpha>_2, z_3 = <alpha>_3 with <alpha>_i = F(k_i, j) ^ F(k_{i-1}, j)
 *   (j = counter), pad bits cleared.  XOR of the z_i = XOR of the y_b.
 */
int rss_from_fss(uint64_t nrows, const uint32_t* const d_y[2], const uint64_t prf_keys[3], uint32_t counter,
                 uint32_t* const d_z[3], void* stream);
int rss_reshare(uint64_t nrows, const uint32_t* const d_x[3], const uint64_t prf_keys[3], uint32_t counter,
                uint32_t* const d_z[3], void* stream);
int rss_and(uint64_t nrows, const uint32_t* const d_x[3], const uint32_t* const d_y[3], const uint64_t prf_keys[3],
            uint32_t counter, uint32_t* const d_z[3], void* stream);

/*
 * Secret-shared shuffle (Alg. 5, after Araki et al.) and secure fetching of the
 * matched records (Alg. 4), three servers simulated.  A table is nrows records
 * of nwords 32-bit words, row-major, in binary RSS: d_in[i] is share i+1 and
 * CS_i holds shares i and i+1.  seeds = {s12, s23, s31}, the pairwise seeds.
 * Each pair derives its permutations (stable sort of one 64-bit key per row)
 * and mask tables from its seed s with ChaCha12 (the ChaCha block function of
 * RFC 8439 with 12 rounds), key words (s mod 2^32, s div 2^32, 6, 0, 0, 0, 0, 0)
 * and state words 12-15 naming the block; a block's 16 words are read column
 * by column (slice word 4c + k = state word 4k + c):
 *   word w of record r of table t = slice word (w mod 16) of block
 *   (r, w div 16, t, nwords), T12 = 1, R2 = 2, T23 = 3, T31 = 4, R1 = 5;
 *   sort key of row r for pi12 / pi23 / pi31 = slice words 2e (low) and 2e+1
 *   (high), e = r mod 8, of block (r div 8, 0, 16+p, 0), p = 0 / 1 / 2;
 *   a permutation applied to a table gathers out[i] = in[perm[i]].
 * Up to 2^23 rows the whole call runs on the caller's stream (a table of at
 * most 1024 rows and 1024 16-word slices is shuffled by one workgroup); with
 * more rows, or a radix permutation method (rss_set_shuffle_tuning), the
 * permutations are made on two streams of the library's own besides the
 * caller's, ordered against the caller's stream with events.  Either way the
 * call's work is complete when the caller's stream reaches the call's end.
 * Up to 2^23 rows the calls hold no memset, host copy or host wait, so
 * rss_shuffle, rss_shuffle_prepare and rss_shuffle_prepared can be captured
 * into a graph and replayed (same seeds, same permutations); beyond that, or
 * with a radix permutation method, they return FSS_EUNSUPPORTED on a stream
 * being captured (their radix passes clear buffers with memset operations).
 * rss_fetch_many, rss_compact_valid and rss_sec_access are not for capture.
 * The messages follow the algorithm (its X_2 in CS2's step is the X1 it
 * received): X1 = pi31[pi12(D1^D2^T12)^T31]; Y1 = pi12(D3^T12);
 * C1 = pi23(X1^T23)^R2; C2 = pi23[pi31(Y1^T31)^T23]^R1; R3 = C1^C2.
 * rss_shuffle: d_out = (R1, R2, R3), an RSS of pi23(pi31(pi12(D))).
 * rss_fetch_unique (Case I, one matching candidate): d_x[i] = packed share i+1
 *   of the predicate bits; d_rows[i] = share i+1 of the records (ncand x nwords);
 *   d_out[i] (nwords) = XOR over candidates of the three-out-of-three products
 *   x_i r_i ^ x_i r_{i+1} ^ x_{i+1} r_i: additive shares of the matching record
 *   (rss_reshare turns them into RSS).
 * rss_fetch_many (Case II): word 0 bit 0 of each record of d_table is the
 *   shared predicate bit.  The table is shuffled, the bit column opened, and the
 *   kept records (words 1..nwords-1 of each share) are written in shuffled order
 *   to d_out[i] (capacity ncand x (nwords-1)), their shuffled positions to
 *   d_rows_out, their number to *d_count (device memory; read after the stream
 *   synchronises).  Workspaces: *_workspace_bytes, caller-provided device memory.
 * Outputs must overlap neither the inputs nor the workspace.
 */
uint64_t rss_shuffle_workspace_bytes(uint64_t nrows, uint32_t nwords);
int rss_shuffle(uint64_t nrows, uint32_t nwords, const uint32_t* const d_in[3], const uint64_t seeds[3],
                uint32_t* const d_out[3], void* d_work, uint64_t work_bytes, void* stream);

/*
 * The shuffle in two parts (Alg. 5 draws its permutations from the pairwise
 * seeds alone, before any data is involved): rss_shuffle_prepare makes the
 * three permutations ahead of the data, rss_shuffle_prepared runs the
 * data-dependent launches with them.  prepare + prepared = rss_shuffle, bit
 * for bit.
 * rss_shuffle_prepare: d_perms (device, 3 x nrows uint32, caller-owned) receives
 *   [inverse of pi12 | inverse of pi31 | pi23] for `seeds`; the call's work is
 *   complete when the stream reaches the call's end (it joins the library's
 *   own streams as rss_shuffle does).  Workspace:
 *   rss_shuffle_prepare_workspace_bytes(nrows).
 * rss_shuffle_prepared: as rss_shuffle, with d_perms as made by
 *   rss_shuffle_prepare for the same nrows and seeds (entries outside
 *   [0, nrows) leave rows unwritten, never an access out of bounds).
 *   Workspace: rss_shuffle_prepared_workspace_bytes(nrows, nwords).
 *   Outputs must overlap neither the inputs, d_perms nor the workspace.
 * Errors as rss_shuffle: more than 2^31 rows FSS_EUNSUPPORTED, NULL arguments
 * FSS_EINVAL, a short workspace FSS_ENOMEM.
 */
uint64_t rss_shuffle_prepare_workspace_bytes(uint64_t nrows);
int rss_shuffle_prepare(uint64_t nrows, const uint64_t seeds[3], uint32_t* d_perms, void* d_work,
                        uint64_t work_bytes, void* stream);
uint64_t rss_shuffle_prepared_workspace_bytes(uint64_t nrows, uint32_t nwords);
int rss_shuffle_prepared(uint64_t nrows, uint32_t nwords, const uint32_t* const d_in[3], const uint64_t seeds[3],
                         const uint32_t* d_perms, uint32_t* const d_out[3], void* d_work, uint64_t work_bytes,
                         void* stream);
int rss_fetch_unique(uint64_t ncand, uint32_t nwords, const uint32_t* const d_x[3], const uint32_t* const d_rows[3],
                     uint32_t* const d_out[3], void* stream);
/*
 * rss_fetch_table: secFetch's input table {x || id || d} (Alg. 4), for each
 *   of the three shares i: record c (1 + id_words + val_words words) holds bit
 *   c of d_bits[i] (packed, ceil(ncand/32) words) in bit 0 of word 0 (bits
 *   1..31 zero), then record c of d_ids[i] (id_words words, candidate-major),
 *   then record c of d_vals[i] (val_words words).  d_ids / d_vals may be NULL
 *   when their width is 0.  The table is the d_table of rss_fetch_many.
 *   Errors: EINVAL for a NULL buffer; EUNSUPPORTED beyond 65535 words per
 *   record or 2^32 candidates.
 */
int rss_fetch_table(uint64_t ncand, const uint32_t* const d_bits[3], uint32_t id_words, const uint32_t* const d_ids[3],
                    uint32_t val_words, const uint32_t* const d_vals[3], uint32_t* const d_out[3], void* stream);
uint64_t rss_fetch_many_workspace_bytes(uint64_t ncand, uint32_t nwords);
/* secAccess filter (Alg. 6): shuffle the fetched posting-list records, open
 * y = XOR of all bits of each record (1 for a one-hot ID, 0 for a dummy
 * all-zero ID), keep the whole records with y = 1 in shuffled order.  Same
 * outputs and workspace as rss_fetch_many, records of nwords words kept whole. */
int rss_compact_valid(uint64_t nrec, uint32_t nwords, const uint32_t* const d_table[3], const uint64_t seeds[3],
                      uint32_t* const d_out[3], uint32_t* d_rows_out, uint32_t* d_count, void* d_work,
                      uint64_t work_bytes, void* stream);
int rss_fetch_many(uint64_t ncand, uint32_t nwords, const uint32_t* const d_table[3], const uint64_t seeds[3],
                   uint32_t* const d_out[3], uint32_t* d_rows_out, uint32_t* d_count, void* d_work,
                   uint64_t work_bytes, void* stream);

/* Tile / occupancy shape of the persistent launches (process-wide):
 * rows_per_thread 1..8 (evaluation tile = 1024 * rows_per_thread rows),
 * wg_per_cu 1..2 (both the evaluation and the keygen queue), and the keygen
 * tile, 512 * tile_mult rows (tile_mult 1..8).  Chosen by the package's
 * autotuner; never changes results.  Not for use while another thread
 * enqueues batch calls. */
int fss_set_tuning(uint32_t rows_per_thread, uint32_t wg_per_cu);
int fss_get_tuning(uint32_t* rows_per_thread, uint32_t* wg_per_cu);
int fss_set_keygen_tuning(uint32_t tile_mult);
int fss_get_keygen_tuning(uint32_t* tile_mult);
/* How the shuffle's permutations of tables above 1024 rows are made
 * (process-wide); every method gives the same permutations (the stable
 * argsort of Alg. 5's keys), so results never change.  perm_method:
 *   0  radix pass on the run id, exact comparisons inside every run;
 *   1  radix pass, sorting networks in the wavefront for runs of <= 128 rows;
 *   2  (default) buckets of about 2^12 rows ordered in LDS, no sort library
 *      (tables of at most 2^23 rows; larger ones take method 1);
 *   3  buckets, exact comparisons inside every run;
 *   4  buckets, every bucket ordered by comparing every pair (the path of a
 *      bucket too large for LDS).
 * EINVAL for a value above 4. */
int rss_set_shuffle_tuning(uint32_t perm_method);
int rss_get_shuffle_tuning(uint32_t* perm_method);

/*
 * The paper's graph encoding with k-groups (Alg. 1) and secure neighbouring-
 * vertex access (Alg. 6) over it.  IDs of the neighbour type are 0 .. X-1
 * (x_bits = X) and travel as one-hot records of ceil(X/32) words; posting
 * lists are stored in CSR order, vertex v's padded list at records
 * [off[v], off[v+1]).
 *
 * rss_group_k (host arrays): Alg. 1's degree protection for one posting-list
 *   type.  The vertices of each type are taken k at a time in order of list
 *   length (ties by vertex ID), the remainder joining the type's last group
 *   (every group holds at least k vertices when the type has k); each list is
 *   padded to its group's longest: padded[v] receives that length, group[v]
 *   (NULL: not written) the group number (types in increasing order, groups
 *   in length order).  EINVAL for NULL arguments or k = 0.
 * rss_group_k_lists (host arrays): the same for vertices with nlists posting-
 *   list types (Alg. 1 groups a vertex once and pads each of its list types
 *   within the group, so every vertex shares its whole vector of padded
 *   lengths with k - 1 others).  lengths / padded: nlists x n, list type l of
 *   vertex v at [l * n + v]; the order is by the vector of lengths, list type
 *   0 first, ties by vertex ID.  rss_group_k is its nlists = 1 case.  EINVAL
 *   also for nlists = 0.
 * rss_enc_posting_lists (device): the padded lists as binary RSS of one-hot
 *   records.  d_adj_off (n+1) / d_adj: the true neighbour IDs of each vertex
 *   in CSR order; d_slot: the slot of each true ID within its padded list (the
 *   data owner's random placement); d_off (n+1): prefix sums of the padded
 *   lengths, nrec = off[n] records.  Every other record is the all-zero dummy
 *   ID.  Share 1 = F(split_keys[0], counter) and share 2 = F(split_keys[1],
 *   counter) over the table's words (row-major; F is the PRF of rss_reshare),
 *   share 3 = records ^ share 1 ^ share 2.  Workspace: 4 * nrec bytes.  A slot
 *   outside its padded list or an ID >= x_bits is skipped (no access out of
 *   bounds).
 * rss_sec_access (device, Alg. 6 for one matched vertex): d_idm: the three RSS
 *   shares of the matched vertex's one-hot ID over the ncand candidates (packed
 *   bits); d_off / d_post: the candidates' padded posting lists (as made
 *   above); lmax: the longest padded list (public); d_attr: the three shares of
 *   the X attribute records of the neighbour type (attr_words words each).
 *     1. P_m[l] = XOR_c id_m[c] AND id_{c,l} for l < lmax (a list shorter than l
 *        adds nothing), re-shared into RSS (prf_keys, counter);
 *     2. the lmax records shuffled (seeds, Alg. 5), the XOR of each record's bits
 *        opened, the records with 1 (valid IDs) kept in shuffled order:
 *        d_ids[i] (capacity lmax x ceil(X/32)), their shuffled positions
 *        d_rows_out, their number *d_count (device memory);
 *     3. per kept ID, d = XOR_x id[x] AND d_x; the kept IDs' attribute records
 *        re-shared together (counter + 1) into d_attrs[i] (capacity lmax x
 *        attr_words; rows beyond *d_count are shares of zero).
 *   Workspace: rss_sec_access_workspace_bytes(lmax, x_bits, attr_words).  lmax
 *   is 1..65535.  Its shuffle runs as rss_shuffle's does (on the caller's
 *   stream at these sizes); not for graph capture.
 */
int rss_group_k(uint64_t n, const uint32_t* lengths, const uint32_t* types, uint32_t k, uint32_t* padded,
                uint32_t* group);
int rss_group_k_lists(uint64_t n, uint32_t nlists, const uint32_t* lengths, const uint32_t* types, uint32_t k,
                      uint32_t* padded, uint32_t* group);
int rss_enc_posting_lists(uint64_t n, uint32_t x_bits, const uint32_t* d_adj_off, const uint32_t* d_adj,
                          const uint32_t* d_slot, const uint32_t* d_off, uint64_t nrec, const uint64_t split_keys[2],
                          uint32_t counter, uint32_t* const d_out[3], void* d_work, uint64_t work_bytes, void* stream);
uint64_t rss_sec_access_workspace_bytes(uint32_t lmax, uint32_t x_bits, uint32_t attr_words);
int rss_sec_access(uint64_t ncand, uint32_t x_bits, const uint32_t* const d_idm[3], const uint32_t* d_off,
                   uint32_t lmax, const uint32_t* const d_post[3], uint32_t attr_words,
                   const uint32_t* const d_attr[3], const uint64_t prf_keys[3], uint32_t counter,
                   const uint64_t seeds[3], uint32_t* const d_ids[3], uint32_t* const d_attrs[3],
                   uint32_t* d_rows_out, uint32_t* d_count, void* d_work, uint64_t work_bytes, void* stream);
/* rss_sec_access_batch: `count` independent rss_sec_access calls over the
 * same posting lists and attributes (Alg. 2 runs one per kept vertex),
 * enqueued on `stream` in order c = 0 .. count-1, one call of the library
 * instead of count.  Call c takes d_idm[3c .. 3c+2] (host array of device
 * pointers), counters[c] and seeds[3c .. 3c+2] (host arrays), and writes
 * d_ids[i] + c * lmax * ceil(x_bits/32), d_attrs[i] + c * lmax * attr_words,
 * d_rows_out + c * lmax and d_count + c; its results are those of the single
 * call with the same arguments.  One workspace of
 * rss_sec_access_workspace_bytes(lmax, x_bits, attr_words) serves every call
 * (they run in stream order).  count = 0 enqueues nothing.  EINVAL for a NULL
 * array or pointer, and the errors of rss_sec_access (returned by the first
 * call, before anything is enqueued). */
int rss_sec_access_batch(uint32_t count, uint64_t ncand, uint32_t x_bits, const uint32_t* const* d_idm,
                         const uint32_t* d_off, uint32_t lmax, const uint32_t* const d_post[3], uint32_t attr_words,
                         const uint32_t* const d_attr[3], const uint64_t prf_keys[3], const uint32_t* counters,
                         const uint64_t* seeds, uint32_t* const d_ids[3], uint32_t* const d_attrs[3],
                         uint32_t* d_rows_out, uint32_t* d_count, void* d_work, uint64_t work_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* OBLIVGM_FSS_H */
