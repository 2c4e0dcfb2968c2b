// fss_lib.hip -- kernels and C ABI of the masked-input FSS library (gfx950).
//
// What is computed, and where the paper defines it, is stated per entry point
// in include/oblivgm_fss.h.  This file holds:
//   k_mask_open            xhat = x0 + x1 + r                          (HBM stream)
//   k_keygen_eq/_range     dealer: DPF / 2xDCF Gen per row             (LDS + VALU, AES)
//   k_eval                 DPF / 2xDCF Eval per row, ballot            (LDS + VALU, AES)
//   k_triples              dealer: Beaver triples                      (LDS + VALU, AES)
//   k_and_open/close, k_and_both, k_interleave, k_gather, k_public_one  ANDs, joins  (HBM stream)
// and the host code of the C ABI (validation, launch, match_query plan).
//
// Every AES-using kernel runs 1024-thread workgroups that first fill the
// 64 KiB replicated T-tables in LDS (aes_gfx950.hpp).  One thread owns one
// table row (one element, one predicate, one party); the 64 lanes of a wave
// own 64 consecutive rows, so the per-level correction words of a wave are one
// contiguous 1 KiB read, and the wave's 64 output bits are one ballot.

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/oblivgm_fss.h"
#include "aes_gfx950.hpp"
#include "chacha_gfx950.hpp"
#include "common.hpp"

using namespace ogm;

namespace ogm {

std::string& last_error() {
    thread_local std::string err;
    return err;
}

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    last_error() = buf;
    return code;
}

int check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FSS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return FSS_OK;
}

RoundKeys seed_key(uint64_t seed) {
    uint8_t k[16];
    for (int i = 0; i < 8; i++) k[i] = (uint8_t)(seed >> (8 * i));
    memcpy(k + 8, "OBLIVGM1", 8);
    return expand_key(k);
}

}  // namespace ogm

namespace {

constexpr int kBlock = 1024;            // threads per AES workgroup
constexpr int kEvalInline = 16;         // eval descriptors carried in kernel arguments

__constant__ AesTables g_tables = kTables;

// ----------------------------------------------------------------- key layout

inline __host__ __device__ uint64_t pad_rows(uint64_t n) { return (n + 63) & ~63ull; }

// Byte offsets of the planes of one DPF / DCF sub-key, relative to its start.
struct DpfPlanes {
    uint64_t np;
    uint32_t nu;            // levels walked: nbits - 7
    __host__ __device__ uint64_t root() const { return 0; }
    __host__ __device__ uint64_t cw(uint32_t i) const { return 16 * np * (1 + (uint64_t)i); }
    __host__ __device__ uint64_t cwleaf() const { return 16 * np * (1 + (uint64_t)nu); }
    __host__ __device__ uint64_t bytes() const { return cwleaf() + 16 * np; }
};

struct DcfPlanes {
    uint64_t np;
    uint32_t nu;
    __host__ __device__ uint64_t root() const { return 0; }
    __host__ __device__ uint64_t cw(uint32_t i) const { return 16 * np * (1 + (uint64_t)i); }
    __host__ __device__ uint64_t vcw() const { return 16 * np * (1 + (uint64_t)nu); }   // bit 31: wrap share c_b
    __host__ __device__ uint64_t cwleaf() const { return vcw() + 4 * np; }
    __host__ __device__ uint64_t bytes() const { return cwleaf() + 16 * np; }
};

template <class T>
__device__ __forceinline__ const T& at(const uint8_t* base, uint64_t off, uint64_t row) {
    return ((const T*)(base + off))[row];
}

template <class T>
__device__ __forceinline__ T& at_w(uint8_t* base, uint64_t off, uint64_t row) {
    return ((T*)(base + off))[row];
}

// ----------------------------------------------------------------- half-tree nodes
//
// A node is a 128-bit seed s with bit 1 clear; t(s) = bit 0.  Expanding it
// costs one hash h = H(s): its bit 1 is the node's value bit v, and with that
// bit cleared (h') the children are
//   left  = h' ^ t(s) * CW_i,      right = left ^ s,
// so one correction word per level serves both children.

// h' (bit 1 of H(s) cleared); v = bit 1 of H(s).
__device__ __forceinline__ uint4 expand(uint4 s, uint32_t& v, const uint32_t* tab, LaneOff loff) {
    uint4 h = tree_hash(s, tab, loff);
    v = (h.x >> 1) & 1u;
    h.x &= ~2u;
    return h;
}

// The child of s on side xi: h' ^ t(s) * cw ^ xi * s.
__device__ __forceinline__ uint4 child(uint4 s, uint4 h, uint4 cw, uint32_t xi) {
    const uint32_t tm = 0u - (s.x & 1u), xm = 0u - xi;
    return make_uint4(xor3(h.x, cw.x & tm, s.x & xm), xor3(h.y, cw.y & tm, s.y & xm),
                      xor3(h.z, cw.z & tm, s.z & xm), xor3(h.w, cw.w & tm, s.w & xm));
}

// Leaf block of node s under its correction word: H(s ^ 2) ^ t(s) * cwleaf
// (tree seeds have bit 1 clear, so a leaf input is never an expansion input).
__device__ __forceinline__ uint4 leaf(uint4 s, uint4 cwleaf, const uint32_t* tab, LaneOff loff) {
    uint4 u = s;
    u.x ^= 2u;
    return xor4(tree_hash(u, tab, loff), and4(cwleaf, 0u - (s.x & 1u)));
}

// Bit idx (0..127) of a 128-bit block.
__device__ __forceinline__ uint32_t block_bit(uint4 g, uint32_t idx) {
    const uint32_t word = idx < 64 ? (idx < 32 ? g.x : g.y) : (idx < 96 ? g.z : g.w);
    return (word >> (idx & 31u)) & 1u;
}

// ----------------------------------------------------------------- Eval (DPF, DCF)

// A party's DPF output bit at x: nu = nbits - 7 levels, then the 128-bit leaf
// answers the low 7 bits.  No party index is needed: t is bit 0 of the seed.
__device__ __forceinline__ uint32_t dpf_eval(const uint8_t* key, uint64_t np, uint64_t row, uint32_t nbits,
                                             uint32_t x, const uint32_t* tab, LaneOff loff) {
    const DpfPlanes P{np, nbits - 7};
    uint4 s = at<uint4>(key, P.root(), row);
    for (uint32_t i = 0; i < P.nu; i++) {
        const uint4 cw = at<uint4>(key, P.cw(i), row);
        const uint32_t xi = (x >> (nbits - 1 - i)) & 1u;
        uint32_t v;
        const uint4 h = expand(s, v, tab, loff);
        s = child(s, h, cw, xi);
    }
    return block_bit(leaf(s, at<uint4>(key, P.cwleaf(), row), tab, loff), x & 127u);
}

// A party's share of [lo <= x < hi]: DCF_U(x) ^ DCF_L(x) ^ c_b, both walks in
// step over the nu high bits, each adding v ^ t * VCW_i of the node it leaves;
// then each DCF's 128-bit leaf answers the low 7 bits.
__device__ __forceinline__ uint32_t range_eval(const uint8_t* key, uint64_t np, uint64_t row, uint32_t nbits,
                                               uint32_t x, const uint32_t* tab, LaneOff loff) {
    const DcfPlanes P{np, nbits - 7};
    const uint8_t* ku = key;
    const uint8_t* kl = key + P.bytes();
    uint4 su = at<uint4>(ku, P.root(), row);
    uint4 sl = at<uint4>(kl, P.root(), row);
    const uint32_t vcu = at<uint32_t>(ku, P.vcw(), row);
    const uint32_t vcl = at<uint32_t>(kl, P.vcw(), row);
    uint32_t v = 0;
    for (uint32_t i = 0; i < P.nu; i++) {
        const uint4 cwu = at<uint4>(ku, P.cw(i), row);
        const uint4 cwl = at<uint4>(kl, P.cw(i), row);
        const uint32_t xi = (x >> (nbits - 1 - i)) & 1u;
        uint32_t vu, vl;
        const uint4 hu = expand(su, vu, tab, loff);
        const uint4 hl = expand(sl, vl, tab, loff);
        v ^= vu ^ vl ^ (su.x & (vcu >> i)) ^ (sl.x & (vcl >> i));
        su = child(su, hu, cwu, xi);
        sl = child(sl, hl, cwl, xi);
    }
    const uint4 gu = leaf(su, at<uint4>(ku, P.cwleaf(), row), tab, loff);
    const uint4 gl = leaf(sl, at<uint4>(kl, P.cwleaf(), row), tab, loff);
    const uint32_t idx = x & 127u;
    return (v ^ block_bit(gu, idx) ^ block_bit(gl, idx) ^ (vcu >> 31)) & 1u;
}

struct EvalDesc {
    const uint8_t* key;
    const uint32_t* xhat;
    uint32_t* out;
    uint64_t n;
    uint32_t kind;
    uint32_t nbits;
    uint32_t party;
    uint32_t block_start;   // first workgroup of this descriptor
};

struct EvalBatch {
    uint32_t count;
    uint32_t total_blocks;
    EvalDesc d[kEvalInline];
};

// One workgroup-sized slice of rows [row0, row0 + kBlock) of descriptor D:
// every thread evaluates one row, each wave stores its 64 bits as two words.
__device__ __forceinline__ void eval_rows(const EvalDesc& D, uint64_t row0, const uint32_t* tab, LaneOff loff) {
    const uint64_t row = row0 + threadIdx.x;
    const uint64_t np = pad_rows(D.n);
    uint32_t bit = 0;
    if (row < D.n) {
        const uint32_t x = D.xhat[row];
        if (D.kind == FSS_EQ)
            bit = dpf_eval(D.key, np, row, D.nbits, x, tab, loff);
        else
            bit = range_eval(D.key, np, row, D.nbits, x, tab, loff);
    }
    const uint64_t ballot = __ballot(bit);
    if ((threadIdx.x & 63u) == 0) {
        const uint64_t w = row >> 5;          // row is a multiple of 64 here
        const uint64_t nwords = (D.n + 31) >> 5;
        if (w < nwords) D.out[w] = (uint32_t)ballot;
        if (w + 1 < nwords) D.out[w + 1] = (uint32_t)(ballot >> 32);
    }
}

__global__ __launch_bounds__(kBlock) void k_eval(EvalBatch batch) {
    __shared__ uint32_t tab[kLdsTableWords];
    lds_table_fill(tab, g_tables.t0);
    __syncthreads();

    uint32_t di = 0;
    while (di + 1 < batch.count && blockIdx.x >= batch.d[di + 1].block_start) di++;
    const EvalDesc& D = batch.d[di];
    eval_rows(D, (uint64_t)(blockIdx.x - D.block_start) * kBlock, tab, lane_offset());
}

// ----------------------------------------------------------------- dealer (keys, triples)

struct DealerArgs {
    RoundKeys rk;           // AES key schedule of LE64(seed) || "OBLIVGM1"
    uint8_t* key0;
    uint8_t* key1;
    const uint32_t* r;
    uint64_t n;
    uint32_t kind;
    uint32_t nbits;
    uint32_t query;
    uint32_t pred;
    uint32_t a_or_lo;
    uint32_t hi;
    uint32_t row_offset;    // table row of key row 0 (dealer randomness is addressed by table row)
    uint32_t pad;
};

// Counter-mode block (domain, j, query, pred, elem) under the dealer key.
__device__ __forceinline__ uint4 rng_block(const RoundKeys& rk, uint32_t domain, uint32_t j, uint32_t query,
                                           uint32_t pred, uint32_t elem, const uint32_t* tab, LaneOff loff) {
    const uint4 in = make_uint4(domain | (j << 16), query, pred, elem);
    return aes128_encrypt(in, ArgKey{rk}, tab, loff);
}

// An empty asm statement that claims to rewrite v and memory: the value is
// complete here, in registers, and neither its computation nor the table reads
// of the next one move across this point (the dealer's root blocks are drawn
// one after the other instead of side by side, which bounds register use).
__device__ __forceinline__ void pin_in_vgprs(uint4& v) {
    asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w) : : "memory");
}

__device__ __forceinline__ void pin_in_vgprs(uint32_t& v) { asm volatile("" : "+v"(v) : : "memory"); }

// The dealer's work for one row is split over a lane pair: even lane = party 0,
// odd lane = party 1.  Each lane expands only its own seed (one hash per
// level); what Gen needs of the other party -- its hash and value bit -- comes
// from the partner lane through a DPP quad permutation (lanes 0<->1, 2<->3),
// so both lanes form the same correction words and each writes them into its
// own party's key.

// Value of `v` in the partner lane (lane ^ 1).
__device__ __forceinline__ uint32_t partner(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
}

__device__ __forceinline__ uint4 partner4(uint4 v) {
    return make_uint4(partner(v.x), partner(v.y), partner(v.z), partner(v.w));
}

// Gen of one DPF (DCF = false) or DCF tree for alpha over nbits, this lane's
// party b, whose root is s; delta is the dealer's offset (both lanes hold it).
// Along alpha's path the parties' seeds differ by delta.  Per level
//   CW_i = h'_0 ^ h'_1 ^ (1 - alpha_i) * delta
// makes the off-path children equal and keeps the on-path difference delta;
// a DCF adds VCW_i = v_0 ^ v_1 ^ V_alpha ^ alpha_i, after which V_alpha is
// alpha_i.  The leaf word is L(s_0) ^ L(s_1) xor e_{alpha mod 128} (DPF) or
// xor the 128-bit mask [j < alpha mod 128], flipped when V_alpha = 1 (DCF).
// `wrap` (DCF only) goes to bit 31 of the VCW word.
template <bool DCF>
__device__ __forceinline__ void tree_gen(uint8_t* k, uint64_t np, uint64_t row, uint32_t nbits, uint32_t alpha,
                                         uint4 s, uint4 delta, uint32_t wrap, const uint32_t* tab, LaneOff loff) {
    const uint32_t nu = nbits - 7;
    const DpfPlanes PP{np, nu};
    const DcfPlanes PC{np, nu};
    at_w<uint4>(k, PP.root(), row) = s;
    uint32_t va = 0, vw = 0;
    for (uint32_t i = 0; i < nu; i++) {
        const uint32_t a = (alpha >> (nbits - 1 - i)) & 1u;
        uint32_t v;
        const uint4 h = expand(s, v, tab, loff);
        const uint4 cw = xor4(xor4(h, partner4(h)), and4(delta, a - 1u));   // a - 1: all ones when a = 0
        if (DCF) {
            const uint32_t vcw = v ^ partner(v) ^ va ^ a;
            vw |= vcw << i;
            va = a;                             // V_alpha ^ (v_0 ^ v_1) ^ VCW_i
        }
        s = child(s, h, cw, a);
        at_w<uint4>(k, PP.cw(i), row) = cw;      // the same offset in both layouts
    }
    uint4 u = s;
    u.x ^= 2u;
    const uint4 g = tree_hash(u, tab, loff);
    uint4 cw = xor4(g, partner4(g));
    const uint32_t low = alpha & 127u;
    if (DCF) {
        // [j < low] for j = 0..127 as a 128-bit mask, flipped when V_alpha = 1
        const uint32_t flip = 0u - va;
        const uint32_t m0 = low >= 32 ? ~0u : (1u << low) - 1u;
        const uint32_t m1 = low >= 64 ? ~0u : (low <= 32 ? 0u : (1u << (low - 32)) - 1u);
        const uint32_t m2 = low >= 96 ? ~0u : (low <= 64 ? 0u : (1u << (low - 64)) - 1u);
        const uint32_t m3 = low <= 96 ? 0u : (1u << (low - 96)) - 1u;
        cw = xor4(cw, make_uint4(m0 ^ flip, m1 ^ flip, m2 ^ flip, m3 ^ flip));
        at_w<uint32_t>(k, PC.vcw(), row) = vw | (wrap << 31);
    } else {
        const uint32_t bit = 1u << (low & 31u);
        cw.x ^= (low >> 5) == 0 ? bit : 0u;
        cw.y ^= (low >> 5) == 1 ? bit : 0u;
        cw.z ^= (low >> 5) == 2 ? bit : 0u;
        cw.w ^= (low >> 5) == 3 ? bit : 0u;
    }
    at_w<uint4>(k, DCF ? PC.cwleaf() : PP.cwleaf(), row) = cw;
}

// Roots of one tree: the even lane draws the block of s_0 (generator block
// j), the odd lane that of delta (block j + 1); the partner exchange gives both
// lanes both.  s_0 keeps bit 1 clear, delta has bit 0 set and bit 1 clear,
// and party b's root is s_0 ^ b * delta.
__device__ __forceinline__ void tree_roots(const DealerArgs& A, uint32_t j, uint32_t e, uint32_t b, uint4& s,
                                           uint4& delta, const uint32_t* tab, LaneOff loff) {
    uint4 mine = rng_block(A.rk, 3, j + b, A.query, A.pred, e, tab, loff);
    pin_in_vgprs(mine);
    const uint4 other = partner4(mine);
    uint4 s0 = b ? other : mine;
    delta = b ? mine : other;
    s0.x &= ~2u;
    delta.x = (delta.x & ~2u) | 1u;
    s = b ? xor4(s0, delta) : s0;
}

// Both lanes of row `row`'s pair (b = party of this lane); KIND is the key kind.
template <int KIND>
__device__ __forceinline__ void keygen_row(const DealerArgs& A, uint64_t row, uint32_t b, const uint32_t* tab,
                                           LaneOff loff) {
    const uint64_t np = pad_rows(A.n);
    const uint32_t mask = A.nbits >= 32 ? 0xFFFFFFFFu : ((1u << A.nbits) - 1u);
    const uint32_t r = A.r[row];
    const uint32_t e = (uint32_t)row + A.row_offset;
    uint8_t* key = b ? A.key1 : A.key0;
    uint4 s, delta;
    tree_roots(A, 0, e, b, s, delta, tab, loff);
    if (KIND == FSS_EQ) {
        tree_gen<false>(key, np, row, A.nbits, (A.a_or_lo + r) & mask, s, delta, 0u, tab, loff);
    } else {
        const uint32_t U = (A.hi + r) & mask, L = (A.a_or_lo + r) & mask;
        uint32_t c0 = rng_block(A.rk, 3, 2, A.query, A.pred, e, tab, loff).x & 1u;
        pin_in_vgprs(c0);
        const uint32_t cb = c0 ^ (b & (L > U ? 1u : 0u));
        tree_gen<true>(key, np, row, A.nbits, U, s, delta, cb, tab, loff);
        tree_roots(A, 3, e, b, s, delta, tab, loff);
        tree_gen<true>(key + DcfPlanes{np, A.nbits - 7}.bytes(), np, row, A.nbits, L, s, delta, 0u, tab, loff);
    }
}

// Two lanes per row (see above); 512 rows per workgroup.  One kernel per key
// kind, so each is compiled for its own Gen alone.
template <int KIND>
__device__ __forceinline__ void keygen_grid(const DealerArgs& A) {
    __shared__ uint32_t tab[kLdsTableWords];
    lds_table_fill(tab, g_tables.t0);
    __syncthreads();
    const uint64_t gid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t row = gid >> 1;
    if (row >= A.n) return;                 // both lanes of a pair leave together
    keygen_row<KIND>(A, row, (uint32_t)(gid & 1u), tab, lane_offset());
}

__global__ __launch_bounds__(kBlock) void k_keygen_eq(DealerArgs A) { keygen_grid<FSS_EQ>(A); }
__global__ __launch_bounds__(kBlock) void k_keygen_range(DealerArgs A) { keygen_grid<FSS_RANGE>(A); }

// ----------------------------------------------------------------- persistent work queue (batches)
//
// A batch is a list of descriptors in device memory; descriptor i owns tiles
// [tile_start_i, tile_start_i + tiles_i) of one global tile range.  A grid of
// at most two workgroups per CU pulls tile numbers from one atomic counter
// (zeroed by the launch before) until the range is exhausted, so every
// workgroup leaves once all tiles are taken.  Each tile is a pure function of
// its descriptor and rows: results do not depend on which workgroup took it.

struct QKeygen {
    DealerArgs a;
    uint32_t tile_start;    // tiles of 512 rows
    uint32_t pad;
};

struct QEval {
    EvalDesc d;             // d.block_start = first tile; tiles of kBlock * rows_per_thread rows
};

__global__ void k_zero_counter(uint32_t* c) {
    if (threadIdx.x == 0) *c = 0u;
}

// Last descriptor whose first tile is <= tile (descriptors in tile order).
template <class F>
__device__ __forceinline__ uint32_t find_desc(uint32_t count, uint32_t tile, F start_of) {
    uint32_t lo = 0, hi = count;    // invariant: start_of(lo) <= tile, answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (start_of(mid) <= tile) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t next_tile(uint32_t* counter, uint32_t* s_tile) {
    __syncthreads();                         // everyone is done with the previous tile number
    if (threadIdx.x == 0) *s_tile = atomicAdd(counter, 1u);
    __syncthreads();
    return *s_tile;
}

// One key kind per launch (the host splits a batch by kind), so each kernel
// holds one Gen's registers.
template <int KIND>
__device__ __forceinline__ void keygen_queue(const QKeygen* __restrict__ q, uint32_t count, uint32_t total_tiles,
                                             uint32_t* counter) {
    __shared__ uint32_t tab[kLdsTableWords];
    __shared__ uint32_t s_tile;
    lds_table_fill(tab, g_tables.t0);
    const LaneOff loff = lane_offset();
    for (;;) {
        const uint32_t tile = next_tile(counter, &s_tile);   // also orders the table fill
        if (tile >= total_tiles) break;
        const uint32_t di = find_desc(count, tile, [&](uint32_t i) { return q[i].tile_start; });
        const DealerArgs& A = q[di].a;
        const uint64_t row = (uint64_t)(tile - q[di].tile_start) * (kBlock / 2) + (threadIdx.x >> 1);
        if (row < A.n) keygen_row<KIND>(A, row, threadIdx.x & 1u, tab, loff);
    }
}

__global__ __launch_bounds__(kBlock, 8) void k_keygen_queue_eq(const QKeygen* __restrict__ q, uint32_t count,
                                                           uint32_t total_tiles, uint32_t* counter) {
    keygen_queue<FSS_EQ>(q, count, total_tiles, counter);
}

__global__ __launch_bounds__(kBlock, 8) void k_keygen_queue_range(const QKeygen* __restrict__ q, uint32_t count,
                                                              uint32_t total_tiles, uint32_t* counter) {
    keygen_queue<FSS_RANGE>(q, count, total_tiles, counter);
}

__global__ __launch_bounds__(kBlock, 8) void k_eval_queue(const QEval* __restrict__ q, uint32_t count,
                                                      uint32_t total_tiles, uint32_t rows_per_thread,
                                                      uint32_t* counter) {
    __shared__ uint32_t tab[kLdsTableWords];
    __shared__ uint32_t s_tile;
    lds_table_fill(tab, g_tables.t0);
    const LaneOff loff = lane_offset();
    for (;;) {
        const uint32_t tile = next_tile(counter, &s_tile);
        if (tile >= total_tiles) break;
        const uint32_t di = find_desc(count, tile, [&](uint32_t i) { return q[i].d.block_start; });
        const EvalDesc& D = q[di].d;
        const uint64_t row0 = (uint64_t)(tile - D.block_start) * kBlock * rows_per_thread;
        for (uint32_t k = 0; k < rows_per_thread; k++) eval_rows(D, row0 + (uint64_t)k * kBlock, tab, loff);
    }
}

struct MaskArgs {
    RoundKeys rk;
    uint32_t* r;
    uint64_t n;
    uint32_t query;
    uint32_t pred;
    uint32_t row_offset;
};

// r[i] = word 0 of the counter-mode block (2, 0, query, pred, row_offset + i).
__global__ __launch_bounds__(kBlock) void k_masks(MaskArgs A) {
    __shared__ uint32_t tab[kLdsTableWords];
    lds_table_fill(tab, g_tables.t0);
    __syncthreads();
    const LaneOff loff = lane_offset();
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < A.n; i += stride)
        A.r[i] = rng_block(A.rk, 2, 0, A.query, A.pred, A.row_offset + (uint32_t)i, tab, loff).x;
}

struct TripleArgs {
    RoundKeys rk;
    uint32_t* t0;           // a0 | b0 | c0
    uint32_t* t1;           // a1 | b1 | c1
    uint64_t nwords;
    uint32_t query;
    uint32_t and_id;
};

// Work item m makes triple words 4m .. 4m+3 from stream blocks 5m .. 5m+4.
__global__ __launch_bounds__(kBlock) void k_triples(TripleArgs A) {
    __shared__ uint32_t tab[kLdsTableWords];
    lds_table_fill(tab, g_tables.t0);
    __syncthreads();
    const LaneOff loff = lane_offset();
    const uint64_t groups = (A.nwords + 3) / 4;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t m = (uint64_t)blockIdx.x * kBlock + threadIdx.x; m < groups; m += stride) {
        uint32_t R[20];
#pragma unroll
        for (int q = 0; q < 5; q++) {
            uint4 b = rng_block(A.rk, 4, 0, A.query, A.and_id, (uint32_t)(5 * m + q), tab, loff);
            pin_in_vgprs(b);        // one block at a time
            R[4 * q + 0] = b.x; R[4 * q + 1] = b.y; R[4 * q + 2] = b.z; R[4 * q + 3] = b.w;
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const uint64_t w = 4 * m + q;
            if (w < A.nwords) {
                const uint32_t a0 = R[5 * q], a1 = R[5 * q + 1], b0 = R[5 * q + 2], b1 = R[5 * q + 3];
                const uint32_t c0 = R[5 * q + 4];
                A.t0[w] = a0; A.t0[A.nwords + w] = b0; A.t0[2 * A.nwords + w] = c0;
                A.t1[w] = a1; A.t1[A.nwords + w] = b1; A.t1[2 * A.nwords + w] = ((a0 ^ a1) & (b0 ^ b1)) ^ c0;
            }
        }
    }
}

// ----------------------------------------------------------------- one-hot RSS secEval (Eq. predEval)

// Full-domain evaluation: key row `row` of a batch (party `party`) at every
// point x in [0, npoints); each wave packs its 64 bits.
__global__ __launch_bounds__(kBlock) void k_eval_points(const uint8_t* key, uint64_t n, uint64_t row, uint32_t kind,
                                                       uint32_t nbits, uint32_t party, uint64_t npoints,
                                                       uint32_t* out) {
    __shared__ uint32_t tab[kLdsTableWords];
    lds_table_fill(tab, g_tables.t0);
    __syncthreads();
    const uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const LaneOff loff = lane_offset();
    const uint64_t np = pad_rows(n);
    uint32_t bit = 0;
    if (x < npoints) {
        if (kind == FSS_EQ)
            bit = dpf_eval(key, np, row, nbits, (uint32_t)x, tab, loff);
        else
            bit = range_eval(key, np, row, nbits, (uint32_t)x, tab, loff);
    }
    const uint64_t ballot = __ballot(bit);
    if ((threadIdx.x & 63u) == 0) {
        const uint64_t w = x >> 5, nwords = (npoints + 31) >> 5;
        if (w < nwords) out[w] = (uint32_t)ballot;
        if (w + 1 < nwords) out[w + 1] = (uint32_t)(ballot >> 32);
    }
}

// Several full-domain evaluations in one launch (blockIdx.y = request): the
// six keys of one secEval predicate (two per server) are small and
// latency-bound, so they run side by side instead of one after another.
constexpr int kEvalAllMax = 8;

struct EvalAllReq {
    const uint8_t* key;         // this party's key batch
    uint32_t* out;
    uint64_t n;                 // rows of the batch
    uint64_t row;               // key row evaluated
    uint64_t npoints;
    uint32_t kind;
    uint32_t nbits;
    uint32_t party;
    uint32_t pad;
};

struct EvalAllBatch {
    EvalAllReq r[kEvalAllMax];
};

__global__ __launch_bounds__(kBlock) void k_eval_points_batch(EvalAllBatch B) {
    const EvalAllReq& R = B.r[blockIdx.y];
    if ((uint64_t)blockIdx.x * kBlock >= R.npoints) return;     // the whole block leaves
    __shared__ uint32_t tab[kLdsTableWords];
    lds_table_fill(tab, g_tables.t0);
    __syncthreads();
    const uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const LaneOff loff = lane_offset();
    const uint64_t np = pad_rows(R.n);
    uint32_t bit = 0;
    if (x < R.npoints) {
        if (R.kind == FSS_EQ)
            bit = dpf_eval(R.key, np, R.row, R.nbits, (uint32_t)x, tab, loff);
        else
            bit = range_eval(R.key, np, R.row, R.nbits, (uint32_t)x, tab, loff);
    }
    const uint64_t ballot = __ballot(bit);
    if ((threadIdx.x & 63u) == 0) {
        const uint64_t w = x >> 5, nwords = (R.npoints + 31) >> 5;
        if (w < nwords) R.out[w] = (uint32_t)ballot;
        if (w + 1 < nwords) R.out[w + 1] = (uint32_t)(ballot >> 32);
    }
}

// One server's share of the predicate bit of every candidate: the XOR over
// positions of Eval(k_a, l) & <e[l]>_a, XORed with the same for (k_b, share b).
// Shares are word-major ([word][candidate]): a wave reads 256 contiguous bytes
// per word; the evaluation words are uniform (scalar loads).
__global__ void k_rss_eval(uint64_t ncand, uint32_t nwords_pos, const uint32_t* __restrict__ eval_a,
                           const uint32_t* __restrict__ eval_b, const uint32_t* __restrict__ share_a,
                           const uint32_t* __restrict__ share_b, uint32_t* __restrict__ out) {
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    if (c < ncand) {
#pragma unroll 8
        for (uint32_t w = 0; w < nwords_pos; w++) {      // unrolled: 16 loads in flight per thread
            const uint64_t at = (uint64_t)w * ncand + c;
            acc = __builtin_amdgcn_bitop3_b32(acc, share_a[at], eval_a[w], 0x78);   // acc ^ (s & e): f(0xF0, 0xCC, 0xAA)
            acc = __builtin_amdgcn_bitop3_b32(acc, share_b[at], eval_b[w], 0x78);
        }
    }
    const uint64_t ballot = __ballot(__builtin_popcount(acc) & 1u);
    if ((threadIdx.x & 63u) == 0) {
        const uint64_t w = c >> 5, nw = (ncand + 31) >> 5;
        if (w < nw) out[w] = (uint32_t)ballot;
        if (w + 1 < nw) out[w + 1] = (uint32_t)(ballot >> 32);
    }
}

// ----------------------------------------------------------------- streaming kernels (open, ANDs, joins)

// xhat = x0 + x1 + r mod 2^32.  With vec (all four buffers 16-byte aligned) a
// thread takes four rows per 16-byte load and store, the last n mod 4 rows
// one by one.
__global__ void k_mask_open(uint64_t n, uint32_t vec, const uint32_t* __restrict__ x0,
                            const uint32_t* __restrict__ x1, const uint32_t* __restrict__ r,
                            uint32_t* __restrict__ xhat) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t done = 0;
    if (vec) {
        const uint64_t n4 = n >> 2;
        for (uint64_t i = t; i < n4; i += stride) {
            const uint4 a = ((const uint4*)x0)[i], b = ((const uint4*)x1)[i], c = ((const uint4*)r)[i];
            ((uint4*)xhat)[i] = make_uint4(a.x + b.x + c.x, a.y + b.y + c.y, a.z + b.z + c.z, a.w + b.w + c.w);
        }
        done = n4 << 2;
    }
    for (uint64_t i = done + t; i < n; i += stride) xhat[i] = x0[i] + x1[i] + r[i];
}

__device__ __forceinline__ uint32_t pad_mask(uint64_t w, uint64_t nrows) {
    const uint64_t first = w * 32;
    if (first + 32 <= nrows) return 0xFFFFFFFFu;
    if (first >= nrows) return 0u;
    return (1u << (uint32_t)(nrows - first)) - 1u;
}

__global__ void k_and_open(uint64_t nwords, const uint32_t* __restrict__ x, const uint32_t* __restrict__ y,
                           const uint32_t* __restrict__ trip, uint32_t* __restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += stride) {
        out[w] = x[w] ^ trip[w];
        out[nwords + w] = y[w] ^ trip[nwords + w];
    }
}

__global__ void k_and_close(uint64_t nwords, uint64_t nrows, uint32_t party, const uint32_t* __restrict__ trip,
                            const uint32_t* __restrict__ de, uint32_t* __restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += stride) {
        const uint32_t d = de[w], e = de[nwords + w];
        uint32_t z = trip[2 * nwords + w] ^ (d & trip[nwords + w]) ^ (e & trip[w]);
        if (party == 0) z ^= d & e;
        out[w] = z & pad_mask(w, nrows);
    }
}

// Both simulated parties at once: open, exchange (an XOR), close.
__global__ void k_and_both(uint64_t nwords, uint64_t nrows, const uint32_t* __restrict__ x0,
                           const uint32_t* __restrict__ x1, const uint32_t* __restrict__ y0,
                           const uint32_t* __restrict__ y1, const uint32_t* __restrict__ t0,
                           const uint32_t* __restrict__ t1, uint32_t* __restrict__ z0, uint32_t* __restrict__ z1) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += stride) {
        const uint32_t a0 = t0[w], b0 = t0[nwords + w], c0 = t0[2 * nwords + w];
        const uint32_t a1 = t1[w], b1 = t1[nwords + w], c1 = t1[2 * nwords + w];
        const uint32_t d = (x0[w] ^ a0) ^ (x1[w] ^ a1);
        const uint32_t e = (y0[w] ^ b0) ^ (y1[w] ^ b1);
        const uint32_t pm = pad_mask(w, nrows);
        z0[w] = (c0 ^ (d & b0) ^ (e & a0) ^ (d & e)) & pm;
        z1[w] = (c1 ^ (d & b1) ^ (e & a1)) & pm;
    }
}

// out_b[e] = bit idx[e] of m_b (each party gathers its own share at a public
// index); an index >= nsrc gathers 0 for both parties.
// The two parties' shares of one vertex bit array side by side: word w of
// party b at pair[w] component b, so that a gather reads both in one 8-byte
// load (one L2 request per edge instead of two).
__global__ void k_interleave(uint64_t nwords, const uint32_t* __restrict__ m0, const uint32_t* __restrict__ m1,
                             uint2* __restrict__ pair) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += stride)
        pair[w] = make_uint2(m0[w], m1[w]);
}

// Edge e of the join takes the endpoint's bit from both parties' arrays: bit
// idx[e] of the interleaved vertex bits, packed by ballot into o0 / o1.
__global__ void k_gather(uint64_t n, uint64_t nsrc, const uint32_t* __restrict__ idx,
                         const uint2* __restrict__ pair, uint32_t* __restrict__ o0, uint32_t* __restrict__ o1) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t b0 = 0, b1 = 0;
    if (e < n && idx[e] < nsrc) {
        const uint32_t v = idx[e];
        const uint2 w = pair[v >> 5];
        b0 = (w.x >> (v & 31u)) & 1u;
        b1 = (w.y >> (v & 31u)) & 1u;
    }
    const uint64_t g0 = __ballot(b0), g1 = __ballot(b1);
    if ((threadIdx.x & 63u) == 0) {
        const uint64_t w = e >> 5, nwords = (n + 31) >> 5;
        if (w < nwords) { o0[w] = (uint32_t)g0; o1[w] = (uint32_t)g1; }
        if (w + 1 < nwords) { o0[w + 1] = (uint32_t)(g0 >> 32); o1[w + 1] = (uint32_t)(g1 >> 32); }
    }
}

// ----------------------------------------------------------------- three-party RSS arithmetic

struct RssArgs {
    ChachaKey prf[3];       // F(k_i, .) = ChaCha12 under (k_i, domain 5)
    const uint32_t* x[3];
    const uint32_t* y[3];   // null for a plain re-share
    uint32_t* z[3];
    uint64_t nrows;
    uint64_t nwords;
    uint32_t counter;
    uint32_t vec;           // every share buffer 16-byte aligned: 16-byte loads / stores
};

constexpr int kRssBlock = 256;

// Thread m owns words 4m .. 4m+3, lane m & 3 of the quad that makes PRF block
// m div 4 (words 16 (m div 4) .. + 15).  For the AND, party P_i first forms
// z_i = x_i y_i ^ x_i y_{i+1} ^ x_{i+1} y_i from the two shares it holds; then
// z_i ^= F(k_i, j) ^ F(k_{i-1}, j) (a fresh sharing of zero), pad bits cleared.
// Every lane of a launched quad makes the PRF blocks; only the loads and
// stores are bounded by the share length.
__global__ __launch_bounds__(kRssBlock) void k_rss(RssArgs A) {
    const uint64_t m = (uint64_t)blockIdx.x * kRssBlock + threadIdx.x;
    const bool any = 4 * m < A.nwords;
    const bool whole = A.vec && 4 * m + 4 <= A.nwords;
    // the shares are loaded before the PRF, so that their latency overlaps it
    uint4 xv[3], yv[3];
    if (whole) {
#pragma unroll
        for (int i = 0; i < 3; i++) {
            xv[i] = ((const uint4*)A.x[i])[m];
            yv[i] = A.y[0] ? ((const uint4*)A.y[i])[m] : make_uint4(0u, 0u, 0u, 0u);
        }
    }
    uint4 f[3];
#pragma unroll
    for (int i = 0; i < 3; i++) f[i] = chacha_quad(A.prf[i], (uint32_t)(m >> 2), A.counter, 0u, 0u);
    if (!any) return;
    if (whole) {
        // four whole words: 16-byte loads and stores
        const uint32_t pm[4] = {pad_mask(4 * m, A.nrows), pad_mask(4 * m + 1, A.nrows), pad_mask(4 * m + 2, A.nrows),
                                pad_mask(4 * m + 3, A.nrows)};
        uint4 z[3];
#pragma unroll
        for (int i = 0; i < 3; i++) {
            const int nx = (i + 1) % 3, pv = (i + 2) % 3;
            const uint4 xi = xv[i], xn = xv[nx], yi = yv[i], yn = yv[nx];
            z[i] = xi;
            if (A.y[0])
                z[i] = make_uint4((xi.x & yi.x) ^ (xi.x & yn.x) ^ (xn.x & yi.x),
                                  (xi.y & yi.y) ^ (xi.y & yn.y) ^ (xn.y & yi.y),
                                  (xi.z & yi.z) ^ (xi.z & yn.z) ^ (xn.z & yi.z),
                                  (xi.w & yi.w) ^ (xi.w & yn.w) ^ (xn.w & yi.w));
            z[i] = xor4(xor4(z[i], f[i]), f[pv]);
        }
#pragma unroll
        for (int i = 0; i < 3; i++)
            ((uint4*)A.z[i])[m] = make_uint4(z[i].x & pm[0], z[i].y & pm[1], z[i].z & pm[2], z[i].w & pm[3]);
        return;
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint64_t w = 4 * m + q;
        if (w >= A.nwords) break;
        const uint32_t pm = pad_mask(w, A.nrows);
#pragma unroll
        for (int i = 0; i < 3; i++) {
            const int nx = (i + 1) % 3, pv = (i + 2) % 3;
            uint32_t zi;
            if (A.y[0]) {
                const uint32_t xi = A.x[i][w], xn = A.x[nx][w], yi = A.y[i][w], yn = A.y[nx][w];
                zi = (xi & yi) ^ (xi & yn) ^ (xn & yi);
            } else {
                zi = A.x[i][w];
            }
            const uint32_t fi = q == 0 ? f[i].x : q == 1 ? f[i].y : q == 2 ? f[i].z : f[i].w;
            const uint32_t fp = q == 0 ? f[pv].x : q == 1 ? f[pv].y : q == 2 ? f[pv].z : f[pv].w;
            A.z[i][w] = (zi ^ fi ^ fp) & pm;
        }
    }
}

// Shares of the public constant 1 over nrows rows.
__global__ void k_public_one(uint64_t nwords, uint64_t nrows, uint32_t* __restrict__ o0, uint32_t* __restrict__ o1) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += stride) {
        o0[w] = pad_mask(w, nrows);
        o1[w] = 0u;
    }
}

// ----------------------------------------------------------------- host side

using ogm::fail;
using ogm::check_launch;

bool valid_nbits(uint32_t nbits) { return nbits >= 8 && nbits <= 32; }

uint64_t key_bytes(int32_t kind, uint32_t nbits) {
    if (!valid_nbits(nbits)) return 0;
    const uint64_t tree = 16ull * (nbits - 5);     // root, nbits - 7 correction words, leaf word
    if (kind == FSS_EQ) return tree;
    if (kind == FSS_RANGE) return 2 * (tree + 4);  // two DCFs, each with its VCW word
    return 0;
}

int staging_release();      // the batch calls' staging ring (defined with it below)

bool aligned256(const void* p) { return ((uintptr_t)p & 255u) == 0; }
bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

// Workgroups of a grid-stride AES kernel over `items` work items: two per CU
// at most (what the LDS holds), so each fills its 64 KiB tables once and then
// loops over many items.
unsigned aes_grid(uint64_t items) {
    const uint64_t need = (items + kBlock - 1) / kBlock;
    const uint64_t cap = 2ull * (uint64_t)device_cus();
    return (unsigned)(need < 1 ? 1 : (need < cap ? need : cap));
}

unsigned grid_for(uint64_t n, unsigned block, unsigned cap) {
    uint64_t g = (n + block - 1) / block;
    if (g == 0) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

RoundKeys dealer_key(uint64_t seed) { return ogm::seed_key(seed); }

int check_batch(const fss_keybatch* k, int32_t want_kind, const char* who) {
    if (!k) return fail(FSS_EINVAL, "%s: key batch is NULL", who);
    if (k->kind != want_kind) return fail(FSS_EINVAL, "%s: key batch kind %d, expected %d", who, k->kind, want_kind);
    if (!valid_nbits(k->nbits)) return fail(FSS_EINVAL, "%s: nbits %u outside 8..32", who, k->nbits);
    if (k->n > 0xFFFFFFFFull) return fail(FSS_EUNSUPPORTED, "%s: more than 2^32 rows", who);
    return FSS_OK;
}

// Enqueue one k_eval launch for up to kEvalInline descriptors (heaviest first).
int launch_eval(EvalDesc* descs, uint32_t count, hipStream_t stream) {
    // range walks cost ~2.5x an equality walk: put them first so the tail is light
    EvalBatch b{};
    uint32_t k = 0;
    for (int pass = 0; pass < 2; pass++)
        for (uint32_t i = 0; i < count; i++)
            if ((pass == 0) == (descs[i].kind == FSS_RANGE) && descs[i].n > 0) b.d[k++] = descs[i];
    b.count = k;
    uint32_t blocks = 0;
    for (uint32_t i = 0; i < k; i++) {
        b.d[i].block_start = blocks;
        blocks += (uint32_t)((b.d[i].n + kBlock - 1) / kBlock);
    }
    b.total_blocks = blocks;
    if (blocks == 0) return FSS_OK;
    hipLaunchKernelGGL(k_eval, dim3(blocks), dim3(kBlock), 0, stream, b);
    return check_launch("k_eval");
}

int eval_one(int32_t party, const fss_keybatch* k, int32_t kind, const uint32_t* d_xhat, uint32_t* d_out,
             void* stream, const char* who) {
    int rc = check_batch(k, kind, who);
    if (rc) return rc;
    if (party != 0 && party != 1) return fail(FSS_EINVAL, "%s: party %d is not 0 or 1", who, party);
    if (k->n == 0) return FSS_OK;
    if (!d_xhat || !d_out || !k->key[party]) return fail(FSS_EINVAL, "%s: NULL buffer", who);
    if (!aligned256(k->key[party])) return fail(FSS_EINVAL, "%s: key buffer not 256-byte aligned", who);
    EvalDesc d{};
    d.key = (const uint8_t*)k->key[party];
    d.xhat = d_xhat;
    d.out = d_out;
    d.n = k->n;
    d.kind = (uint32_t)kind;
    d.nbits = k->nbits;
    d.party = (uint32_t)party;
    return launch_eval(&d, 1, (hipStream_t)stream);
}

int launch_triples(uint64_t seed, uint32_t query_id, uint32_t and_id, uint64_t nwords, uint32_t* t0, uint32_t* t1,
                   hipStream_t stream) {
    if (nwords == 0) return FSS_OK;
    TripleArgs A{};
    A.rk = dealer_key(seed);
    A.t0 = t0;
    A.t1 = t1;
    A.nwords = nwords;
    A.query = query_id;
    A.and_id = and_id;
    hipLaunchKernelGGL(k_triples, dim3(aes_grid((nwords + 3) / 4)), dim3(kBlock), 0, stream, A);
    return check_launch("k_triples");
}

}  // namespace

// ================================================================= C ABI

extern "C" {

uint64_t fss_key_bytes(int32_t kind, uint32_t nbits) { return key_bytes(kind, nbits); }

uint64_t fss_keybatch_bytes(int32_t kind, uint32_t nbits, uint64_t n) { return key_bytes(kind, nbits) * pad_rows(n); }

const char* fss_last_error(void) { return ogm::last_error().c_str(); }

const char* fss_version(void) { return "oblivgm-fss 0.1 gfx950 lds-ttable"; }

int fss_shutdown(void) {
    ogm::last_error().clear();
    const int rc = staging_release();
    const int rc_streams = ogm::shuffle_release();
    if (rc) return fail(rc, "fss_shutdown: a staging buffer could not be released");
    if (rc_streams) return fail(rc_streams, "fss_shutdown: a shuffle stream could not be released");
    return FSS_OK;
}

int fss_mask_open(uint64_t n, const uint32_t* d_x0, const uint32_t* d_x1, const uint32_t* d_r, uint32_t* d_xhat,
                  void* stream) {
    ogm::last_error().clear();
    if (n == 0) return FSS_OK;
    if (!d_x0 || !d_x1 || !d_r || !d_xhat) return fail(FSS_EINVAL, "fss_mask_open: NULL buffer");
    const bool vec = aligned16(d_x0) && aligned16(d_x1) && aligned16(d_r) && aligned16(d_xhat);
    hipLaunchKernelGGL(k_mask_open, dim3(grid_for(vec ? (n + 3) / 4 : n, 256, 8192)), dim3(256), 0, (hipStream_t)stream,
                       n, (uint32_t)vec, d_x0, d_x1, d_r, d_xhat);
    return check_launch("k_mask_open");
}

int fss_keygen(uint64_t seed, uint32_t query_id, uint32_t pred_id, uint32_t a_or_lo, uint32_t hi,
               const uint32_t* d_r, const fss_keybatch* out, void* stream) {
    ogm::last_error().clear();
    if (!out) return fail(FSS_EINVAL, "fss_keygen: out is NULL");
    if (out->kind != FSS_EQ && out->kind != FSS_RANGE) return fail(FSS_EINVAL, "fss_keygen: bad kind %d", out->kind);
    if (!valid_nbits(out->nbits)) return fail(FSS_EINVAL, "fss_keygen: nbits %u outside 8..32", out->nbits);
    if (out->n > 0xFFFFFFFFull) return fail(FSS_EUNSUPPORTED, "fss_keygen: more than 2^32 rows");
    const uint64_t lim = 1ull << out->nbits;
    if (out->kind == FSS_EQ && a_or_lo >= lim) return fail(FSS_EINVAL, "fss_keygen: a does not fit nbits");
    if (out->kind == FSS_RANGE) {
        if (a_or_lo > hi) return fail(FSS_EINVAL, "fss_keygen: lo %u > hi %u", a_or_lo, hi);
        if (hi >= lim) return fail(FSS_EINVAL, "fss_keygen: hi does not fit nbits (full domain not expressible)");
    }
    if (out->n == 0) return FSS_OK;
    if (!d_r || !out->key[0] || !out->key[1]) return fail(FSS_EINVAL, "fss_keygen: NULL buffer");
    if (!aligned256(out->key[0]) || !aligned256(out->key[1]))
        return fail(FSS_EINVAL, "fss_keygen: key buffers must be 256-byte aligned");
    DealerArgs A{};
    A.rk = dealer_key(seed);
    A.key0 = (uint8_t*)out->key[0];
    A.key1 = (uint8_t*)out->key[1];
    A.r = d_r;
    A.n = out->n;
    A.kind = (uint32_t)out->kind;
    A.nbits = out->nbits;
    A.query = query_id;
    A.pred = pred_id;
    A.a_or_lo = a_or_lo;
    A.hi = hi;
    const dim3 grid((unsigned)((2 * out->n + kBlock - 1) / kBlock));
    if (out->kind == FSS_EQ)
        hipLaunchKernelGGL(k_keygen_eq, grid, dim3(kBlock), 0, (hipStream_t)stream, A);
    else
        hipLaunchKernelGGL(k_keygen_range, grid, dim3(kBlock), 0, (hipStream_t)stream, A);
    return check_launch("k_keygen");
}

int fss_dealer_masks(uint64_t seed, uint32_t query_id, uint32_t pred_id, uint32_t row_offset, uint64_t n,
                     uint32_t* d_r, void* stream) {
    ogm::last_error().clear();
    if (n == 0) return FSS_OK;
    if (!d_r) return fail(FSS_EINVAL, "fss_dealer_masks: NULL buffer");
    if ((uint64_t)row_offset + n > (1ull << 32)) return fail(FSS_EUNSUPPORTED, "fss_dealer_masks: rows beyond 2^32");
    MaskArgs A{};
    A.rk = dealer_key(seed);
    A.r = d_r;
    A.n = n;
    A.query = query_id;
    A.pred = pred_id;
    A.row_offset = row_offset;
    hipLaunchKernelGGL(k_masks, dim3(aes_grid(n)), dim3(kBlock), 0, (hipStream_t)stream, A);
    return check_launch("k_masks");
}

int fss_eval_eq(int32_t party, const fss_keybatch* k, const uint32_t* d_xhat, uint32_t* d_out_bits, void* stream) {
    ogm::last_error().clear();
    return eval_one(party, k, FSS_EQ, d_xhat, d_out_bits, stream, "fss_eval_eq");
}

int fss_eval_lt(int32_t party, const fss_keybatch* k, const uint32_t* d_xhat, uint32_t* d_out_bits, void* stream) {
    ogm::last_error().clear();
    return eval_one(party, k, FSS_RANGE, d_xhat, d_out_bits, stream, "fss_eval_lt");
}

int ss_triples(uint64_t seed, uint32_t query_id, uint32_t and_id, uint64_t nwords, uint32_t* d_trip0,
               uint32_t* d_trip1, void* stream) {
    ogm::last_error().clear();
    if (nwords == 0) return FSS_OK;
    if (!d_trip0 || !d_trip1) return fail(FSS_EINVAL, "ss_triples: NULL buffer");
    // four triple words take five generator blocks, counted in 32 bits
    if ((nwords + 3) / 4 * 5 > (1ull << 32)) return fail(FSS_EUNSUPPORTED, "ss_triples: too many words");
    return launch_triples(seed, query_id, and_id, nwords, d_trip0, d_trip1, (hipStream_t)stream);
}

int ss_and(int32_t phase, int32_t party, uint64_t nrows, const uint32_t* d_x, const uint32_t* d_y,
           const uint32_t* d_triple, const uint32_t* d_de_open, uint32_t* d_out, void* stream) {
    ogm::last_error().clear();
    if (party != 0 && party != 1) return fail(FSS_EINVAL, "ss_and: party %d is not 0 or 1", party);
    const uint64_t nwords = (nrows + 31) / 32;
    if (nwords == 0) return FSS_OK;
    if (!d_triple || !d_out) return fail(FSS_EINVAL, "ss_and: NULL buffer");
    const unsigned grid = grid_for(nwords, 256, 8192);
    if (phase == SS_AND_OPEN) {
        if (!d_x || !d_y) return fail(FSS_EINVAL, "ss_and: NULL input");
        hipLaunchKernelGGL(k_and_open, dim3(grid), dim3(256), 0, (hipStream_t)stream, nwords, d_x, d_y, d_triple,
                           d_out);
        return check_launch("k_and_open");
    }
    if (phase == SS_AND_CLOSE) {
        if (!d_de_open) return fail(FSS_EINVAL, "ss_and: NULL opened values");
        hipLaunchKernelGGL(k_and_close, dim3(grid), dim3(256), 0, (hipStream_t)stream, nwords, nrows,
                           (uint32_t)party, d_triple, d_de_open, d_out);
        return check_launch("k_and_close");
    }
    return fail(FSS_EINVAL, "ss_and: phase %d is neither OPEN nor CLOSE", phase);
}

}  // extern "C"

// ----------------------------------------------------------------- match_query

namespace {

struct Shares {
    uint32_t* p[2] = {nullptr, nullptr};   // both null: the public constant 1
    bool is_public() const { return p[0] == nullptr; }
};

struct Arena {
    uint8_t* base;
    uint64_t size;
    uint64_t used;
    uint32_t* take(uint64_t words) {
        uint64_t bytes = (words * 4 + 255) & ~255ull;
        if (used + bytes > size) return nullptr;
        uint32_t* p = (uint32_t*)(base + used);
        used += bytes;
        return p;
    }
};

uint64_t words_of(uint64_t rows) { return (rows + 31) / 32; }

// Workspace bytes the plan needs (an upper bound): predicate bits and at most
// one AND result per predicate, per hop two gathers and two AND results, and
// one triple buffer -- per party.
uint64_t plan_workspace(const match_plan* P) {
    auto rnd = [](uint64_t words) { return (words * 4 + 255) & ~255ull; };
    const uint64_t wv = words_of(P->n_vertices), we = words_of(P->n_edges);
    uint64_t total = 0;
    for (uint32_t k = 0; k < P->n_pred; k++)
        total += 4 * rnd((uint32_t)P->preds[k].target < P->n_qv ? wv : we);
    if (P->n_qv > 1) total += 8 * (uint64_t)(P->n_qv - 1) * rnd(we) + rnd(2 * wv);   // + the interleaved vertex bits
    const uint64_t wmax = wv > we ? wv : we;
    total += 2 * rnd(3 * wmax);
    return total;
}

__global__ void k_copy_words(uint64_t nwords, const uint32_t* __restrict__ a0, const uint32_t* __restrict__ a1,
                             uint32_t* __restrict__ o0, uint32_t* __restrict__ o1) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += stride) {
        o0[w] = a0[w];
        o1[w] = a1[w];
    }
}

int validate_plan(const match_plan* P, const char* who) {
    if (!P) return fail(FSS_EINVAL, "%s: plan is NULL", who);
    if (P->n_qv == 0 || P->n_qv > FSS_MAX_QV) return fail(FSS_EINVAL, "%s: n_qv %u outside 1..%d", who, P->n_qv, FSS_MAX_QV);
    if (P->n_pred > FSS_MAX_PREDS) return fail(FSS_EINVAL, "%s: more than %d predicates", who, FSS_MAX_PREDS);
    if (P->n_pred && !P->preds) return fail(FSS_EINVAL, "%s: preds is NULL", who);
    if (P->n_vertices > 0xFFFFFFFFull || P->n_edges > 0xFFFFFFFFull)
        return fail(FSS_EUNSUPPORTED, "%s: more than 2^32 rows", who);
    if (!P->d_out[0] || !P->d_out[1]) return fail(FSS_EINVAL, "%s: NULL output", who);
    if (P->n_qv > 1 && P->n_edges && (!P->d_src || !P->d_dst)) return fail(FSS_EINVAL, "%s: NULL edge endpoints", who);
    const uint32_t ntarget = 2 * P->n_qv - 1;
    for (uint32_t k = 0; k < P->n_pred; k++) {
        const fss_pred& p = P->preds[k];
        if (p.target < 0 || (uint32_t)p.target >= ntarget)
            return fail(FSS_EINVAL, "%s: predicate %u targets %d (of %u)", who, k, p.target, ntarget);
        const uint64_t rows = (uint32_t)p.target < P->n_qv ? P->n_vertices : P->n_edges;
        if (p.d_bits[0] || p.d_bits[1]) {
            if (!p.d_bits[0] || !p.d_bits[1]) return fail(FSS_EINVAL, "%s: predicate %u has one bit pointer", who, k);
            continue;   // share bits already evaluated: keys and d_xhat are not used
        }
        if (!p.keys || (p.keys->kind != FSS_EQ && p.keys->kind != FSS_RANGE))
            return fail(FSS_EINVAL, "%s: predicate %u has no valid key batch", who, k);
        int rc = check_batch(p.keys, p.keys->kind, who);
        if (rc) return rc;
        if (p.keys->n != rows)
            return fail(FSS_EINVAL, "%s: predicate %u keys cover %llu rows, table has %llu", who, k,
                        (unsigned long long)p.keys->n, (unsigned long long)rows);
        if (rows && (!p.d_xhat || !p.keys->key[0] || !p.keys->key[1]))
            return fail(FSS_EINVAL, "%s: predicate %u has a NULL buffer", who, k);
        if (rows && (!aligned256(p.keys->key[0]) || !aligned256(p.keys->key[1])))
            return fail(FSS_EINVAL, "%s: predicate %u key buffers not 256-byte aligned", who, k);
    }
    const uint64_t need = plan_workspace(P);
    if (!P->d_workspace || P->workspace_bytes < need)
        return fail(FSS_ENOMEM, "%s: workspace needs %llu bytes", who, (unsigned long long)need);
    return FSS_OK;
}

struct PlanRun {
    const match_plan* P;
    hipStream_t s;
    Arena ws;
    uint32_t next_and = 0;
    uint32_t* trip[2] = {nullptr, nullptr};
    uint2* pair = nullptr;      // interleaved vertex bits of the join, reused by every gather
    Shares pbits[FSS_MAX_PREDS];

    // Carve the triple buffers and the predicate-bit buffers; append one eval
    // descriptor per (predicate, party) with rows to `out`.
    int setup(std::vector<EvalDesc>& out) {
        const uint64_t wv = words_of(P->n_vertices), we = words_of(P->n_edges);
        const uint64_t wmax = wv > we ? wv : we;
        for (int b = 0; b < 2; b++)
            if (!(trip[b] = ws.take(3 * wmax))) return fail(FSS_ENOMEM, "match_query: workspace too small");
        for (uint32_t k = 0; k < P->n_pred; k++) {
            const fss_pred& p = P->preds[k];
            const uint64_t rows = (uint32_t)p.target < P->n_qv ? P->n_vertices : P->n_edges;
            if (p.d_bits[0]) {       // evaluated by the caller
                pbits[k].p[0] = const_cast<uint32_t*>(p.d_bits[0]);
                pbits[k].p[1] = const_cast<uint32_t*>(p.d_bits[1]);
                continue;
            }
            for (int b = 0; b < 2; b++) {
                if (!(pbits[k].p[b] = ws.take(words_of(rows))))
                    return fail(FSS_ENOMEM, "match_query: workspace too small");
                if (rows == 0) continue;
                EvalDesc d{};
                d.key = (const uint8_t*)p.keys->key[b];
                d.xhat = p.d_xhat;
                d.out = pbits[k].p[b];
                d.n = rows;
                d.kind = (uint32_t)p.keys->kind;
                d.nbits = p.keys->nbits;
                d.party = (uint32_t)b;
                out.push_back(d);
            }
        }
        return FSS_OK;
    }

    int AND(const Shares& x, const Shares& y, uint64_t nrows, Shares* z) {
        if (x.is_public()) { *z = y; return FSS_OK; }
        if (y.is_public()) { *z = x; return FSS_OK; }
        const uint64_t nw = words_of(nrows);
        Shares out;
        for (int b = 0; b < 2; b++)
            if (!(out.p[b] = ws.take(nw))) return fail(FSS_ENOMEM, "match_query: workspace too small");
        int rc = launch_triples(P->seed, P->query_id, next_and++, nw, trip[0], trip[1], s);
        if (rc) return rc;
        if (nw) {
            hipLaunchKernelGGL(k_and_both, dim3(grid_for(nw, 256, 8192)), dim3(256), 0, s, nw, nrows, x.p[0],
                               x.p[1], y.p[0], y.p[1], trip[0], trip[1], out.p[0], out.p[1]);
            rc = check_launch("k_and_both");
        }
        *z = out;
        return rc;
    }

    int gather(const Shares& m, const uint32_t* idx, Shares* out) {
        if (m.is_public()) { *out = m; return FSS_OK; }
        const uint64_t ne = P->n_edges, nw = words_of(ne);
        for (int b = 0; b < 2; b++)
            if (!(out->p[b] = ws.take(nw))) return fail(FSS_ENOMEM, "match_query: workspace too small");
        if (ne == 0) return FSS_OK;
        const uint64_t nwv = words_of(P->n_vertices);
        if (!pair && !(pair = (uint2*)ws.take(2 * nwv))) return fail(FSS_ENOMEM, "match_query: workspace too small");
        if (nwv) {
            hipLaunchKernelGGL(k_interleave, dim3(grid_for(nwv, 256, 8192)), dim3(256), 0, s, nwv, m.p[0], m.p[1],
                               pair);
            int rc = check_launch("k_interleave");
            if (rc) return rc;
        }
        hipLaunchKernelGGL(k_gather, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, ne, P->n_vertices, idx,
                           (const uint2*)pair, out->p[0], out->p[1]);
        return check_launch("k_gather");
    }

    int emit(const Shares& m, uint64_t nrows, uint64_t word_offset) {
        const uint64_t nw = words_of(nrows);
        if (nw == 0) return FSS_OK;
        uint32_t* o0 = P->d_out[0] + word_offset;
        uint32_t* o1 = P->d_out[1] + word_offset;
        if (m.is_public()) {
            hipLaunchKernelGGL(k_public_one, dim3(grid_for(nw, 256, 8192)), dim3(256), 0, s, nw, nrows, o0, o1);
            return check_launch("k_public_one");
        }
        hipLaunchKernelGGL(k_copy_words, dim3(grid_for(nw, 256, 8192)), dim3(256), 0, s, nw, m.p[0], m.p[1], o0, o1);
        return check_launch("k_copy_words");
    }

    // Steps 2 and 3 of the plan, after the predicate bits exist.
    int finish() {
        Shares m[FSS_MAX_QV], q[FSS_MAX_QV];
        for (uint32_t i = 0; i < P->n_qv; i++)
            for (uint32_t k = 0; k < P->n_pred; k++)
                if ((uint32_t)P->preds[k].target == i) {
                    int rc = AND(m[i], pbits[k], P->n_vertices, &m[i]);
                    if (rc) return rc;
                }
        for (uint32_t j = 0; j + 1 < P->n_qv; j++)
            for (uint32_t k = 0; k < P->n_pred; k++)
                if ((uint32_t)P->preds[k].target == P->n_qv + j) {
                    int rc = AND(q[j], pbits[k], P->n_edges, &q[j]);
                    if (rc) return rc;
                }
        if (P->n_qv == 1) return emit(m[0], P->n_vertices, 0);
        const uint64_t we = words_of(P->n_edges);
        for (uint32_t j = 0; j + 1 < P->n_qv; j++) {
            Shares g, h, r1, r2;
            int rc = gather(m[j], P->d_src, &g);
            if (!rc) rc = gather(m[j + 1], P->d_dst, &h);
            if (!rc) rc = AND(g, h, P->n_edges, &r1);
            if (!rc) rc = AND(r1, q[j], P->n_edges, &r2);
            if (!rc) rc = emit(r2, P->n_edges, (uint64_t)j * we);
            if (rc) return rc;
        }
        return FSS_OK;
    }
};

// ----------------------------------------------------------------- batch queue plumbing

struct Tuning {
    uint32_t rows_per_thread = 1;   // eval tile = 1024 * rows_per_thread rows
    uint32_t wg_per_cu = 2;         // persistent grid = wg_per_cu * CUs
};
Tuning g_tuning;

// Descriptor uploads go through a ring of pinned host slots.  A slot is
// rewritten only after the copy that last read it has executed (its event),
// so the host can run several batch calls ahead of the stream.  Device-side
// queue buffers need no such care: an upload and the kernel that reads it are
// ordered on the caller's stream.
constexpr int kStagingSlots = 8;

struct StagingSlot {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};

struct Staging {
    std::mutex mu;
    StagingSlot slot[kStagingSlots];
    int next = 0;
};
Staging g_staging;

// Under stream capture the ring cannot serve: a captured copy would read its
// pinned slot at every replay, after later calls have rewritten it, and the
// slot wait is a host synchronisation.  There the descriptors travel as
// kernel arguments instead, 2 KiB per launch, which a graph keeps by value.
constexpr size_t kArgChunk = 2048;

struct ArgChunk {
    uint32_t w[kArgChunk / 4];
};

__global__ void k_put_words(uint32_t* __restrict__ dst, uint32_t nwords, ArgChunk c) {
    for (uint32_t i = threadIdx.x; i < nwords; i += blockDim.x) dst[i] = c.w[i];
}

int upload_as_arguments(const void* src, size_t bytes, void* d_dst, hipStream_t s) {
    for (size_t off = 0; off < bytes; off += kArgChunk) {
        const size_t n = bytes - off < kArgChunk ? bytes - off : kArgChunk;
        ArgChunk c{};
        memcpy(c.w, (const uint8_t*)src + off, n);
        hipLaunchKernelGGL(k_put_words, dim3(1), dim3(256), 0, s, (uint32_t*)((uint8_t*)d_dst + off),
                           (uint32_t)((n + 3) / 4), c);
        const int rc = check_launch("k_put_words");
        if (rc) return rc;
    }
    return FSS_OK;
}

int upload(const void* src, size_t bytes, void* d_dst, hipStream_t s) {
    hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
    if (s && hipStreamIsCapturing(s, &capture) == hipSuccess && capture != hipStreamCaptureStatusNone)
        return upload_as_arguments(src, bytes, d_dst, s);
    std::lock_guard<std::mutex> lock(g_staging.mu);
    StagingSlot& sl = g_staging.slot[g_staging.next];
    g_staging.next = (g_staging.next + 1) % kStagingSlots;
    if (sl.pending) {
        if (hipEventSynchronize(sl.done) != hipSuccess) return fail(FSS_EDEVICE, "batch: staging wait failed");
        sl.pending = false;
    }
    if (!sl.done && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
        return fail(FSS_EDEVICE, "batch: event creation failed");
    if (sl.cap < bytes) {
        if (sl.host) (void)hipHostFree(sl.host);
        sl.host = nullptr;
        sl.cap = 0;
        if (hipHostMalloc(&sl.host, bytes, hipHostMallocDefault) != hipSuccess)
            return fail(FSS_EDEVICE, "batch: pinned staging allocation failed");
        sl.cap = bytes;
    }
    memcpy(sl.host, src, bytes);
    if (hipMemcpyAsync(d_dst, sl.host, bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipEventRecord(sl.done, s) != hipSuccess)
        return fail(FSS_EDEVICE, "batch: descriptor upload failed");
    sl.pending = true;
    return FSS_OK;
}

// Release the ring: wait for each slot's last copy, then free its pinned
// buffer and event.  Slots are re-created on demand afterwards.
int staging_release() {
    std::lock_guard<std::mutex> lock(g_staging.mu);
    int rc = FSS_OK;
    for (StagingSlot& sl : g_staging.slot) {
        if (sl.pending && hipEventSynchronize(sl.done) != hipSuccess) rc = FSS_EDEVICE;
        sl.pending = false;
        if (sl.host && hipHostFree(sl.host) != hipSuccess) rc = FSS_EDEVICE;
        if (sl.done && hipEventDestroy(sl.done) != hipSuccess) rc = FSS_EDEVICE;
        sl = StagingSlot{};
    }
    g_staging.next = 0;
    return rc;
}

constexpr uint64_t kQueueHeader = 256;   // the tile counter

uint64_t queue_bytes(uint64_t count) {
    const uint64_t per = sizeof(QKeygen) > sizeof(QEval) ? sizeof(QKeygen) : sizeof(QEval);
    return kQueueHeader + ((count * per + 255) & ~255ull);
}

// Heaviest descriptors first (ranges, then larger tables), tile offsets, one launch.
int launch_eval_queue(std::vector<EvalDesc>& descs, void* d_ws, uint64_t ws_bytes, hipStream_t s) {
    std::vector<QEval> q;
    q.reserve(descs.size());
    for (int pass = 0; pass < 2; pass++)
        for (auto& d : descs)
            if ((pass == 0) == (d.kind == FSS_RANGE) && d.n > 0) q.push_back(QEval{d});
    std::stable_sort(q.begin(), q.end(), [](const QEval& a, const QEval& b) {
        return (a.d.kind == FSS_RANGE) != (b.d.kind == FSS_RANGE) ? a.d.kind == FSS_RANGE : a.d.n > b.d.n;
    });
    if (q.empty()) return FSS_OK;
    const uint64_t tile_rows = (uint64_t)kBlock * g_tuning.rows_per_thread;
    uint64_t tiles = 0;
    for (auto& e : q) {
        e.d.block_start = (uint32_t)tiles;
        tiles += (e.d.n + tile_rows - 1) / tile_rows;
    }
    if (tiles > 0xFFFFFFF0ull) return fail(FSS_EUNSUPPORTED, "batch: too many tiles");
    if (!d_ws || ws_bytes < queue_bytes(q.size()))
        return fail(FSS_ENOMEM, "batch: queue workspace needs %llu bytes", (unsigned long long)queue_bytes(q.size()));
    uint32_t* counter = (uint32_t*)d_ws;
    QEval* dq = (QEval*)((uint8_t*)d_ws + kQueueHeader);
    int rc = upload(q.data(), q.size() * sizeof(QEval), dq, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s, counter);
    const uint64_t grid = std::min<uint64_t>(tiles, (uint64_t)g_tuning.wg_per_cu * device_cus());
    hipLaunchKernelGGL(k_eval_queue, dim3((unsigned)grid), dim3(kBlock), 0, s, dq, (uint32_t)q.size(),
                       (uint32_t)tiles, g_tuning.rows_per_thread, counter);
    return check_launch("k_eval_queue");
}

}  // namespace

extern "C" {

uint64_t match_workspace_bytes(const match_plan* plan) {
    if (!plan || plan->n_qv == 0 || plan->n_qv > FSS_MAX_QV || plan->n_pred > FSS_MAX_PREDS) return 0;
    if (plan->n_pred && !plan->preds) return 0;
    return plan_workspace(plan);
}

int match_query(const match_plan* P, int32_t party_mask, void* stream) {
    ogm::last_error().clear();
    if (party_mask != 3) return fail(FSS_EUNSUPPORTED, "match_query: party_mask must be 3 (both parties simulated)");
    int rc = validate_plan(P, "match_query");
    if (rc) return rc;
    PlanRun R{P, (hipStream_t)stream, Arena{(uint8_t*)P->d_workspace, P->workspace_bytes, 0}};
    std::vector<EvalDesc> descs;
    rc = R.setup(descs);
    if (rc) return rc;
    // every predicate, both parties, in launches of up to kEvalInline descriptors
    for (size_t i = 0; i < descs.size(); i += kEvalInline) {
        rc = launch_eval(descs.data() + i, (uint32_t)std::min<size_t>(kEvalInline, descs.size() - i), R.s);
        if (rc) return rc;
    }
    return R.finish();
}

uint64_t fss_queue_workspace_bytes(uint64_t count) { return queue_bytes(count); }

int fss_eval_all(int32_t party, const fss_keybatch* k, uint64_t key_row, uint64_t npoints, uint32_t* d_out_bits,
                 void* stream) {
    ogm::last_error().clear();
    if (!k) return fail(FSS_EINVAL, "fss_eval_all: key batch is NULL");
    int rc = check_batch(k, k->kind, "fss_eval_all");
    if (rc) return rc;
    if (party != 0 && party != 1) return fail(FSS_EINVAL, "fss_eval_all: party %d is not 0 or 1", party);
    if (key_row >= k->n) return fail(FSS_EINVAL, "fss_eval_all: key row %llu of %llu", (unsigned long long)key_row,
                                     (unsigned long long)k->n);
    if (npoints > (1ull << k->nbits)) return fail(FSS_EINVAL, "fss_eval_all: more points than the domain");
    if (npoints == 0) return FSS_OK;
    if (!d_out_bits || !k->key[party] || !aligned256(k->key[party])) return fail(FSS_EINVAL, "fss_eval_all: buffers");
    hipLaunchKernelGGL(k_eval_points, dim3((unsigned)((npoints + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       (hipStream_t)stream, (const uint8_t*)k->key[party], k->n, key_row, (uint32_t)k->kind,
                       k->nbits, (uint32_t)party, npoints, d_out_bits);
    return check_launch("k_eval_points");
}

int fss_eval_all_batch(const fss_eval_all_req* reqs, uint32_t count, void* stream) {
    ogm::last_error().clear();
    if (count == 0) return FSS_OK;
    if (!reqs) return fail(FSS_EINVAL, "fss_eval_all_batch: reqs is NULL");
    for (uint32_t i = 0; i < count; i++) {
        const fss_eval_all_req& r = reqs[i];
        const fss_keybatch* k = r.keys;
        if (!k) return fail(FSS_EINVAL, "fss_eval_all_batch: request %u has no keys", i);
        int rc = check_batch(k, k->kind, "fss_eval_all_batch");
        if (rc) return rc;
        if (r.party != 0 && r.party != 1) return fail(FSS_EINVAL, "fss_eval_all_batch: request %u party", i);
        if (r.key_row >= k->n) return fail(FSS_EINVAL, "fss_eval_all_batch: request %u key row", i);
        if (r.npoints > (1ull << k->nbits)) return fail(FSS_EINVAL, "fss_eval_all_batch: request %u points", i);
        if (r.npoints && (!r.d_out_bits || !k->key[r.party] || !aligned256(k->key[r.party])))
            return fail(FSS_EINVAL, "fss_eval_all_batch: request %u buffers", i);
    }
    for (uint32_t i0 = 0; i0 < count; i0 += kEvalAllMax) {
        EvalAllBatch B{};
        uint64_t blocks = 0;
        const uint32_t m = count - i0 < (uint32_t)kEvalAllMax ? count - i0 : (uint32_t)kEvalAllMax;
        for (uint32_t j = 0; j < m; j++) {
            const fss_eval_all_req& r = reqs[i0 + j];
            EvalAllReq& e = B.r[j];
            e.key = (const uint8_t*)r.keys->key[r.party];
            e.out = r.d_out_bits;
            e.n = r.keys->n;
            e.row = r.key_row;
            e.npoints = r.npoints;
            e.kind = (uint32_t)r.keys->kind;
            e.nbits = r.keys->nbits;
            e.party = (uint32_t)r.party;
            const uint64_t b = (r.npoints + kBlock - 1) / kBlock;
            blocks = b > blocks ? b : blocks;
        }
        if (blocks == 0) continue;
        hipLaunchKernelGGL(k_eval_points_batch, dim3((unsigned)blocks, m), dim3(kBlock), 0, (hipStream_t)stream, B);
        int rc = check_launch("k_eval_points_batch");
        if (rc) return rc;
    }
    return FSS_OK;
}

static int rss_run(uint64_t nrows, const uint32_t* const* d_x, const uint32_t* const* d_y, const uint64_t* prf_keys,
            uint32_t counter, uint32_t* const* d_z, void* stream, const char* who) {
    ogm::last_error().clear();
    if (nrows == 0) return FSS_OK;
    if (!d_x || !d_z || !prf_keys) return fail(FSS_EINVAL, "%s: NULL argument", who);
    RssArgs A{};
    for (int i = 0; i < 3; i++) {
        if (!d_x[i] || !d_z[i] || (d_y && !d_y[i])) return fail(FSS_EINVAL, "%s: NULL share %d", who, i);
        A.prf[i] = ogm::chacha_key(prf_keys[i], 5);
        A.x[i] = d_x[i];
        A.y[i] = d_y ? d_y[i] : nullptr;
        A.z[i] = d_z[i];
    }
    A.nrows = nrows;
    A.nwords = (nrows + 31) / 32;
    A.counter = counter;
    A.vec = 1;
    for (int i = 0; i < 3; i++)
        if (!aligned16(A.x[i]) || !aligned16(A.y[i]) || !aligned16(A.z[i])) A.vec = 0;
    const uint64_t groups = (A.nwords + 3) / 4;
    if (A.nwords > (1ull << 36))        // PRF block numbers are 32-bit: 16 words a block
        return fail(FSS_EUNSUPPORTED, "%s: %llu rows is more than 2^41", who, (unsigned long long)nrows);
    hipLaunchKernelGGL(k_rss, dim3((unsigned)((groups + kRssBlock - 1) / kRssBlock)), dim3(kRssBlock), 0,
                       (hipStream_t)stream, A);
    return check_launch("k_rss");
}


int rss_reshare(uint64_t nrows, const uint32_t* const d_x[3], const uint64_t prf_keys[3], uint32_t counter,
                uint32_t* const d_z[3], void* stream) {
    return rss_run(nrows, d_x, nullptr, prf_keys, counter, d_z, stream, "rss_reshare");
}

int rss_and(uint64_t nrows, const uint32_t* const d_x[3], const uint32_t* const d_y[3], const uint64_t prf_keys[3],
            uint32_t counter, uint32_t* const d_z[3], void* stream) {
    if (!d_y) { ogm::last_error() = "rss_and: NULL y"; return FSS_EINVAL; }
    return rss_run(nrows, d_x, d_y, prf_keys, counter, d_z, stream, "rss_and");
}

int rss_sec_eval(uint64_t ncand, uint32_t npos, const uint32_t* d_eval_a, const uint32_t* d_eval_b,
                 const uint32_t* d_share_a, const uint32_t* d_share_b, uint32_t* d_out_bits, void* stream) {
    ogm::last_error().clear();
    if (ncand == 0) return FSS_OK;
    if (npos == 0) return fail(FSS_EINVAL, "rss_sec_eval: no positions");
    if (!d_eval_a || !d_eval_b || !d_share_a || !d_share_b || !d_out_bits)
        return fail(FSS_EINVAL, "rss_sec_eval: NULL buffer");
    hipLaunchKernelGGL(k_rss_eval, dim3((unsigned)((ncand + 255) / 256)), dim3(256), 0, (hipStream_t)stream, ncand,
                       (npos + 31) / 32, d_eval_a, d_eval_b, d_share_a, d_share_b, d_out_bits);
    return check_launch("k_rss_eval");
}

int fss_set_tuning(uint32_t rows_per_thread, uint32_t wg_per_cu) {
    ogm::last_error().clear();
    if (rows_per_thread < 1 || rows_per_thread > 8 || wg_per_cu < 1 || wg_per_cu > 2)
        return fail(FSS_EINVAL, "fss_set_tuning: rows_per_thread 1..8, wg_per_cu 1..2");
    g_tuning.rows_per_thread = rows_per_thread;
    g_tuning.wg_per_cu = wg_per_cu;
    return FSS_OK;
}

int fss_get_tuning(uint32_t* rows_per_thread, uint32_t* wg_per_cu) {
    if (rows_per_thread) *rows_per_thread = g_tuning.rows_per_thread;
    if (wg_per_cu) *wg_per_cu = g_tuning.wg_per_cu;
    return FSS_OK;
}

int fss_keygen_batch(const fss_keygen_req* reqs, uint32_t count, void* d_queue, uint64_t queue_bytes_avail,
                     void* stream) {
    ogm::last_error().clear();
    if (count == 0) return FSS_OK;
    if (!reqs) return fail(FSS_EINVAL, "fss_keygen_batch: reqs is NULL");
    std::vector<QKeygen> q;
    q.reserve(count);
    for (uint32_t i = 0; i < count; i++) {
        const fss_keygen_req& r = reqs[i];
        const fss_keybatch* out = r.out;
        if (!out) return fail(FSS_EINVAL, "fss_keygen_batch: request %u has no output", i);
        if (out->kind != FSS_EQ && out->kind != FSS_RANGE)
            return fail(FSS_EINVAL, "fss_keygen_batch: request %u bad kind", i);
        if (!valid_nbits(out->nbits)) return fail(FSS_EINVAL, "fss_keygen_batch: request %u nbits", i);
        if (out->n > 0xFFFFFFFFull) return fail(FSS_EUNSUPPORTED, "fss_keygen_batch: more than 2^32 rows");
        const uint64_t lim = 1ull << out->nbits;
        if (out->kind == FSS_EQ && r.a_or_lo >= lim) return fail(FSS_EINVAL, "fss_keygen_batch: request %u a", i);
        if (out->kind == FSS_RANGE && (r.a_or_lo > r.hi || r.hi >= lim))
            return fail(FSS_EINVAL, "fss_keygen_batch: request %u bounds", i);
        if (out->n == 0) continue;
        if (!r.d_r || !out->key[0] || !out->key[1] || !aligned256(out->key[0]) || !aligned256(out->key[1]))
            return fail(FSS_EINVAL, "fss_keygen_batch: request %u buffers", i);
        QKeygen e{};
        e.a.rk = dealer_key(r.seed);
        e.a.key0 = (uint8_t*)out->key[0];
        e.a.key1 = (uint8_t*)out->key[1];
        e.a.r = r.d_r;
        e.a.n = out->n;
        e.a.kind = (uint32_t)out->kind;
        e.a.nbits = out->nbits;
        e.a.query = r.query_id;
        e.a.pred = r.pred_id;
        e.a.a_or_lo = r.a_or_lo;
        e.a.hi = r.hi;
        e.a.row_offset = r.row_offset;
        if ((uint64_t)r.row_offset + out->n > (1ull << 32))
            return fail(FSS_EUNSUPPORTED, "fss_keygen_batch: request %u rows beyond 2^32", i);
        q.push_back(e);
    }
    if (q.empty()) return FSS_OK;
    std::stable_sort(q.begin(), q.end(), [](const QKeygen& a, const QKeygen& b) {
        return (a.a.kind == FSS_RANGE) != (b.a.kind == FSS_RANGE) ? a.a.kind == FSS_RANGE : a.a.n > b.a.n;
    });
    // range descriptors first, then equality ones; tile numbers restart per kind
    const size_t n_range = (size_t)(std::find_if(q.begin(), q.end(),
                                                 [](const QKeygen& e) { return e.a.kind != FSS_RANGE; }) -
                                    q.begin());
    uint64_t tiles[2] = {0, 0};
    for (size_t i = 0; i < q.size(); i++) {
        uint64_t& t = tiles[i < n_range ? 0 : 1];
        q[i].tile_start = (uint32_t)t;
        t += (q[i].a.n + kBlock / 2 - 1) / (kBlock / 2);
    }
    if (tiles[0] > 0xFFFFFFF0ull || tiles[1] > 0xFFFFFFF0ull)
        return fail(FSS_EUNSUPPORTED, "fss_keygen_batch: too many tiles");
    if (!d_queue || queue_bytes_avail < queue_bytes(q.size()))
        return fail(FSS_ENOMEM, "fss_keygen_batch: queue workspace needs %llu bytes",
                    (unsigned long long)queue_bytes(q.size()));
    hipStream_t s = (hipStream_t)stream;
    uint32_t* counter = (uint32_t*)d_queue;
    QKeygen* dq = (QKeygen*)((uint8_t*)d_queue + kQueueHeader);
    int rc = upload(q.data(), q.size() * sizeof(QKeygen), dq, s);
    if (rc) return rc;
    const uint64_t slots = (uint64_t)g_tuning.wg_per_cu * device_cus();
    // the two launches share the counter; stream order puts each zeroing
    // after the previous launch has drained
    if (tiles[0]) {
        hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s, counter);
        hipLaunchKernelGGL(k_keygen_queue_range, dim3((unsigned)std::min(tiles[0], slots)), dim3(kBlock), 0, s,
                           dq, (uint32_t)n_range, (uint32_t)tiles[0], counter);
        rc = check_launch("k_keygen_queue_range");
        if (rc) return rc;
    }
    if (tiles[1]) {
        hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s, counter);
        hipLaunchKernelGGL(k_keygen_queue_eq, dim3((unsigned)std::min(tiles[1], slots)), dim3(kBlock), 0, s,
                           dq + n_range, (uint32_t)(q.size() - n_range), (uint32_t)tiles[1], counter);
        rc = check_launch("k_keygen_queue_eq");
    }
    return rc;
}

int fss_eval_batch(const fss_eval_req* reqs, uint32_t count, void* d_queue, uint64_t queue_bytes_avail,
                   void* stream) {
    ogm::last_error().clear();
    if (count == 0) return FSS_OK;
    if (!reqs) return fail(FSS_EINVAL, "fss_eval_batch: reqs is NULL");
    std::vector<EvalDesc> descs;
    descs.reserve(count);
    for (uint32_t i = 0; i < count; i++) {
        const fss_eval_req& r = reqs[i];
        if (!r.keys) return fail(FSS_EINVAL, "fss_eval_batch: request %u has no keys", i);
        int rc = check_batch(r.keys, r.keys->kind, "fss_eval_batch");
        if (rc) return rc;
        if (r.party != 0 && r.party != 1) return fail(FSS_EINVAL, "fss_eval_batch: request %u party", i);
        if (r.keys->n == 0) continue;
        if (!r.d_xhat || !r.d_out_bits || !r.keys->key[r.party] || !aligned256(r.keys->key[r.party]))
            return fail(FSS_EINVAL, "fss_eval_batch: request %u buffers", i);
        EvalDesc d{};
        d.key = (const uint8_t*)r.keys->key[r.party];
        d.xhat = r.d_xhat;
        d.out = r.d_out_bits;
        d.n = r.keys->n;
        d.kind = (uint32_t)r.keys->kind;
        d.nbits = r.keys->nbits;
        d.party = (uint32_t)r.party;
        descs.push_back(d);
    }
    return launch_eval_queue(descs, d_queue, queue_bytes_avail, (hipStream_t)stream);
}

int match_query_batch(const match_plan* plans, uint32_t count, int32_t party_mask, void* d_queue,
                      uint64_t queue_bytes_avail, void* stream) {
    ogm::last_error().clear();
    if (count == 0) return FSS_OK;
    if (!plans) return fail(FSS_EINVAL, "match_query_batch: plans is NULL");
    if (party_mask != 3)
        return fail(FSS_EUNSUPPORTED, "match_query_batch: party_mask must be 3 (both parties simulated)");
    for (uint32_t i = 0; i < count; i++) {
        int rc = validate_plan(&plans[i], "match_query_batch");
        if (rc) return rc;
    }
    hipStream_t s = (hipStream_t)stream;
    std::vector<PlanRun> runs;
    runs.reserve(count);
    std::vector<EvalDesc> descs;
    for (uint32_t i = 0; i < count; i++) {
        const match_plan* P = &plans[i];
        runs.push_back(PlanRun{P, s, Arena{(uint8_t*)P->d_workspace, P->workspace_bytes, 0}});
        int rc = runs.back().setup(descs);
        if (rc) return rc;
    }
    int rc = launch_eval_queue(descs, d_queue, queue_bytes_avail, s);
    if (rc) return rc;
    for (auto& R : runs) {
        rc = R.finish();
        if (rc) return rc;
    }
    return FSS_OK;
}

}  // extern "C"
