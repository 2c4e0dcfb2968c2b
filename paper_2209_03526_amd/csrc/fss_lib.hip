// fss_lib.hip -- kernels and C ABI of the masked-input FSS library (gfx950).
//
// What is computed, and where the paper defines it, is stated per entry point
// in include/oblivgm_fss.h.  This file holds:
//   k_mask_open            xhat = x0 + x1 + r                          (HBM stream)
//   k_keygen_eq/_range     dealer: DPF / 2xDCF Gen per row             (LDS + VALU, AES)
//   k_eval                 DPF / 2xDCF Eval per row, ballot            (LDS + VALU, AES)
//   k_triples              dealer: Beaver triples (ss_triples)         (LDS + VALU, AES)
//   k_and_open/close       one party's AND phases (ss_and)             (HBM stream)
//   k_tail                 a plan's ANDs and hop joins, triples drawn in registers
//                                                                      (gathers + AES)
//   k_rss, k_rss_eval, k_eval_points*   the paper's own secEval and RSS arithmetic
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
// A tile is tile_mult groups of kBlock / 2 rows (a lane pair per row).
template <int KIND>
__device__ __forceinline__ void keygen_queue(const QKeygen* __restrict__ q, uint32_t count, uint32_t total_tiles,
                                             uint32_t tile_mult, uint32_t* counter) {
    __shared__ uint32_t tab[kLdsTableWords];
    __shared__ uint32_t s_tile;
    lds_table_fill(tab, g_tables.t0);
    const LaneOff loff = lane_offset();
    for (;;) {
        const uint32_t tile = next_tile(counter, &s_tile);   // also orders the table fill
        if (tile >= total_tiles) break;
        const uint32_t di = find_desc(count, tile, [&](uint32_t i) { return q[i].tile_start; });
        const DealerArgs& A = q[di].a;
        const uint64_t row0 = (uint64_t)(tile - q[di].tile_start) * tile_mult * (kBlock / 2) + (threadIdx.x >> 1);
        for (uint32_t k = 0; k < tile_mult; k++) {
            const uint64_t row = row0 + (uint64_t)k * (kBlock / 2);
            if (row < A.n) keygen_row<KIND>(A, row, threadIdx.x & 1u, tab, loff);
        }
    }
}

__global__ __launch_bounds__(kBlock, 8) void k_keygen_queue_eq(const QKeygen* __restrict__ q, uint32_t count,
                                                           uint32_t total_tiles, uint32_t tile_mult,
                                                           uint32_t* counter) {
    keygen_queue<FSS_EQ>(q, count, total_tiles, tile_mult, counter);
}

__global__ __launch_bounds__(kBlock, 8) void k_keygen_queue_range(const QKeygen* __restrict__ q, uint32_t count,
                                                              uint32_t total_tiles, uint32_t tile_mult,
                                                              uint32_t* counter) {
    keygen_queue<FSS_RANGE>(q, count, total_tiles, tile_mult, counter);
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

// The same with candidate-major shares (word w of candidate c at
// [c * nwords_pos + w]): the one-hot records that secFetch and secAccess hand
// over.  One thread per candidate reads its record's words in turn.
__global__ void k_rss_eval_rec(uint64_t ncand, uint32_t nwords_pos, const uint32_t* __restrict__ eval_a,
                               const uint32_t* __restrict__ eval_b, const uint32_t* __restrict__ share_a,
                               const uint32_t* __restrict__ share_b, uint32_t* __restrict__ out) {
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    if (c < ncand) {
        const uint64_t base = c * nwords_pos;
        for (uint32_t w = 0; w < nwords_pos; w++) {
            acc = __builtin_amdgcn_bitop3_b32(acc, share_a[base + w], eval_a[w], 0x78);
            acc = __builtin_amdgcn_bitop3_b32(acc, share_b[base + w], eval_b[w], 0x78);
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

// ----------------------------------------------------------------- three-party RSS arithmetic

struct RssArgs {
    ChachaKey prf[3];       // F(k_i, .) = ChaCha12 under (k_i, domain 5)
    const uint32_t* x[3];   // re-share: x[2] may be null (a share of zero: the two-party conversion)
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
            xv[i] = A.x[i] ? ((const uint4*)A.x[i])[m] : make_uint4(0u, 0u, 0u, 0u);   // null: a zero share
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
                zi = A.x[i] ? A.x[i][w] : 0u;
            }
            const uint32_t fi = q == 0 ? f[i].x : q == 1 ? f[i].y : q == 2 ? f[i].z : f[i].w;
            const uint32_t fp = q == 0 ? f[pv].x : q == 1 ? f[pv].y : q == 2 ? f[pv].z : f[pv].w;
            A.z[i][w] = (zi ^ fi ^ fp) & pm;
        }
    }
}

// ----------------------------------------------------------------- plan tail: ANDs and hop joins
//
// The steps of a plan after its predicate bits exist (the ANDs of each vertex
// and edge fold, the hop joins) run as tail ops, many ops per launch: op i
// owns tiles [tile_start_i, tile_start_i + tiles_i) of one global tile range,
// and each workgroup walks tiles blockIdx.x, blockIdx.x + gridDim.x, ...  A
// tile is 1024 packed words: one word per thread for the word ops, one wave
// per 64 words (2048 edges) for the gathering ops.  The Beaver triple words
// an AND consumes are drawn in registers from the dealer's generator, so no
// triple buffer exists.

enum TailKind : uint32_t {
    TK_AND = 0,         // both parties: z = x AND y
    TK_AND_OPEN = 1,    // one party: msg = (x_b ^ a_b) || (y_b ^ b_b)
    TK_AND_CLOSE = 2,   // one party: z_b from d = x_b ^ a_b ^ d', e = y_b ^ b_b ^ e' (peer message d' || e')
    TK_PAIR = 3,        // both parties: pair[w] = (m_0[w], m_1[w])
    TK_HOP = 4,         // both parties: z = (m_j[src] AND m_j+1[dst]) AND q_j (public operands skipped)
    TK_GATHER = 5,      // one party: z_b = bits of m_b at the public indices
    TK_COPY = 6,        // the parties in `party`: z_b = x_b
    TK_ONE = 7,         // the parties in `party`: their shares of the public constant 1
};

constexpr uint32_t kTailTileWords = 1024;
constexpr uint32_t kNoAnd = 0xFFFFFFFFu;
// TK_HOP flags
constexpr uint32_t kHopSrc = 1, kHopDst = 2, kHopQ = 4;

struct TailOp {
    uint32_t kind;
    uint32_t party;         // single-party kinds: 0 / 1; COPY / ONE: bit mask of parties; AND: 1 = pairs
                            // out; HOP: flags
    uint32_t query;
    uint32_t and1;          // AND number of the (first) AND
    uint32_t and2;          // TK_HOP: number of the AND with q_j
    uint32_t rk;            // dealer key schedule (index into the launch's table)
    uint32_t tile_start;
    uint32_t pad;
    uint64_t nrows;         // rows of the output table
    uint64_t nsrc;          // gathering ops: rows of the vertex table
    const uint32_t* x[2];   // AND: x; PAIR / COPY / GATHER: the source; HOP: q_j
    const uint32_t* y[2];   // AND: y; AND_CLOSE: y[1] = the peer message d' || e'
    uint32_t* z[2];         // outputs (AND_OPEN: z[0] = this party's message; PAIR: z[0] = the pairs)
    const uint32_t* src;    // gathering ops: public indices (HOP: sources)
    const uint32_t* dst;    // HOP: destinations
    const uint2* gsrc;      // HOP: interleaved shares of m_j
    const uint2* gdst;      // HOP: interleaved shares of m_j+1
};

constexpr int kTailInline = 24;

struct TailLaunch {
    const TailOp* ops;      // device array, or nullptr: the inline ops below
    const RoundKeys* rks;   // device array, or nullptr: the inline key below
    uint32_t count;
    uint32_t total_tiles;
    RoundKeys rk;
    TailOp op[kTailInline];
};

__device__ __forceinline__ uint32_t pick4(uint32_t off, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    return off == 0 ? a : off == 1 ? b : off == 2 ? c : d;
}

// Triple word w of Beaver stream (query, and_id): stream words 5w .. 5w+4 are
// a0, a1, b0, b1, c0; stream word k is word k mod 4 of generator block
// (4, 0, query, and_id, k div 4).  Five consecutive words span two blocks.
struct Triple {
    uint32_t a0, a1, b0, b1, c0;
    __device__ uint32_t c1() const { return ((a0 ^ a1) & (b0 ^ b1)) ^ c0; }
};

__device__ __forceinline__ Triple triple_word(const RoundKeys& rk, uint32_t query, uint32_t and_id, uint64_t w,
                                              const uint32_t* tab, LaneOff loff) {
    const uint64_t k0 = 5 * w;
    const uint32_t blk = (uint32_t)(k0 >> 2), off = (uint32_t)(k0 & 3u);
    uint4 p = rng_block(rk, 4, 0, query, and_id, blk, tab, loff);
    pin_in_vgprs(p);
    const uint4 q = rng_block(rk, 4, 0, query, and_id, blk + 1, tab, loff);
    const uint32_t s0 = p.x, s1 = p.y, s2 = p.z, s3 = p.w, s4 = q.x, s5 = q.y, s6 = q.z, s7 = q.w;
    Triple t;
    t.a0 = pick4(off, s0, s1, s2, s3);
    t.a1 = pick4(off, s1, s2, s3, s4);
    t.b0 = pick4(off, s2, s3, s4, s5);
    t.b1 = pick4(off, s3, s4, s5, s6);
    t.c0 = pick4(off, s4, s5, s6, s7);
    return t;
}

// Both parties' AND of one word (open, exchange and close at once).
__device__ __forceinline__ void and_both(const Triple& t, uint32_t x0, uint32_t x1, uint32_t y0, uint32_t y1,
                                         uint32_t pm, uint32_t& z0, uint32_t& z1) {
    const uint32_t d = x0 ^ t.a0 ^ x1 ^ t.a1;
    const uint32_t e = y0 ^ t.b0 ^ y1 ^ t.b1;
    z0 = (t.c0 ^ (d & t.b0) ^ (e & t.a0) ^ (d & e)) & pm;
    z1 = (t.c1() ^ (d & t.b1) ^ (e & t.a1)) & pm;
}

// The bits of the 64 rows [row0, row0 + 64) of one wave, gathered at the
// public indices, become words row0 / 32 and row0 / 32 + 1: lane 2k + h of the
// wave keeps half h of iteration k's ballot.
struct WaveWords {
    uint32_t lane;
    uint32_t w[2];
    __device__ __forceinline__ void keep(uint32_t it, uint32_t k, uint64_t ballot) {
        if (lane == 2 * it) w[k] = (uint32_t)ballot;
        if (lane == 2 * it + 1) w[k] = (uint32_t)(ballot >> 32);
    }
};

// One tile (1024 words) of op o; `tile` counts from the op's first tile.
__device__ __forceinline__ void tail_tile(const TailOp& o, const RoundKeys& rk, uint64_t tile, const uint32_t* tab,
                                          LaneOff loff) {
    const uint64_t nwords = (o.nrows + 31) >> 5;
    if (o.kind == TK_HOP || o.kind == TK_GATHER) {
        // wave v of the workgroup owns words [w0, w0 + 64); lane l ends with word w0 + l
        const uint32_t lane = threadIdx.x & 63u;
        const uint64_t w0 = tile * kTailTileWords + (threadIdx.x & ~63u);
        if (w0 >= nwords) return;                    // whole waves leave
        WaveWords g{lane, {0u, 0u}}, h{lane, {0u, 0u}};
        const bool hop = o.kind == TK_HOP;
        const uint32_t fl = o.party;
        const bool gs = hop ? (fl & kHopSrc) != 0 : true, gd = hop && (fl & kHopDst) != 0;
#pragma unroll 4
        for (uint32_t it = 0; it < 32; it++) {
            const uint64_t e = (w0 + 2 * it) * 32 + lane;
            uint32_t bs0 = 0, bs1 = 0, bd0 = 0, bd1 = 0;
            if (e < o.nrows) {
                if (gs) {
                    const uint32_t v = o.src[e];
                    if (v < o.nsrc) {
                        if (hop) {
                            const uint2 p = o.gsrc[v >> 5];
                            bs0 = (p.x >> (v & 31u)) & 1u;
                            bs1 = (p.y >> (v & 31u)) & 1u;
                        } else {
                            bs0 = (o.x[0][v >> 5] >> (v & 31u)) & 1u;
                        }
                    }
                }
                if (gd) {
                    const uint32_t v = o.dst[e];
                    if (v < o.nsrc) {
                        const uint2 p = o.gdst[v >> 5];
                        bd0 = (p.x >> (v & 31u)) & 1u;
                        bd1 = (p.y >> (v & 31u)) & 1u;
                    }
                }
            }
            if (gs) g.keep(it, 0, __ballot(bs0));
            if (gs && hop) g.keep(it, 1, __ballot(bs1));
            if (gd) h.keep(it, 0, __ballot(bd0));
            if (gd) h.keep(it, 1, __ballot(bd1));
        }
        const uint64_t w = w0 + lane;
        if (w >= nwords) return;
        const uint32_t pm = pad_mask(w, o.nrows);
        if (!hop) {
            o.z[0][w] = g.w[0];
            return;
        }
        // r1 = g AND h (or the one gathered, or public 1); out = r1 AND q (or r1, or q, or public 1)
        bool r1pub = false;
        uint32_t r0, r1;
        if (gs && gd) {
            and_both(triple_word(rk, o.query, o.and1, w, tab, loff), g.w[0], g.w[1], h.w[0], h.w[1], pm, r0, r1);
        } else if (gs) {
            r0 = g.w[0]; r1 = g.w[1];
        } else if (gd) {
            r0 = h.w[0]; r1 = h.w[1];
        } else {
            r0 = pm; r1 = 0u; r1pub = true;
        }
        if (fl & kHopQ) {
            const uint32_t q0 = o.x[0][w], q1 = o.x[1][w];
            if (r1pub) {
                r0 = q0; r1 = q1;
            } else {
                and_both(triple_word(rk, o.query, o.and2, w, tab, loff), r0, r1, q0, q1, pm, r0, r1);
            }
        }
        o.z[0][w] = r0;
        o.z[1][w] = r1;
        return;
    }
    const uint64_t w = tile * kTailTileWords + threadIdx.x;
    if (w >= nwords) return;
    const uint32_t pm = pad_mask(w, o.nrows);
    switch (o.kind) {
    case TK_AND: {
        uint32_t z0, z1;
        and_both(triple_word(rk, o.query, o.and1, w, tab, loff), o.x[0][w], o.x[1][w], o.y[0][w], o.y[1][w], pm, z0,
                 z1);
        if (o.party & 1u) {                              // the fold's last AND: pairs for the join
            ((uint2*)o.z[0])[w] = make_uint2(z0, z1);
        } else {
            o.z[0][w] = z0;
            o.z[1][w] = z1;
        }
        break;
    }
    case TK_AND_OPEN: {
        const Triple t = triple_word(rk, o.query, o.and1, w, tab, loff);
        const uint32_t b = o.party;
        o.z[0][w] = o.x[0][w] ^ (b ? t.a1 : t.a0);
        o.z[0][nwords + w] = o.y[0][w] ^ (b ? t.b1 : t.b0);
        break;
    }
    case TK_AND_CLOSE: {
        const Triple t = triple_word(rk, o.query, o.and1, w, tab, loff);
        const uint32_t b = o.party;
        const uint32_t ab = b ? t.a1 : t.a0, bb = b ? t.b1 : t.b0, cb = b ? t.c1() : t.c0;
        const uint32_t d = o.x[0][w] ^ ab ^ o.y[1][w];
        const uint32_t e = o.y[0][w] ^ bb ^ o.y[1][nwords + w];
        uint32_t z = cb ^ (d & bb) ^ (e & ab);
        if (b == 0) z ^= d & e;
        o.z[0][w] = z & pm;
        break;
    }
    case TK_PAIR:
        ((uint2*)o.z[0])[w] = make_uint2(o.x[0][w], o.x[1][w]);
        break;
    case TK_COPY:
        if (o.party & 1u) o.z[0][w] = o.x[0][w];
        if (o.party & 2u) o.z[1][w] = o.x[1][w];
        break;
    case TK_ONE:
        if (o.party & 1u) o.z[0][w] = pm;
        if (o.party & 2u) o.z[1][w] = 0u;
        break;
    default:
        break;
    }
}

// Ops in tile order; a workgroup fills the AES tables once, then takes every
// gridDim.x-th tile.
__global__ __launch_bounds__(kBlock) void k_tail(TailLaunch L) {
    __shared__ uint32_t tab[kLdsTableWords];
    lds_table_fill(tab, g_tables.t0);
    __syncthreads();
    const LaneOff loff = lane_offset();
    const TailOp* ops = L.ops ? L.ops : L.op;
    for (uint32_t tile = blockIdx.x; tile < L.total_tiles; tile += gridDim.x) {
        const uint32_t di = find_desc(L.count, tile, [&](uint32_t i) { return ops[i].tile_start; });
        const TailOp& o = ops[di];
        tail_tile(o, L.rks ? L.rks[o.rk] : L.rk, tile - o.tile_start, tab, loff);
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

// Carves 256-byte aligned pieces off the workspace.  measuring() gives an
// arena that only counts bytes (its pointers are never dereferenced).
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
    bool take2(uint64_t words, Shares& s) { return (s.p[0] = take(words)) && (s.p[1] = take(words)); }
    static Arena measuring() { return Arena{(uint8_t*)(uintptr_t)256, ~0ull >> 1, 0}; }
};

uint64_t words_of(uint64_t rows) { return (rows + 31) / 32; }

// The plan's query edges (a_j, b_j): q_edges, or the path (j, j + 1) when n_qe
// is 0.  Returns nullptr when they are valid, else what is wrong with them.
const char* query_edges(const match_plan* P, uint32_t* qa, uint32_t* qb, uint32_t* n_qe) {
    if (P->n_qe > FSS_MAX_QE) return "more query edges than FSS_MAX_QE";
    if (P->n_qe && !P->q_edges) return "q_edges is NULL";
    *n_qe = 0;
    if (P->n_qv <= 1) return P->n_qe ? "a one-vertex query has no edges" : nullptr;
    const uint32_t n = P->n_qe ? P->n_qe : P->n_qv - 1;
    uint32_t covered = 0;
    for (uint32_t j = 0; j < n; j++) {
        const uint32_t a = P->n_qe ? P->q_edges[2 * j] : j;
        const uint32_t b = P->n_qe ? P->q_edges[2 * j + 1] : j + 1;
        if (a >= P->n_qv || b >= P->n_qv || a == b) return "a query edge does not join two distinct query vertices";
        for (uint32_t i = 0; i < j; i++)
            if (qa[i] == a && qb[i] == b) return "a query edge is given twice";
        qa[j] = a;
        qb[j] = b;
        covered |= 1u << a | 1u << b;
    }
    if (covered != (1u << P->n_qv) - 1) return "a query vertex is on no query edge";
    *n_qe = n;
    return nullptr;
}

// The plan's steps after evaluation, laid out in the workspace -- a pure
// function of the plan, so every call on the same plan finds the same
// buffers (the single-party rounds rely on it).
//   folds: per target t (query vertices 0..n_qv-1, then query edges) its
//          predicates ANDed as a left fold; step s of a fold is AND level s;
//   hops:  per query edge j = (a_j, b_j), h_j = (m_a[src] AND m_b[dst]) AND q_j;
// AND numbers follow that order (vertex folds, edge folds, then per hop the
// AND of the endpoints and the AND with q_j); an AND with a public operand is
// skipped and takes no number.  Level L of an AND: in a single-party run it
// is opened in round L - 1 and closed in round L.
struct TailPlan {
    struct And {
        uint32_t id, level;
        uint64_t nrows;
        Shares x, y, z;
        int32_t vertex;     // fold AND: the query vertex whose fold it ends, else -1
        bool hop;           // an AND of a hop join
    };
    struct Hop {
        bool g, h, q;               // m_a, m_b, q_j not public
        int32_t a1 = -1, a2 = -1;   // indices into ands
        uint32_t lg = 0;            // round in which the gathers run (single party)
        uint32_t lq = 0;            // round from which q_j is ready
        Shares gs, hs, r1;          // single party: gathered endpoint bits, g AND h
        uint32_t* out[2];
    };
    const match_plan* P = nullptr;
    uint32_t n_qv = 0, n_qe = 0, ntarget = 0;
    uint32_t qa[FSS_MAX_QE] = {}, qb[FSS_MAX_QE] = {};     // query edge j = (qa[j], qb[j])
    uint64_t wv = 0, we = 0;
    Shares pbits[FSS_MAX_PREDS];
    Shares fold[FSS_MAX_QV + FSS_MAX_QE];
    uint32_t depth[FSS_MAX_QV + FSS_MAX_QE] = {};
    uint32_t npred_of[FSS_MAX_QV + FSS_MAX_QE] = {};
    uint32_t first_pred[FSS_MAX_QV + FSS_MAX_QE] = {};
    uint2* pair[FSS_MAX_QV] = {};
    std::vector<And> ands;          // in AND-number order
    Hop hop[FSS_MAX_QE];
    uint32_t rounds = 0;            // single-party exchange rounds

    uint64_t rows_of(uint32_t t) const { return t < n_qv ? P->n_vertices : P->n_edges; }

    int build(const match_plan* plan, Arena& ws) {
        P = plan;
        n_qv = P->n_qv;
        if (const char* bad = query_edges(P, qa, qb, &n_qe)) return fail(FSS_EINVAL, "match_query: %s", bad);
        ntarget = n_qv + n_qe;
        wv = words_of(P->n_vertices);
        we = words_of(P->n_edges);
        auto nomem = [] { return fail(FSS_ENOMEM, "match_query: workspace too small"); };
        for (uint32_t k = 0; k < P->n_pred; k++) {
            const fss_pred& p = P->preds[k];
            if (p.d_bits[0]) {
                pbits[k].p[0] = const_cast<uint32_t*>(p.d_bits[0]);
                pbits[k].p[1] = const_cast<uint32_t*>(p.d_bits[1]);
            } else if (!ws.take2(words_of(rows_of((uint32_t)p.target)), pbits[k])) {
                return nomem();
            }
        }
        for (uint32_t t = 0; t < ntarget; t++) {
            Shares acc;
            for (uint32_t k = 0; k < P->n_pred; k++) {
                if ((uint32_t)P->preds[k].target != t) continue;
                if (npred_of[t]++ == 0) {
                    acc = pbits[k];
                    first_pred[t] = k;
                    continue;
                }
                And a{};
                a.id = (uint32_t)ands.size();
                a.level = ++depth[t];
                a.nrows = rows_of(t);
                a.x = acc;
                a.y = pbits[k];
                a.vertex = -1;
                a.hop = false;
                if (!ws.take2(words_of(a.nrows), a.z)) return nomem();
                acc = a.z;
                ands.push_back(a);
            }
            fold[t] = acc;
            // the fold's last AND ends query vertex t (pairs for the joins)
            if (t < n_qv && depth[t] > 0) ands.back().vertex = (int32_t)t;
        }
        if (n_qv == 1) {
            // the output is m_0: its last AND writes it
            if (depth[0] > 0) {
                ands.back().z.p[0] = P->d_out[0];
                ands.back().z.p[1] = P->d_out[1];
            }
        } else {
            for (uint32_t i = 0; i < n_qv; i++)
                if (!fold[i].is_public() && !(pair[i] = (uint2*)ws.take(2 * wv))) return nomem();
        }
        for (uint32_t j = 0; j < n_qe; j++) {
            Hop& H = hop[j];
            H.g = !fold[qa[j]].is_public();
            H.h = !fold[qb[j]].is_public();
            H.q = !fold[n_qv + j].is_public();
            H.out[0] = P->d_out[0] + (uint64_t)j * we;
            H.out[1] = P->d_out[1] + (uint64_t)j * we;
            H.lg = std::max(H.g ? depth[qa[j]] : 0u, H.h ? depth[qb[j]] : 0u);
            H.lq = depth[n_qv + j];
            if (H.g && !ws.take2(we, H.gs)) return nomem();
            if (H.h && !ws.take2(we, H.hs)) return nomem();
            uint32_t ready = H.lg;          // round in which r1 is ready
            Shares r1 = H.g ? H.gs : H.hs;  // public if neither
            if (H.g && H.h) {
                And a{};
                a.id = (uint32_t)ands.size();
                a.level = H.lg + 1;
                a.nrows = P->n_edges;
                a.x = H.gs;
                a.y = H.hs;
                a.vertex = -1;
                a.hop = true;
                if (!ws.take2(we, H.r1)) return nomem();
                a.z = H.r1;
                H.a1 = (int32_t)ands.size();
                ands.push_back(a);
                ready = a.level;
                r1 = H.r1;
            }
            if (!r1.is_public() && H.q) {
                And a{};
                a.id = (uint32_t)ands.size();
                a.level = std::max(ready, H.lq) + 1;
                a.nrows = P->n_edges;
                a.x = r1;
                a.y = fold[n_qv + j];
                a.z.p[0] = H.out[0];
                a.z.p[1] = H.out[1];
                a.vertex = -1;
                a.hop = true;
                H.a2 = (int32_t)ands.size();
                ands.push_back(a);
            } else if (H.a1 >= 0) {
                ands[H.a1].z.p[0] = H.out[0];   // g AND h is the hop's result
                ands[H.a1].z.p[1] = H.out[1];
            }
        }
        for (const And& a : ands) rounds = std::max(rounds, a.level);
        return FSS_OK;
    }

    // 32-bit words of the message of round r (the openings of the ANDs of level r + 1).
    uint64_t msg_words(uint32_t r) const {
        uint64_t n = 0;
        for (const And& a : ands)
            if (a.level == r + 1) n += 2 * words_of(a.nrows);
        return n;
    }
};

// Workspace bytes of the plan (at least 256, so that 0 can mean "invalid").
uint64_t plan_workspace(const match_plan* P) {
    Arena measure = Arena::measuring();
    TailPlan T;
    if (T.build(P, measure)) return 0;
    return std::max<uint64_t>(measure.used, 256);
}

// Number of tail tiles of an op over `nrows` rows.
uint32_t tail_tiles(uint64_t nrows) { return (uint32_t)((words_of(nrows) + kTailTileWords - 1) / kTailTileWords); }

TailOp tail_op(uint32_t kind, const match_plan* P, uint64_t nrows) {
    TailOp o{};
    o.kind = kind;
    o.query = P->query_id;
    o.and1 = o.and2 = kNoAnd;
    o.nrows = nrows;
    return o;
}

// Both parties at once: per AND level the fold ANDs (a vertex's last AND
// writes its pairs for the joins), with the pairs of one-predicate vertices
// and the output of a one-vertex query in the first level, then one level of
// hop joins.  Level i of the result holds the ops of launch i.
void fused_levels(const TailPlan& T, uint32_t rk, std::vector<std::vector<TailOp>>& levels) {
    const match_plan* P = T.P;
    uint32_t nlev = 0;
    for (const auto& a : T.ands) nlev = std::max(nlev, a.level);
    const uint32_t first = 0, hops = std::max(nlev, 1u);
    if (levels.size() < hops + 1) levels.resize(hops + 1);
    auto put = [&](uint32_t lev, TailOp o) { o.rk = rk; levels[lev].push_back(o); };
    for (const auto& a : T.ands) {
        if (a.hop) continue;
        TailOp o = tail_op(TK_AND, P, a.nrows);
        o.and1 = a.id;
        o.x[0] = a.x.p[0]; o.x[1] = a.x.p[1];
        o.y[0] = a.y.p[0]; o.y[1] = a.y.p[1];
        o.z[0] = a.z.p[0]; o.z[1] = a.z.p[1];
        if (T.n_qv > 1 && a.vertex >= 0) {
            o.party = 1;                           // pairs out
            o.z[0] = (uint32_t*)T.pair[a.vertex];
            o.z[1] = nullptr;
        }
        put(a.level - 1, o);
    }
    if (T.n_qv == 1) {
        if (T.npred_of[0] == 0) {
            TailOp o = tail_op(TK_ONE, P, P->n_vertices);
            o.party = 3;
            o.z[0] = P->d_out[0]; o.z[1] = P->d_out[1];
            put(first, o);
        } else if (T.depth[0] == 0) {
            TailOp o = tail_op(TK_COPY, P, P->n_vertices);
            o.party = 3;
            o.x[0] = T.fold[0].p[0]; o.x[1] = T.fold[0].p[1];
            o.z[0] = P->d_out[0]; o.z[1] = P->d_out[1];
            put(first, o);
        }
        return;
    }
    for (uint32_t i = 0; i < T.n_qv; i++) {
        if (T.fold[i].is_public() || T.depth[i] > 0) continue;
        TailOp o = tail_op(TK_PAIR, P, P->n_vertices);
        o.x[0] = T.fold[i].p[0]; o.x[1] = T.fold[i].p[1];
        o.z[0] = (uint32_t*)T.pair[i];
        put(first, o);
    }
    for (uint32_t j = 0; j < T.n_qe; j++) {
        const TailPlan::Hop& H = T.hop[j];
        TailOp o = tail_op(TK_HOP, P, P->n_edges);
        o.party = (H.g ? kHopSrc : 0) | (H.h ? kHopDst : 0) | (H.q ? kHopQ : 0);
        o.nsrc = P->n_vertices;
        o.src = P->d_src;
        o.dst = P->d_dst;
        o.gsrc = T.pair[T.qa[j]];
        o.gdst = T.pair[T.qb[j]];
        if (H.q) { o.x[0] = T.fold[T.n_qv + j].p[0]; o.x[1] = T.fold[T.n_qv + j].p[1]; }
        if (H.a1 >= 0) o.and1 = T.ands[H.a1].id;
        if (H.a2 >= 0) o.and2 = T.ands[H.a2].id;
        o.z[0] = H.out[0]; o.z[1] = H.out[1];
        put(hops, o);
    }
}

// Party b, round r: the closes of level r (peer: the other party's message of
// round r - 1), then the gathers and copies that become ready in round r, then
// the openings of level r + 1 (msg: this party's message of round r).  The
// three phases are three launches (phase[0..2]).
void party_round(const TailPlan& T, uint32_t b, uint32_t r, const uint32_t* peer, uint32_t* msg, uint32_t rk,
                 std::vector<TailOp> phase[3]) {
    const match_plan* P = T.P;
    uint64_t off = 0;
    for (const auto& a : T.ands) {                 // closes: offsets in round r - 1's message
        if (r == 0 || a.level != r) continue;
        TailOp o = tail_op(TK_AND_CLOSE, P, a.nrows);
        o.party = b;
        o.rk = rk;
        o.and1 = a.id;
        o.x[0] = a.x.p[b];
        o.y[0] = a.y.p[b];
        o.y[1] = peer + off;
        o.z[0] = a.z.p[b];
        phase[0].push_back(o);
        off += 2 * words_of(a.nrows);
    }
    // this party's copy of a share (or of the public 1) into an output
    auto copy = [&](const Shares& from, uint32_t* to0, uint32_t* to1, uint64_t nrows) {
        TailOp o = tail_op(from.is_public() ? TK_ONE : TK_COPY, P, nrows);
        o.party = 1u << b;
        o.rk = rk;
        o.x[0] = from.p[0]; o.x[1] = from.p[1];
        o.z[0] = to0; o.z[1] = to1;
        phase[1].push_back(o);
    };
    if (T.n_qv == 1) {
        if (r == 0 && T.depth[0] == 0) {
            if (T.npred_of[0] == 0) {
                TailOp o = tail_op(TK_ONE, P, P->n_vertices);
                o.rk = rk;
                o.party = 1u << b;
                o.z[0] = P->d_out[0]; o.z[1] = P->d_out[1];
                phase[1].push_back(o);
            } else {
                copy(T.fold[0], P->d_out[0], P->d_out[1], P->n_vertices);
            }
        }
    } else {
        for (uint32_t j = 0; j < T.n_qe; j++) {
            const TailPlan::Hop& H = T.hop[j];
            const bool final_gather = H.a1 < 0 && H.a2 < 0;   // the gathered bits are the result
            if (H.lg == r) {
                for (int side = 0; side < 2; side++) {
                    if (!(side ? H.h : H.g)) continue;
                    TailOp o = tail_op(TK_GATHER, P, P->n_edges);
                    o.party = b;
                    o.rk = rk;
                    o.nsrc = P->n_vertices;
                    o.src = side ? P->d_dst : P->d_src;
                    o.x[0] = T.fold[side ? T.qb[j] : T.qa[j]].p[b];
                    o.z[0] = final_gather ? H.out[b] : (side ? H.hs.p[b] : H.gs.p[b]);
                    phase[1].push_back(o);
                }
            }
            if (!H.g && !H.h) {                    // r1 public: the result is q_j, or the public 1
                if (H.lq == r && H.q) copy(T.fold[T.n_qv + j], H.out[0], H.out[1], P->n_edges);
                if (r == 0 && !H.q) {
                    TailOp o = tail_op(TK_ONE, P, P->n_edges);
                    o.rk = rk;
                    o.party = 1u << b;
                    o.z[0] = H.out[0]; o.z[1] = H.out[1];
                    phase[1].push_back(o);
                }
            }
        }
    }
    off = 0;
    for (const auto& a : T.ands) {                 // openings of level r + 1
        if (a.level != r + 1) continue;
        TailOp o = tail_op(TK_AND_OPEN, P, a.nrows);
        o.party = b;
        o.rk = rk;
        o.and1 = a.id;
        o.x[0] = a.x.p[b];
        o.y[0] = a.y.p[b];
        o.z[0] = msg + off;
        phase[2].push_back(o);
        off += 2 * words_of(a.nrows);
    }
}

int validate_plan(const match_plan* P, int32_t party_mask, const char* who) {
    if (!P) return fail(FSS_EINVAL, "%s: plan is NULL", who);
    if (party_mask < 1 || party_mask > 3) return fail(FSS_EINVAL, "%s: party_mask %d is not 1, 2 or 3", who, party_mask);
    if (P->n_qv == 0 || P->n_qv > FSS_MAX_QV) return fail(FSS_EINVAL, "%s: n_qv %u outside 1..%d", who, P->n_qv, FSS_MAX_QV);
    if (P->n_pred > FSS_MAX_PREDS) return fail(FSS_EINVAL, "%s: more than %d predicates", who, FSS_MAX_PREDS);
    if (P->n_pred && !P->preds) return fail(FSS_EINVAL, "%s: preds is NULL", who);
    if (P->n_vertices > 0xFFFFFFFFull || P->n_edges > 0xFFFFFFFFull)
        return fail(FSS_EUNSUPPORTED, "%s: more than 2^32 rows", who);
    for (int b = 0; b < 2; b++)
        if ((party_mask >> b & 1) && !P->d_out[b]) return fail(FSS_EINVAL, "%s: NULL output of party %d", who, b);
    if (party_mask == 3 && (!P->d_out[0] || !P->d_out[1])) return fail(FSS_EINVAL, "%s: NULL output", who);
    if (P->n_qv > 1 && P->n_edges && (!P->d_src || !P->d_dst)) return fail(FSS_EINVAL, "%s: NULL edge endpoints", who);
    uint32_t qa[FSS_MAX_QE], qb[FSS_MAX_QE], n_qe = 0;
    if (const char* bad = query_edges(P, qa, qb, &n_qe)) return fail(FSS_EINVAL, "%s: %s", who, bad);
    const uint32_t ntarget = P->n_qv + n_qe;
    for (uint32_t k = 0; k < P->n_pred; k++) {
        const fss_pred& p = P->preds[k];
        if (p.target < 0 || (uint32_t)p.target >= ntarget)
            return fail(FSS_EINVAL, "%s: predicate %u targets %d (of %u)", who, k, p.target, ntarget);
        const uint64_t rows = (uint32_t)p.target < P->n_qv ? P->n_vertices : P->n_edges;
        if (p.d_bits[0] || p.d_bits[1]) {
            if (party_mask == 3 && (!p.d_bits[0] || !p.d_bits[1]))
                return fail(FSS_EINVAL, "%s: predicate %u has one bit pointer", who, k);
            if (party_mask != 3 && !p.d_bits[party_mask - 1])
                return fail(FSS_EINVAL, "%s: predicate %u has no bits of party %d", who, k, party_mask - 1);
            continue;   // share bits already evaluated: keys and d_xhat are not used
        }
        if (!p.keys || (p.keys->kind != FSS_EQ && p.keys->kind != FSS_RANGE))
            return fail(FSS_EINVAL, "%s: predicate %u has no valid key batch", who, k);
        int rc = check_batch(p.keys, p.keys->kind, who);
        if (rc) return rc;
        if (p.keys->n != rows)
            return fail(FSS_EINVAL, "%s: predicate %u keys cover %llu rows, table has %llu", who, k,
                        (unsigned long long)p.keys->n, (unsigned long long)rows);
        for (int b = 0; b < 2; b++) {
            if (!(party_mask >> b & 1) || !rows) continue;
            if (!p.d_xhat || !p.keys->key[b]) return fail(FSS_EINVAL, "%s: predicate %u has a NULL buffer", who, k);
            if (!aligned256(p.keys->key[b]))
                return fail(FSS_EINVAL, "%s: predicate %u key buffers not 256-byte aligned", who, k);
        }
    }
    const uint64_t need = plan_workspace(P);
    if (!P->d_workspace || P->workspace_bytes < need)
        return fail(FSS_ENOMEM, "%s: workspace needs %llu bytes", who, (unsigned long long)need);
    return FSS_OK;
}

// Eval descriptors of the plan's predicates for the parties in mask (the
// bits of predicates evaluated by the caller are left alone).
void plan_evals(const TailPlan& T, int32_t mask, std::vector<EvalDesc>& out) {
    const match_plan* P = T.P;
    for (uint32_t k = 0; k < P->n_pred; k++) {
        const fss_pred& p = P->preds[k];
        if (p.d_bits[0] || p.d_bits[1]) continue;
        const uint64_t rows = T.rows_of((uint32_t)p.target);
        if (rows == 0) continue;
        for (int b = 0; b < 2; b++) {
            if (!(mask >> b & 1)) continue;
            EvalDesc d{};
            d.key = (const uint8_t*)p.keys->key[b];
            d.xhat = p.d_xhat;
            d.out = T.pbits[k].p[b];
            d.n = rows;
            d.kind = (uint32_t)p.keys->kind;
            d.nbits = p.keys->nbits;
            d.party = (uint32_t)b;
            out.push_back(d);
        }
    }
}

// Workgroups of a tail launch: two per CU at most (the LDS holds two tables).
unsigned tail_grid(uint32_t tiles) {
    const uint32_t cap = 2u * (uint32_t)device_cus();
    return tiles < 1 ? 1u : (tiles < cap ? tiles : cap);
}

// One launch per kTailInline ops, all carried in kernel arguments (one plan:
// its key schedule rides along).
int launch_tail_inline(const std::vector<TailOp>& ops, const RoundKeys& rk, hipStream_t s) {
    for (size_t i0 = 0; i0 < ops.size(); i0 += kTailInline) {
        TailLaunch L{};
        L.rk = rk;
        uint32_t tiles = 0;
        const size_t n = std::min<size_t>(kTailInline, ops.size() - i0);
        for (size_t i = 0; i < n; i++) {
            L.op[i] = ops[i0 + i];
            L.op[i].rk = 0;
            L.op[i].tile_start = tiles;
            tiles += tail_tiles(L.op[i].nrows);
        }
        L.count = (uint32_t)n;
        L.total_tiles = tiles;
        if (tiles == 0) continue;
        hipLaunchKernelGGL(k_tail, dim3(tail_grid(tiles)), dim3(kBlock), 0, s, L);
        int rc = check_launch("k_tail");
        if (rc) return rc;
    }
    return FSS_OK;
}

// ----------------------------------------------------------------- batch queue plumbing

struct Tuning {
    uint32_t rows_per_thread = 1;   // eval tile = 1024 * rows_per_thread rows
    uint32_t wg_per_cu = 2;         // persistent grid = wg_per_cu * CUs
    uint32_t keygen_tile_mult = 1;  // keygen tile = 512 * keygen_tile_mult rows
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

// Queue order of two requests: ranges before equalities, larger tables first;
// equal keys keep their request order (the sort is stable).
bool eval_before(uint32_t kind_a, uint64_t n_a, uint32_t kind_b, uint64_t n_b) {
    const bool ra = kind_a == FSS_RANGE, rb = kind_b == FSS_RANGE;
    return ra != rb ? ra : n_a > n_b;
}

// The persistent evaluation over a queue already in device memory.
int launch_eval_kernel(const QEval* dq, uint32_t n, uint64_t tiles, uint32_t* counter, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s, counter);
    const uint64_t grid = std::min<uint64_t>(tiles, (uint64_t)g_tuning.wg_per_cu * device_cus());
    hipLaunchKernelGGL(k_eval_queue, dim3((unsigned)grid), dim3(kBlock), 0, s, dq, n, (uint32_t)tiles,
                       g_tuning.rows_per_thread, counter);
    return check_launch("k_eval_queue");
}

// Heaviest descriptors first, tile offsets, one upload, one launch.
int launch_eval_queue(std::vector<EvalDesc>& descs, void* d_ws, uint64_t ws_bytes, hipStream_t s) {
    std::vector<QEval> q;
    q.reserve(descs.size());
    for (auto& d : descs)
        if (d.n > 0) q.push_back(QEval{d});
    std::stable_sort(q.begin(), q.end(), [](const QEval& a, const QEval& b) {
        return eval_before(a.d.kind, a.d.n, b.d.kind, b.d.n);
    });
    if (q.empty()) return FSS_OK;
    const uint64_t tile_rows = (uint64_t)kBlock * g_tuning.rows_per_thread;
    uint64_t tiles = 0;
    for (auto& e : q) {
        e.d.block_start = (uint32_t)tiles;
        tiles += (e.d.n + tile_rows - 1) / tile_rows;
    }
    if (tiles > 0xFFFFFFF0ull) return fail(FSS_EUNSUPPORTED, "batch: too many tiles");
    const uint64_t need = kQueueHeader + q.size() * sizeof(QEval);
    if (!d_ws || ws_bytes < need)
        return fail(FSS_ENOMEM, "batch: queue workspace needs %llu bytes", (unsigned long long)need);
    uint32_t* counter = (uint32_t*)d_ws;
    QEval* dq = (QEval*)((uint8_t*)d_ws + kQueueHeader);
    const int rc = upload(q.data(), q.size() * sizeof(QEval), dq, s);
    if (rc) return rc;
    return launch_eval_kernel(dq, (uint32_t)q.size(), tiles, counter, s);
}

// Device image of a batch's tail: the plans' key schedules, then the ops of
// every launch, one upload for all launches.
uint64_t tail_queue_bytes(uint64_t nplans, uint64_t nops) {
    return kQueueHeader + ((nplans * sizeof(RoundKeys) + 255) & ~255ull) + nops * sizeof(TailOp);
}

int launch_tail_queue(const match_plan* plans, uint32_t count, const std::vector<std::vector<TailOp>>& levels,
                      void* d_ws, uint64_t ws_bytes, hipStream_t s) {
    uint64_t nops = 0;
    for (const auto& l : levels) nops += l.size();
    if (nops == 0) return FSS_OK;
    const uint64_t need = tail_queue_bytes(count, nops);
    if (!d_ws || ws_bytes < need)
        return fail(FSS_ENOMEM, "match_query_batch: queue workspace needs %llu bytes (match_batch_queue_bytes)",
                    (unsigned long long)need);
    const uint64_t rk_bytes = (count * sizeof(RoundKeys) + 255) & ~255ull;
    std::vector<uint8_t> img(rk_bytes + nops * sizeof(TailOp));
    RoundKeys* rks = (RoundKeys*)img.data();
    for (uint32_t i = 0; i < count; i++) rks[i] = dealer_key(plans[i].seed);
    TailOp* ops = (TailOp*)(img.data() + rk_bytes);
    struct Launch { uint64_t first; uint32_t n, tiles; };
    std::vector<Launch> launches;
    uint64_t k = 0;
    for (const auto& l : levels) {
        Launch ln{k, (uint32_t)l.size(), 0};
        for (const TailOp& o : l) {
            ops[k] = o;
            ops[k].tile_start = ln.tiles;
            ln.tiles += tail_tiles(o.nrows);
            k++;
        }
        if (ln.tiles) launches.push_back(ln);
    }
    uint8_t* dbase = (uint8_t*)d_ws + kQueueHeader;
    int rc = upload(img.data(), img.size(), dbase, s);
    if (rc) return rc;
    for (const Launch& ln : launches) {
        TailLaunch L{};
        L.ops = (const TailOp*)(dbase + rk_bytes) + ln.first;
        L.rks = (const RoundKeys*)dbase;
        L.count = ln.n;
        L.total_tiles = ln.tiles;
        hipLaunchKernelGGL(k_tail, dim3(tail_grid(ln.tiles)), dim3(kBlock), 0, s, L);
        rc = check_launch("k_tail");
        if (rc) return rc;
    }
    return FSS_OK;
}

// Requests of a batch evaluation -> descriptors (same checks as the single calls).
// One request's checks; *d gets its descriptor (d->n == 0: nothing to evaluate).
int eval_request(const fss_eval_req& r, uint32_t i, const char* who, EvalDesc* d) {
    if (!r.keys) return fail(FSS_EINVAL, "%s: request %u has no keys", who, i);
    int rc = check_batch(r.keys, r.keys->kind, who);
    if (rc) return rc;
    if (r.party != 0 && r.party != 1) return fail(FSS_EINVAL, "%s: request %u party", who, i);
    *d = EvalDesc{};
    if (r.keys->n == 0) return FSS_OK;
    if (!r.d_xhat || !r.d_out_bits || !r.keys->key[r.party] || !aligned256(r.keys->key[r.party]))
        return fail(FSS_EINVAL, "%s: request %u buffers", who, i);
    d->key = (const uint8_t*)r.keys->key[r.party];
    d->xhat = r.d_xhat;
    d->out = r.d_out_bits;
    d->n = r.keys->n;
    d->kind = (uint32_t)r.keys->kind;
    d->nbits = r.keys->nbits;
    d->party = (uint32_t)r.party;
    return FSS_OK;
}

int eval_requests(const fss_eval_req* reqs, uint32_t count, std::vector<EvalDesc>& descs, const char* who) {
    if (!reqs) return fail(FSS_EINVAL, "%s: reqs is NULL", who);
    descs.reserve(count);
    for (uint32_t i = 0; i < count; i++) {
        EvalDesc d;
        const int rc = eval_request(reqs[i], i, who, &d);
        if (rc) return rc;
        if (d.n) descs.push_back(d);
    }
    return FSS_OK;
}

// The allocation-free batch evaluation keeps its queue (tile counter and up
// to FSS_NOALLOC_EVAL_MAX descriptors) in this file-scope device array: one
// copy per GPU, alive until the process ends, shared by every call on that GPU.
constexpr uint64_t kScratchBytes = 64 * 1024;
static_assert(kQueueHeader + FSS_NOALLOC_EVAL_MAX * sizeof(QEval) <= kScratchBytes, "scratch too small");
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once
// per device with that device current (the array's name is a host-side
// stand-in, not a device address).
int scratch_ptr(void** out, const char* who) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(FSS_EDEVICE, "%s: no current device", who);
    if (dev < 0 || dev >= kMaxDevices) return fail(FSS_EUNSUPPORTED, "%s: device %d", who, dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(FSS_EDEVICE, "%s: scratch address: %s", who, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FSS_OK;
}

}  // namespace

extern "C" {

uint64_t match_workspace_bytes(const match_plan* plan) {
    if (!plan || plan->n_qv == 0 || plan->n_qv > FSS_MAX_QV || plan->n_pred > FSS_MAX_PREDS) return 0;
    if (plan->n_pred && !plan->preds) return 0;
    uint32_t qa[FSS_MAX_QE], qb[FSS_MAX_QE], n_qe = 0;
    if (query_edges(plan, qa, qb, &n_qe)) return 0;
    for (uint32_t k = 0; k < plan->n_pred; k++)
        if (plan->preds[k].target < 0 || (uint32_t)plan->preds[k].target >= plan->n_qv + n_qe) return 0;
    return plan_workspace(plan);
}

int match_rounds(const match_plan* plan, uint32_t* n_rounds, uint64_t* msg_words, uint32_t cap) {
    ogm::last_error().clear();
    if (!n_rounds) return fail(FSS_EINVAL, "match_rounds: n_rounds is NULL");
    if (!match_workspace_bytes(plan)) return fail(FSS_EINVAL, "match_rounds: invalid plan");
    Arena measure = Arena::measuring();
    TailPlan T;
    int rc = T.build(plan, measure);
    if (rc) return rc;
    *n_rounds = T.rounds;
    if (msg_words)
        for (uint32_t r = 0; r < T.rounds && r < cap; r++) msg_words[r] = T.msg_words(r);
    return FSS_OK;
}

int match_query(const match_plan* P, int32_t party_mask, void* stream) {
    ogm::last_error().clear();
    int rc = validate_plan(P, party_mask, "match_query");
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    Arena ws{(uint8_t*)P->d_workspace, P->workspace_bytes, 0};
    TailPlan T;
    rc = T.build(P, ws);
    if (rc) return rc;
    const RoundKeys rk = dealer_key(P->seed);
    if (party_mask == 3) {
        std::vector<EvalDesc> descs;
        plan_evals(T, 3, descs);
        for (size_t i = 0; i < descs.size(); i += kEvalInline) {
            rc = launch_eval(descs.data() + i, (uint32_t)std::min<size_t>(kEvalInline, descs.size() - i), s);
            if (rc) return rc;
        }
        std::vector<std::vector<TailOp>> levels;
        fused_levels(T, 0, levels);
        for (const auto& ops : levels) {
            rc = launch_tail_inline(ops, rk, s);
            if (rc) return rc;
        }
        return FSS_OK;
    }
    // one party, one round
    const uint32_t b = (uint32_t)party_mask - 1, r = P->round;
    if (r > T.rounds) return fail(FSS_EINVAL, "match_query: round %u of %u", r, T.rounds);
    if (r > 0 && !P->d_peer_msg) return fail(FSS_EINVAL, "match_query: round %u needs the peer's message", r);
    if (r < T.rounds && !P->d_msg) return fail(FSS_EINVAL, "match_query: round %u writes a message; d_msg is NULL", r);
    if (r == 0) {
        std::vector<EvalDesc> descs;
        plan_evals(T, party_mask, descs);
        for (size_t i = 0; i < descs.size(); i += kEvalInline) {
            rc = launch_eval(descs.data() + i, (uint32_t)std::min<size_t>(kEvalInline, descs.size() - i), s);
            if (rc) return rc;
        }
    }
    std::vector<TailOp> phase[3];
    party_round(T, b, r, P->d_peer_msg, P->d_msg, 0, phase);
    for (auto& ops : phase) {
        rc = launch_tail_inline(ops, rk, s);
        if (rc) return rc;
    }
    return FSS_OK;
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
            uint32_t counter, uint32_t* const* d_z, void* stream, const char* who, bool third_zero = false) {
    ogm::last_error().clear();
    if (nrows == 0) return FSS_OK;
    if (!d_x || !d_z || !prf_keys) return fail(FSS_EINVAL, "%s: NULL argument", who);
    RssArgs A{};
    for (int i = 0; i < 3; i++) {
        if ((!d_x[i] && !(third_zero && i == 2)) || !d_z[i] || (d_y && !d_y[i]))
            return fail(FSS_EINVAL, "%s: NULL share %d", who, i);
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

int rss_from_fss(uint64_t nrows, const uint32_t* const d_y[2], const uint64_t prf_keys[3], uint32_t counter,
                 uint32_t* const d_z[3], void* stream) {
    ogm::last_error().clear();
    if (nrows == 0) return FSS_OK;
    if (!d_y) return fail(FSS_EINVAL, "rss_from_fss: NULL y");
    const uint32_t* x[3] = {d_y[0], d_y[1], nullptr};
    return rss_run(nrows, x, nullptr, prf_keys, counter, d_z, stream, "rss_from_fss", true);
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

int rss_sec_eval_records(uint64_t ncand, uint32_t npos, const uint32_t* d_eval_a, const uint32_t* d_eval_b,
                         const uint32_t* d_share_a, const uint32_t* d_share_b, uint32_t* d_out_bits, void* stream) {
    ogm::last_error().clear();
    if (ncand == 0) return FSS_OK;
    if (npos == 0) return fail(FSS_EINVAL, "rss_sec_eval_records: no positions");
    if (ncand > 0xFFFFFFFFull) return fail(FSS_EUNSUPPORTED, "rss_sec_eval_records: more than 2^32 candidates");
    if (!d_eval_a || !d_eval_b || !d_share_a || !d_share_b || !d_out_bits)
        return fail(FSS_EINVAL, "rss_sec_eval_records: NULL buffer");
    hipLaunchKernelGGL(k_rss_eval_rec, dim3((unsigned)((ncand + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       ncand, (npos + 31) / 32, d_eval_a, d_eval_b, d_share_a, d_share_b, d_out_bits);
    return check_launch("k_rss_eval_rec");
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

int fss_set_keygen_tuning(uint32_t tile_mult) {
    ogm::last_error().clear();
    if (tile_mult < 1 || tile_mult > 8) return fail(FSS_EINVAL, "fss_set_keygen_tuning: tile_mult 1..8");
    g_tuning.keygen_tile_mult = tile_mult;
    return FSS_OK;
}

int fss_get_keygen_tuning(uint32_t* tile_mult) {
    if (tile_mult) *tile_mult = g_tuning.keygen_tile_mult;
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
    const uint32_t mult = g_tuning.keygen_tile_mult;
    const uint64_t tile_rows = (uint64_t)mult * (kBlock / 2);
    uint64_t tiles[2] = {0, 0};
    for (size_t i = 0; i < q.size(); i++) {
        uint64_t& t = tiles[i < n_range ? 0 : 1];
        q[i].tile_start = (uint32_t)t;
        t += (q[i].a.n + tile_rows - 1) / tile_rows;
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
                           dq, (uint32_t)n_range, (uint32_t)tiles[0], mult, counter);
        rc = check_launch("k_keygen_queue_range");
        if (rc) return rc;
    }
    if (tiles[1]) {
        hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s, counter);
        hipLaunchKernelGGL(k_keygen_queue_eq, dim3((unsigned)std::min(tiles[1], slots)), dim3(kBlock), 0, s,
                           dq + n_range, (uint32_t)(q.size() - n_range), (uint32_t)tiles[1], mult, counter);
        rc = check_launch("k_keygen_queue_eq");
    }
    return rc;
}

int fss_eval_batch(const fss_eval_req* reqs, uint32_t count, void* d_queue, uint64_t queue_bytes_avail,
                   void* stream) {
    ogm::last_error().clear();
    if (count == 0) return FSS_OK;
    std::vector<EvalDesc> descs;
    int rc = eval_requests(reqs, count, descs, "fss_eval_batch");
    if (rc) return rc;
    return launch_eval_queue(descs, d_queue, queue_bytes_avail, (hipStream_t)stream);
}

int fss_eval_batch_noalloc(const fss_eval_req* reqs, uint32_t count, void* stream) {
    ogm::last_error().clear();
    const char* who = "fss_eval_batch_noalloc";
    if (count == 0) return FSS_OK;
    if (count > FSS_NOALLOC_EVAL_MAX)
        return fail(FSS_EINVAL, "%s: %u requests, at most %d", who, count, FSS_NOALLOC_EVAL_MAX);
    if (!reqs) return fail(FSS_EINVAL, "%s: reqs is NULL", who);
    // Host side without allocation: the queue order (as fss_eval_batch's) is a
    // stable bottom-up merge of 16-bit request indices on the stack, and the
    // descriptors go out as kernel arguments, one chunk at a time.
    static_assert(FSS_NOALLOC_EVAL_MAX <= 65536, "indices are 16-bit");
    uint16_t idx[2][FSS_NOALLOC_EVAL_MAX];
    uint32_t m = 0;
    for (uint32_t i = 0; i < count; i++) {
        EvalDesc d;
        const int rc = eval_request(reqs[i], i, who, &d);
        if (rc) return rc;
        if (d.n) idx[0][m++] = (uint16_t)i;
    }
    if (m == 0) return FSS_OK;
    auto before = [&](uint16_t a, uint16_t b) {
        return eval_before((uint32_t)reqs[a].keys->kind, reqs[a].keys->n, (uint32_t)reqs[b].keys->kind,
                           reqs[b].keys->n);
    };
    int cur = 0;
    for (uint32_t w = 1; w < m; w *= 2, cur ^= 1) {
        const uint16_t* src = idx[cur];
        uint16_t* dst = idx[cur ^ 1];
        for (uint32_t lo = 0; lo < m; lo += 2 * w) {
            const uint32_t mid = std::min(lo + w, m), hi = std::min(lo + 2 * w, m);
            uint32_t a = lo, b = mid, o = lo;
            while (a < mid && b < hi) dst[o++] = before(src[b], src[a]) ? src[b++] : src[a++];
            while (a < mid) dst[o++] = src[a++];
            while (b < hi) dst[o++] = src[b++];
        }
    }
    const uint16_t* order = idx[cur];
    const uint64_t tile_rows = (uint64_t)kBlock * g_tuning.rows_per_thread;
    uint64_t tiles = 0;
    for (uint32_t j = 0; j < m; j++) tiles += (reqs[order[j]].keys->n + tile_rows - 1) / tile_rows;
    if (tiles > 0xFFFFFFF0ull) return fail(FSS_EUNSUPPORTED, "%s: too many tiles", who);
    void* d_scratch = nullptr;
    int rc = scratch_ptr(&d_scratch, who);
    if (rc) return rc;
    uint32_t* counter = (uint32_t*)d_scratch;
    QEval* dq = (QEval*)((uint8_t*)d_scratch + kQueueHeader);
    hipStream_t s = (hipStream_t)stream;
    constexpr uint32_t kPerChunk = kArgChunk / sizeof(QEval);
    static_assert(sizeof(QEval) % 4 == 0, "descriptors are whole words");
    uint64_t tile = 0;
    for (uint32_t first = 0; first < m; first += kPerChunk) {
        const uint32_t nq = std::min(kPerChunk, m - first);
        ArgChunk c{};
        for (uint32_t j = 0; j < nq; j++) {
            QEval e{};
            eval_request(reqs[order[first + j]], order[first + j], who, &e.d);   // checked above
            e.d.block_start = (uint32_t)tile;
            tile += (e.d.n + tile_rows - 1) / tile_rows;
            memcpy((uint8_t*)c.w + (size_t)j * sizeof(QEval), &e, sizeof(QEval));
        }
        hipLaunchKernelGGL(k_put_words, dim3(1), dim3(256), 0, s, (uint32_t*)(dq + first),
                           (uint32_t)(nq * sizeof(QEval) / 4), c);
        rc = check_launch("k_put_words");
        if (rc) return rc;
    }
    return launch_eval_kernel(dq, m, tiles, counter, s);
}

int match_query_batch(const match_plan* plans, uint32_t count, int32_t party_mask, void* d_queue,
                      uint64_t queue_bytes_avail, void* stream) {
    ogm::last_error().clear();
    if (count == 0) return FSS_OK;
    if (!plans) return fail(FSS_EINVAL, "match_query_batch: plans is NULL");
    for (uint32_t i = 0; i < count; i++) {
        int rc = validate_plan(&plans[i], party_mask, "match_query_batch");
        if (rc) return rc;
        if (party_mask != 3) {
            const match_plan& P = plans[i];
            uint32_t R = 0;
            rc = match_rounds(&P, &R, nullptr, 0);
            if (rc) return rc;
            if (P.round > R) return fail(FSS_EINVAL, "match_query_batch: plan %u round %u of %u", i, P.round, R);
            if (P.round > 0 && !P.d_peer_msg) return fail(FSS_EINVAL, "match_query_batch: plan %u needs the peer's message", i);
            if (P.round < R && !P.d_msg) return fail(FSS_EINVAL, "match_query_batch: plan %u d_msg is NULL", i);
        }
    }
    hipStream_t s = (hipStream_t)stream;
    std::vector<TailPlan> tails(count);
    std::vector<EvalDesc> descs;
    for (uint32_t i = 0; i < count; i++) {
        const match_plan* P = &plans[i];
        Arena ws{(uint8_t*)P->d_workspace, P->workspace_bytes, 0};
        int rc = tails[i].build(P, ws);
        if (rc) return rc;
        if (party_mask == 3 || P->round == 0) plan_evals(tails[i], party_mask, descs);
    }
    int rc = launch_eval_queue(descs, d_queue, queue_bytes_avail, s);
    if (rc) return rc;
    // the tail: ops of every plan merged per launch, with one key schedule per plan
    std::vector<std::vector<TailOp>> levels;
    for (uint32_t i = 0; i < count; i++) {
        if (party_mask == 3) {
            fused_levels(tails[i], i, levels);
        } else {
            std::vector<TailOp> phase[3];
            const match_plan& P = plans[i];
            party_round(tails[i], (uint32_t)party_mask - 1, P.round, P.d_peer_msg, P.d_msg, i, phase);
            if (levels.size() < 3) levels.resize(3);
            for (int k = 0; k < 3; k++) levels[k].insert(levels[k].end(), phase[k].begin(), phase[k].end());
        }
    }
    return launch_tail_queue(plans, count, levels, d_queue, queue_bytes_avail, s);
}

uint64_t match_batch_queue_bytes(const match_plan* plans, uint32_t count) {
    if (!plans) return 0;
    uint64_t nevals = 0, nops = 0;
    for (uint32_t i = 0; i < count; i++) {
        if (!match_workspace_bytes(&plans[i])) return 0;
        Arena measure = Arena::measuring();
        TailPlan T;
        if (T.build(&plans[i], measure)) return 0;
        std::vector<EvalDesc> d;
        plan_evals(T, 3, d);
        nevals += d.size();
        // every AND, two gathers per hop, one pair op per vertex and one copy per output, at most,
        // in any launch
        nops += T.ands.size() + 3 * (uint64_t)T.n_qe + T.n_qv + 2;
    }
    return std::max(queue_bytes(nevals), tail_queue_bytes(count, nops));
}

}  // extern "C"
