// shuffle.hip -- three-party secret-shared shuffle (Alg. 5) and secure fetching
// of matched records (Alg. 4, Cases I and II), all three servers simulated.
//
// Tables are row-major: record r of a W-word table at words [r*W, r*W + W).
// Each pair of servers derives from its seed, with the counter-mode generator
// (domain 6), its permutations (stable sort of one 64-bit key per row) and
// mask tables (one AES block per four words); applying a permutation is the
// row gather out[i] = in[perm[i]].  The servers' steps of Alg. 5 are grouped
// by the pair permutation they apply: one launch per round (pi12, pi31, pi23)
// forms every table that pair permutes in that round, with the pair's mask
// computed where it is XORed, so that each mask word is made once, no mask
// table is stored, and the AES overlaps with the rounds' random-row traffic.
// Rounds pi12 and pi31 run as scatters through the inverse permutation
// (in-order reads, random writes: a random 64-byte read costs a whole
// 128-byte line, a random write only its bytes); round pi23, whose outputs
// are the result shares, is a gather.  The messages X1 and Y1 are stored
// between rounds; C1 and C2 meet in R3 = C1 ^ C2 as they are formed.

#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <stdint.h>

#include "../../include/oblivgm_fss.h"
#include "aes_gfx950.hpp"
#include "common.hpp"

using namespace ogm;

namespace {

constexpr int kBlock = 1024;
__constant__ AesTables g_tab = kTables;

enum { kT12 = 1, kR2 = 2, kT23 = 3, kT31 = 4, kR1 = 5 };
enum { kP12 = 0, kP23 = 1, kP31 = 2 };

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }   // NULL counts as aligned

// Number of workgroups for a grid-stride AES kernel: enough to fill every CU
// twice, never more than the work needs.  A workgroup fills its 64 KiB LDS
// tables once and then loops, so the fill is spread over many blocks.
unsigned aes_grid(uint64_t items) {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    const uint64_t need = (items + kBlock - 1) / kBlock;
    const uint64_t cap = 2ull * (uint64_t)cus;
    return (unsigned)(need < 1 ? 1 : (need < cap ? need : cap));
}

// Sort keys of permutation p: row r -> words 0-1 of block (6, 16 + p, 0, 0, r).
// The key is stored rotated left by hb bits, so that its top hb bits (the
// row's run id) sit in bits 0 .. hb-1, the range the radix pass sorts, and
// the whole key travels with it; the row number goes beside it.
__global__ __launch_bounds__(kBlock) void k_perm_keys(RoundKeys rk, uint32_t p, uint64_t nrows, uint32_t hb,
                                                     uint64_t* __restrict__ keys, uint32_t* __restrict__ idx) {
    __shared__ uint32_t tab[kLdsTableWords];
    lds_table_fill(tab, g_tab.t0);
    __syncthreads();
    const LaneOff lo = lane_offset();
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t r = (uint64_t)blockIdx.x * kBlock + threadIdx.x; r < nrows; r += stride) {
        const uint4 b = aes128_encrypt(make_uint4(6u | ((16u + p) << 16), 0u, 0u, (uint32_t)r), ArgKey{rk}, tab, lo);
        const uint64_t key = (uint64_t)b.x | ((uint64_t)b.y << 32);
        keys[r] = hb ? (key << hb) | (key >> (64 - hb)) : key;
        idx[r] = (uint32_t)r;
    }
}

// The permutation is the stable argsort of the 64-bit keys.  It is made in two
// steps: a stable radix sort of the rows by run id (the top hb key bits, hb =
// ceil(log2 n) - 6, so that a run holds 64 rows on average), then each run
// ordered by its full keys.  Inside a run the radix sort has kept the rows in
// their original order, so "equal key, earlier position" is "equal key,
// smaller row" and the result is the full stable argsort.

// starts[b] = first position of run b in the sorted keys (lower bound of run
// id b by binary search), b = 0 .. 2^hb; starts[2^hb] = n.  A lower bound is
// non-decreasing in b over any array, so the runs always partition [0, n):
// the ranking below stays in bounds whatever the sort returned.
__global__ void k_run_starts(uint64_t n, uint32_t hb, const uint64_t* __restrict__ keys,
                             uint32_t* __restrict__ starts) {
    const uint32_t nruns = 1u << hb;
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nruns) return;
    const uint32_t id_mask = nruns - 1u;
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (((uint32_t)keys[mid] & id_mask) < b)
            lo = mid + 1;
        else
            hi = mid;
    }
    starts[b] = (uint32_t)lo;
}

// Broadcast of lane t's 64-bit value to the whole wavefront (t uniform).
__device__ __forceinline__ uint64_t lane_value(uint64_t v, uint32_t t) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, (int)t);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)t);
    return ((uint64_t)hi << 32) | lo;
}

// One wavefront per run: row e of the run goes to position start + rank(e),
// rank = number of rows of the run with a smaller key, or an equal key at an
// earlier position.  The run's keys are taken 64 at a time into the lanes and
// broadcast with readlane, so any run length is ordered exactly (the cost
// grows as the square of the length; the runs of uniform keys are short).
// All keys of a run share their id bits (bits 0 .. hb-1 of the rotated key);
// when the run has at most 2^hb rows those bits are replaced by the row's
// position in the run, which makes every key of the run distinct and ordered
// as (key, position), so one compare per row does.
// With `inverse` the kernel writes the inverse permutation instead:
// out[row] = its position.
__global__ __launch_bounds__(256) void k_rank_runs(uint32_t hb, uint32_t inverse, const uint32_t* __restrict__ starts,
                                                   const uint64_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ rows, uint32_t* __restrict__ perm) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t nruns = 1u << hb;
    const uint64_t id_mask = (uint64_t)(nruns - 1u);
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    // the run number is the same on every lane of the wavefront; saying so
    // keeps the run bounds and loop counters in scalar registers
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (uint32_t b = blockIdx.x * (blockDim.x >> 6) + wave; b < nruns; b += waves) {
        const uint32_t s = starts[b], m = starts[b + 1] - s;
        const bool distinct = m <= nruns;
        for (uint32_t c0 = 0; c0 < m; c0 += 64) {
            const uint32_t e = c0 + lane;
            const bool has = e < m;
            uint64_t ke = has ? keys[s + e] : 0ull;
            if (distinct) ke = (ke & ~id_mask) | e;
            uint32_t rank = 0;
            for (uint32_t j0 = 0; j0 < m; j0 += 64) {
                uint64_t kj = j0 + lane < m ? keys[s + j0 + lane] : 0ull;
                const uint32_t cnt = (uint32_t)__builtin_amdgcn_readfirstlane((int)(m - j0 < 64 ? m - j0 : 64));
                if (distinct) {
                    kj = (kj & ~id_mask) | (j0 + lane);
                    for (uint32_t t = 0; t < cnt; t++) rank += (uint32_t)(lane_value(kj, t) < ke);
                } else {
                    // no short-circuit: three compares and no branch per row
                    for (uint32_t t = 0; t < cnt; t++) {
                        const uint64_t kt = lane_value(kj, t);
                        rank += (uint32_t)(kt < ke) | ((uint32_t)(kt == ke) & (uint32_t)(j0 + t < e));
                    }
                }
            }
            if (has) {
                if (inverse)
                    perm[rows[s + e]] = s + rank;
                else
                    perm[s + rank] = rows[s + e];
            }
        }
    }
}

// Mask of one unit of table `table` under the pair key rk: with VEC the
// 16-byte unit u is block u of the table (the record width is a multiple of 4
// words, so units and blocks coincide); else word u is word (u mod 4) of
// block u div 4.
template <bool VEC>
__device__ __forceinline__ uint4 mask_unit(const RoundKeys& rk, uint32_t table, uint32_t nwords, uint64_t u,
                                           const uint32_t* tab, LaneOff lo) {
    const uint32_t blk = (uint32_t)(VEC ? u : u >> 2);
    const uint4 b = aes128_encrypt(make_uint4(6u | (table << 16), nwords, 0u, blk), ArgKey{rk}, tab, lo);
    if (VEC) return b;
    const uint32_t q = (uint32_t)u & 3u;
    return make_uint4(q == 0 ? b.x : q == 1 ? b.y : q == 2 ? b.z : b.w, 0u, 0u, 0u);
}

// An empty asm statement that the value passes through: its block is complete
// here, in registers, and the next block's work does not move across this
// point (two mask blocks side by side would need more than 64 VGPRs, which
// would leave room for one workgroup per CU instead of two).  It also keeps
// the compiler from cancelling a mask that two messages share (C1 and C2).
__device__ __forceinline__ void pin(uint4& v) {
    asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w) : : "memory");
}

template <bool VEC>
__device__ __forceinline__ uint4 load_unit(const uint32_t* __restrict__ t, uint64_t u) {
    if (VEC) return ((const uint4*)t)[u];
    return make_uint4(t[u], 0u, 0u, 0u);
}

template <bool VEC>
__device__ __forceinline__ void store_unit(uint32_t* __restrict__ t, uint64_t u, uint4 v) {
    if (VEC)
        ((uint4*)t)[u] = v;
    else
        t[u] = v.x;
}

// One round of Alg. 5 is the permutation of one pair of servers applied, with
// that pair's mask T, to every table the pair permutes in that round.  The
// kernels compute the mask words where they XOR them (a mask word is a
// counter-mode block of its table), so no mask table is stored and the AES
// overlaps with the rounds' random-row traffic.  Units are 16-byte quarters
// of a record with VEC (width a multiple of 4 words, every table 16-byte
// aligned), else words.
enum { kRound12 = 0, kRound31 = 1 };

// Rounds pi12 and pi31 as scatters: source row j of the permuted tables goes
// to output row inv[j] (inv the inverse permutation), so the tables are read
// in order and written at random rows; the pair mask T is indexed by the
// source row and R by the output row:
//   kRound12: o0[inv[j]] = (g0 ^ g1 ^ T12)[j], o1[inv[j]] = (g2 ^ T12)[j], rout = R2
//             (CS1's pi12(D1 ^ D2 ^ T12) and CS2's Y1 = pi12(D3 ^ T12))
//   kRound31: o0[inv[j]] = (g0 ^ T31)[j],      o1[inv[j]] = (g1 ^ T31)[j], rout = R1
//             (CS1's X1 and CS3's pi31(Y1 ^ T31))
template <int ROUND, bool VEC>
__global__ __launch_bounds__(kBlock) void k_shuffle_scatter(uint64_t nrows, uint32_t nwords, RoundKeys rk,
                                                          uint32_t t_mask, uint32_t r_mask,
                                                          const uint32_t* __restrict__ inv,
                                                          const uint32_t* __restrict__ g0,
                                                          const uint32_t* __restrict__ g1,
                                                          const uint32_t* __restrict__ g2, uint32_t* __restrict__ o0,
                                                          uint32_t* __restrict__ o1, uint32_t* __restrict__ rout) {
    __shared__ uint32_t tab[kLdsTableWords];
    lds_table_fill(tab, g_tab.t0);
    __syncthreads();
    const LaneOff lo = lane_offset();
    const uint32_t q = VEC ? nwords >> 2 : nwords;       // units per record
    const uint64_t total = nrows * q;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x; k < total; k += stride) {
        const uint32_t j = (uint32_t)(k / q), w = (uint32_t)(k - (uint64_t)j * q);
        const uint64_t d = (uint64_t)inv[j] * q + w;
        const uint4 a = load_unit<VEC>(g0, k), b = load_unit<VEC>(g1, k);
        uint4 t = mask_unit<VEC>(rk, t_mask, nwords, k, tab, lo);
        pin(t);
        if (ROUND == kRound12) {
            const uint4 c = load_unit<VEC>(g2, k);
            store_unit<VEC>(o0, d, xor4(xor4(a, b), t));
            store_unit<VEC>(o1, d, xor4(c, t));
        } else {
            store_unit<VEC>(o0, d, xor4(a, t));
            store_unit<VEC>(o1, d, xor4(b, t));
        }
        uint4 r = mask_unit<VEC>(rk, r_mask, nwords, k, tab, lo);
        pin(r);
        store_unit<VEC>(rout, k, r);
    }
}

// Round pi23 as a gather (its outputs are the result shares, written in
// order): with p = perm[i],
//   out[i] = C1 ^ C2, C1 = (g0 ^ T23)[p] ^ s0[i], C2 = (g1 ^ T23)[p] ^ s1[i]
// (CS2's C1 = pi23(X1 ^ T23) ^ R2, CS3's C2 = pi23(pi31(Y1 ^ T31) ^ T23) ^ R1
// and CS2's R3 = C1 ^ C2; with the servers simulated together C1 and C2 are
// not stored).
template <bool VEC>
__global__ __launch_bounds__(kBlock) void k_shuffle_final(uint64_t nrows, uint32_t nwords, RoundKeys rk,
                                                        uint32_t t_mask, const uint32_t* __restrict__ perm,
                                                        const uint32_t* __restrict__ g0,
                                                        const uint32_t* __restrict__ g1,
                                                        const uint32_t* __restrict__ s0,
                                                        const uint32_t* __restrict__ s1, uint32_t* __restrict__ out) {
    __shared__ uint32_t tab[kLdsTableWords];
    lds_table_fill(tab, g_tab.t0);
    __syncthreads();
    const LaneOff lo = lane_offset();
    const uint32_t q = VEC ? nwords >> 2 : nwords;       // units per record
    const uint64_t total = nrows * q;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x; k < total; k += stride) {
        const uint32_t i = (uint32_t)(k / q), w = (uint32_t)(k - (uint64_t)i * q);
        const uint64_t u = (uint64_t)perm[i] * q + w;
        const uint4 a = load_unit<VEC>(g0, u), b = load_unit<VEC>(g1, u);
        uint4 t = mask_unit<VEC>(rk, t_mask, nwords, u, tab, lo);
        pin(t);
        uint4 c1 = xor4(xor4(a, t), load_unit<VEC>(s0, k));
        pin(c1);
        const uint4 c2 = xor4(xor4(b, t), load_unit<VEC>(s1, k));
        store_unit<VEC>(out, k, xor4(c1, c2));
    }
}

// Case I: XOR over candidates of (r_i & m_i) ^ (r_j & m_i) ^ (r_i & m_j), the
// three-out-of-three products of record shares with the predicate-bit
// shares, j = i + 1.  The block walks its candidates record by record with
// the words of a tile of each record on consecutive threads (coalesced), each
// thread keeping one word's partial; the partials of equal words meet in LDS
// and one atomicXor per word and share goes to the zeroed output (XOR is
// order-free, so the result does not depend on the order).
constexpr int kFetchBlock = 256;

__global__ __launch_bounds__(kFetchBlock) void k_fetch_unique(
    uint64_t ncand, uint32_t nwords, const uint32_t* __restrict__ x0, const uint32_t* __restrict__ x1,
    const uint32_t* __restrict__ x2, const uint32_t* __restrict__ r0, const uint32_t* __restrict__ r1,
    const uint32_t* __restrict__ r2, uint32_t* __restrict__ out0, uint32_t* __restrict__ out1,
    uint32_t* __restrict__ out2) {
    __shared__ uint32_t part[3][kFetchBlock];
    const uint32_t* xs[3] = {x0, x1, x2};
    const uint32_t* rs[3] = {r0, r1, r2};
    uint32_t* outs[3] = {out0, out1, out2};
    // this block's candidates
    const uint64_t per = (ncand + gridDim.x - 1) / gridDim.x;
    const uint64_t c0 = (uint64_t)blockIdx.x * per;
    const uint64_t c1 = c0 + per < ncand ? c0 + per : ncand;
    const uint32_t t = threadIdx.x;
    for (uint32_t w0 = 0; w0 < nwords; w0 += kFetchBlock) {
        const uint32_t tw = nwords - w0 < kFetchBlock ? nwords - w0 : kFetchBlock;   // words in this tile
        const uint32_t lanes = kFetchBlock / tw;                                       // candidates per pass
        const uint32_t w = t % tw, g = t / tw;
        uint32_t acc[3] = {0, 0, 0};
        if (g < lanes) {
            for (uint64_t c = c0 + g; c < c1; c += lanes) {
                uint32_t m[3], rv[3];
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    m[i] = 0u - ((xs[i][c >> 5] >> (c & 31)) & 1u);
                    rv[i] = rs[i][c * nwords + w0 + w];
                }
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    const int j = (i + 1) % 3;
                    acc[i] ^= (rv[i] & m[i]) ^ (rv[j] & m[i]) ^ (rv[i] & m[j]);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 3; i++) part[i][t] = acc[i];
        __syncthreads();
        if (t < tw) {
#pragma unroll
            for (int i = 0; i < 3; i++) {
                uint32_t v = 0;
                for (uint32_t k = 0; k < lanes; k++) v ^= part[i][k * tw + t];
                if (v) atomicXor(&outs[i][w0 + t], v);
            }
        }
        __syncthreads();
    }
}

__global__ void k_zero(uint64_t n, uint32_t* __restrict__ p) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) p[k] = 0u;
}

// Case II: flag of shuffled record i = bit 0 of word 0 of R1 ^ R2 ^ R3 (the opened x).
__global__ void k_open_flags(uint64_t nrows, uint32_t nwords, const uint32_t* __restrict__ a,
                             const uint32_t* __restrict__ b, const uint32_t* __restrict__ c,
                             uint32_t* __restrict__ flags) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nrows) flags[i] = (a[i * nwords] ^ b[i * nwords] ^ c[i * nwords]) & 1u;
}

// secAccess filter: flag of shuffled record i = parity of all bits of R1 ^ R2 ^ R3
// (1 for a one-hot ID, 0 for a dummy all-zero ID).  With vec (width a
// multiple of 4 words, tables 16-byte aligned) the loads are 16 bytes.
__global__ void k_open_parity(uint64_t nrows, uint32_t nwords, uint32_t vec, const uint32_t* __restrict__ a,
                              const uint32_t* __restrict__ b, const uint32_t* __restrict__ c,
                              uint32_t* __restrict__ flags) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    uint32_t acc = 0;
    if (vec) {
        const uint64_t base = i * (nwords >> 2);
        for (uint32_t w = 0; w < (nwords >> 2); w++) {
            const uint4 v = xor4(xor4(((const uint4*)a)[base + w], ((const uint4*)b)[base + w]),
                                 ((const uint4*)c)[base + w]);
            acc ^= v.x ^ v.y ^ v.z ^ v.w;
        }
    } else {
        for (uint32_t w = 0; w < nwords; w++) acc ^= a[i * nwords + w] ^ b[i * nwords + w] ^ c[i * nwords + w];
    }
    flags[i] = __builtin_popcount(acc) & 1u;
}

// Copy the kept records (words first..W-1) of the three share tables to their
// slots: one thread per (record, word) so that reads and writes are coalesced.
__global__ void k_compact(uint64_t nrows, uint32_t nwords, uint32_t first, const uint32_t* __restrict__ flags,
                          const uint32_t* __restrict__ pos, const uint32_t* __restrict__ s0,
                          const uint32_t* __restrict__ s1, const uint32_t* __restrict__ s2,
                          uint32_t* __restrict__ o0, uint32_t* __restrict__ o1, uint32_t* __restrict__ o2,
                          uint32_t* __restrict__ rows_out) {
    const uint32_t rw = nwords - first;
    const uint64_t total = nrows * rw;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += stride) {
        const uint32_t i = (uint32_t)(k / rw), w = (uint32_t)(k - (uint64_t)i * rw);
        if (!flags[i]) continue;
        const uint64_t d = pos[i];
        const uint64_t src = (uint64_t)i * nwords + first + w;
        o0[d * rw + w] = s0[src];
        o1[d * rw + w] = s1[src];
        o2[d * rw + w] = s2[src];
        if (w == 0) rows_out[d] = i;
    }
}

// count of kept records = last exclusive prefix + last flag
__global__ void k_count(uint64_t n, const uint32_t* __restrict__ flags, const uint32_t* __restrict__ pos,
                        uint32_t* __restrict__ count) {
    if (threadIdx.x == 0) *count = pos[n - 1] + flags[n - 1];
}

unsigned grid_of(uint64_t n, unsigned block) {
    uint64_t g = (n + block - 1) / block;
    if (g == 0) g = 1;
    if (g > 16384) g = 16384;
    return (unsigned)g;
}

struct Carve {
    uint8_t* p;
    uint64_t left;
    bool ok = true;
    template <class T>
    T* take(uint64_t count) {
        const uint64_t bytes = (count * sizeof(T) + 255) & ~255ull;
        if (bytes > left) { ok = false; return nullptr; }
        T* r = (T*)p;
        p += bytes;
        left -= bytes;
        return r;
    }
};

// Top key bits the radix pass sorts: ceil(log2 n) - 6, at least 0.
// Run-id bits the radix pass sorts: ceil(log2 n) - 6, at least 0 (at most 25
// for n < 2^31).  The ids are the low hb bits of the rotated keys, so the
// sort asks for bits [0, hb): a range that ends at the key type's top bit
// makes rocPRIM's merge-sort path (1 Ki - 1 Mi items) build its comparison
// mask with a full-width shift, which compares the wrong bits.
uint32_t run_bits(uint64_t nrows) {
    uint32_t lg = 0;
    while ((1ull << lg) < nrows) lg++;
    return lg > 6 ? lg - 6 : 0;
}

size_t sort_temp_bytes(uint64_t nrows) {
    const uint32_t hb = run_bits(nrows);
    if (!hb) return 0;
    size_t b = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, b, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                             (const uint32_t*)nullptr, (uint32_t*)nullptr, (int)nrows, 0, (int)hb);
    return b;
}

uint64_t shuffle_ws(uint64_t nrows, uint32_t nwords) {
    auto r = [](uint64_t b) { return (b + 255) & ~255ull; };
    const uint64_t tw = nrows * nwords * 4;
    // pi12(D1^D2^T12), Y1, X1, pi31(Y1^T31); three permutations; rotated keys
    // in and out; row numbers in and out; run starts; the sort's temporary
    // storage
    return 4 * r(tw) + 3 * r(nrows * 4) + 2 * r(nrows * 8) + 2 * r(nrows * 4) + r(((1ull << run_bits(nrows)) + 1) * 4) +
           r(sort_temp_bytes(nrows)) + 4096;
}

// perm = stable argsort of the pair seed's row keys (or its inverse): radix
// sort by run id, then each run ordered by rank.
struct PermScratch {
    uint64_t* keys;
    uint64_t* keys_sorted;
    uint32_t* idx;
    uint32_t* idx_sorted;
    uint32_t* starts;
    void* temp;
    size_t temp_bytes;
};

int make_perm(const RoundKeys& rk, uint32_t p, uint64_t nrows, const PermScratch& w, bool inverse, uint32_t* perm,
              hipStream_t s) {
    const uint32_t hb = run_bits(nrows);
    hipLaunchKernelGGL(k_perm_keys, dim3(aes_grid(nrows)), dim3(kBlock), 0, s, rk, p, nrows, hb, w.keys, w.idx);
    int rc = check_launch("k_perm_keys");
    if (rc) return rc;
    const uint64_t* keys = w.keys;
    const uint32_t* rows = w.idx;
    if (hb) {          // with no run-id bits there is one run, already in row order
        size_t temp_bytes = w.temp_bytes;
        if (hipcub::DeviceRadixSort::SortPairs(w.temp, temp_bytes, w.keys, w.keys_sorted, w.idx, w.idx_sorted,
                                               (int)nrows, 0, (int)hb, s) != hipSuccess)
            return fail(FSS_EDEVICE, "rss_shuffle: radix sort failed");
        keys = w.keys_sorted;
        rows = w.idx_sorted;
    }
    const uint64_t nruns = 1ull << hb;
    hipLaunchKernelGGL(k_run_starts, dim3((unsigned)((nruns + 1 + 255) / 256)), dim3(256), 0, s, nrows, hb, keys,
                       w.starts);
    rc = check_launch("k_run_starts");
    if (rc) return rc;
    hipLaunchKernelGGL(k_rank_runs, dim3(grid_of(nruns * 64, 256)), dim3(256), 0, s, hb, (uint32_t)inverse, w.starts,
                       keys, rows, perm);
    return check_launch("k_rank_runs");
}

// Round pi23 (k_shuffle_final); the 16-byte path when the width is a multiple
// of 4 words and every table is 16-byte aligned.
int shuffle_final(uint64_t nrows, uint32_t nwords, const RoundKeys& rk, uint32_t t_mask, const uint32_t* perm,
                  const uint32_t* g0, const uint32_t* g1, const uint32_t* s0, const uint32_t* s1, uint32_t* out,
                  hipStream_t s) {
    const bool vec = (nwords & 3u) == 0 && aligned16(g0) && aligned16(g1) && aligned16(s0) && aligned16(s1) &&
                     aligned16(out);
    const uint64_t units = vec ? nrows * (nwords >> 2) : nrows * nwords;
    if (vec)
        hipLaunchKernelGGL(k_shuffle_final<true>, dim3(aes_grid(units)), dim3(kBlock), 0, s, nrows, nwords, rk, t_mask,
                           perm, g0, g1, s0, s1, out);
    else
        hipLaunchKernelGGL(k_shuffle_final<false>, dim3(aes_grid(units)), dim3(kBlock), 0, s, nrows, nwords, rk, t_mask,
                           perm, g0, g1, s0, s1, out);
    return check_launch("k_shuffle_final");
}

// Rounds pi12 / pi31 as scatters (k_shuffle_scatter), with the same 16-byte
// path condition.
template <int ROUND>
int shuffle_scatter(uint64_t nrows, uint32_t nwords, const RoundKeys& rk, uint32_t t_mask, uint32_t r_mask,
                    const uint32_t* inv, const uint32_t* g0, const uint32_t* g1, const uint32_t* g2, uint32_t* o0,
                    uint32_t* o1, uint32_t* rout, hipStream_t s) {
    const bool vec = (nwords & 3u) == 0 && aligned16(g0) && aligned16(g1) && aligned16(g2) && aligned16(o0) &&
                     aligned16(o1) && aligned16(rout);
    const uint64_t units = vec ? nrows * (nwords >> 2) : nrows * nwords;
    if (vec)
        hipLaunchKernelGGL((k_shuffle_scatter<ROUND, true>), dim3(aes_grid(units)), dim3(kBlock), 0, s, nrows, nwords,
                           rk, t_mask, r_mask, inv, g0, g1, g2, o0, o1, rout);
    else
        hipLaunchKernelGGL((k_shuffle_scatter<ROUND, false>), dim3(aes_grid(units)), dim3(kBlock), 0, s, nrows, nwords,
                           rk, t_mask, r_mask, inv, g0, g1, g2, o0, o1, rout);
    return check_launch("k_shuffle_scatter");
}

// Alg. 5 with all three servers simulated; out[0..2] = R1, R2, R3.  The
// servers' steps are grouped by the pair permutation they apply, one launch
// per round: pi12 (CS1, CS2), pi31 (CS1, CS3), pi23 (CS2, CS3).
int run_shuffle(uint64_t nrows, uint32_t nwords, const uint32_t* const d[3], const uint64_t seeds[3],
                uint32_t* const out[3], Carve& ws, hipStream_t s) {
    const uint64_t tw = nrows * nwords;
    const RoundKeys k12 = seed_key(seeds[0]), k23 = seed_key(seeds[1]), k31 = seed_key(seeds[2]);
    uint32_t* z = ws.take<uint32_t>(tw);       // CS1: pi12(D1 ^ D2 ^ T12)
    uint32_t* y1 = ws.take<uint32_t>(tw);      // CS2 -> CS3: Y1
    uint32_t* x1 = ws.take<uint32_t>(tw);      // CS1 -> CS2: X1
    uint32_t* v = ws.take<uint32_t>(tw);       // CS3: pi31(Y1 ^ T31)
    uint32_t* p12 = ws.take<uint32_t>(nrows);
    uint32_t* p23 = ws.take<uint32_t>(nrows);
    uint32_t* p31 = ws.take<uint32_t>(nrows);
    PermScratch pw;
    pw.keys = ws.take<uint64_t>(nrows);
    pw.keys_sorted = ws.take<uint64_t>(nrows);
    pw.idx = ws.take<uint32_t>(nrows);
    pw.idx_sorted = ws.take<uint32_t>(nrows);
    pw.starts = ws.take<uint32_t>((1ull << run_bits(nrows)) + 1);
    pw.temp_bytes = sort_temp_bytes(nrows);
    pw.temp = ws.take<uint8_t>(pw.temp_bytes);
    if (!ws.ok) return fail(FSS_ENOMEM, "rss_shuffle: workspace too small");
    // pair seeds: s12 -> pi12, T12, R2; s23 -> pi23, T23; s31 -> pi31, T31, R1.
    // pi12 and pi31 are applied as scatters (their inverses), pi23 as a gather
    int rc = make_perm(k12, kP12, nrows, pw, true, p12, s);
    if (!rc) rc = make_perm(k23, kP23, nrows, pw, false, p23, s);
    if (!rc) rc = make_perm(k31, kP31, nrows, pw, true, p31, s);
    // pi12: CS1 forms pi12(D1 ^ D2 ^ T12), CS2 forms Y1 = pi12(D3 ^ T12); R2 drawn
    if (!rc)
        rc = shuffle_scatter<kRound12>(nrows, nwords, k12, kT12, kR2, p12, d[0], d[1], d[2], z, y1, out[1], s);
    // pi31: CS1 forms X1 = pi31(pi12(...) ^ T31), CS3 forms pi31(Y1 ^ T31); R1 drawn
    if (!rc)
        rc = shuffle_scatter<kRound31>(nrows, nwords, k31, kT31, kR1, p31, z, y1, nullptr, x1, v, out[0], s);
    // pi23: CS2 forms C1 = pi23(X1 ^ T23) ^ R2, CS3 forms C2 = pi23(pi31(Y1 ^ T31) ^ T23) ^ R1,
    // and R3 = C1 ^ C2 (with the servers simulated together, C1 and C2 are not stored)
    if (!rc) rc = shuffle_final(nrows, nwords, k23, kT23, p23, x1, v, out[1], out[0], out[2], s);
    return rc;
}

}  // namespace

extern "C" {

uint64_t rss_shuffle_workspace_bytes(uint64_t nrows, uint32_t nwords) {
    if (nrows == 0 || nwords == 0) return 0;
    return shuffle_ws(nrows, nwords);
}

int rss_shuffle(uint64_t nrows, uint32_t nwords, const uint32_t* const d_in[3], const uint64_t seeds[3],
                uint32_t* const d_out[3], void* d_work, uint64_t work_bytes, void* stream) {
    last_error().clear();
    if (nrows == 0 || nwords == 0) return FSS_OK;
    if (nrows > 0x7FFFFFFFull) return fail(FSS_EUNSUPPORTED, "rss_shuffle: more than 2^31 rows");
    if (!d_in || !d_out || !seeds) return fail(FSS_EINVAL, "rss_shuffle: NULL argument");
    for (int i = 0; i < 3; i++)
        if (!d_in[i] || !d_out[i]) return fail(FSS_EINVAL, "rss_shuffle: NULL share %d", i);
    if (!d_work || work_bytes < shuffle_ws(nrows, nwords))
        return fail(FSS_ENOMEM, "rss_shuffle: workspace needs %llu bytes",
                    (unsigned long long)shuffle_ws(nrows, nwords));
    Carve ws{(uint8_t*)d_work, work_bytes};
    return run_shuffle(nrows, nwords, d_in, seeds, d_out, ws, (hipStream_t)stream);
}

int rss_fetch_unique(uint64_t ncand, uint32_t nwords, const uint32_t* const d_x[3], const uint32_t* const d_rows[3],
                     uint32_t* const d_out[3], void* stream) {
    last_error().clear();
    if (nwords == 0) return FSS_OK;
    if (nwords > 65535) return fail(FSS_EUNSUPPORTED, "rss_fetch_unique: more than 65535 words per record");
    if (!d_x || !d_rows || !d_out) return fail(FSS_EINVAL, "rss_fetch_unique: NULL argument");
    for (int i = 0; i < 3; i++)
        if (!d_x[i] || !d_rows[i] || !d_out[i]) return fail(FSS_EINVAL, "rss_fetch_unique: NULL share %d", i);
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < 3; i++) {
        hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, s, (uint64_t)nwords, d_out[i]);
        int rc = check_launch("k_zero");
        if (rc) return rc;
    }
    if (ncand == 0) return FSS_OK;
    // about 8 blocks per CU; each block takes a contiguous run of candidates
    const unsigned grid = grid_of(ncand, kFetchBlock) > 2048 ? 2048 : grid_of(ncand, kFetchBlock);
    hipLaunchKernelGGL(k_fetch_unique, dim3(grid), dim3(kFetchBlock), 0, s, ncand, nwords, d_x[0], d_x[1], d_x[2], d_rows[0],
                       d_rows[1], d_rows[2], d_out[0], d_out[1], d_out[2]);
    return check_launch("k_fetch_unique");
}

uint64_t rss_fetch_many_workspace_bytes(uint64_t ncand, uint32_t nwords) {
    if (ncand == 0 || nwords == 0) return 0;
    size_t scan = 0;
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, scan, (const uint32_t*)nullptr, (uint32_t*)nullptr, (int)ncand);
    const uint64_t tw = ncand * nwords * 4;
    return shuffle_ws(ncand, nwords) + 3 * ((tw + 255) & ~255ull) + 2 * ((ncand * 4 + 255) & ~255ull) +
           ((scan + 255) & ~255ull) + 4096;
}

static int shuffle_open_compact(uint64_t ncand, uint32_t nwords, const uint32_t* const d_table[3],
                                const uint64_t seeds[3], uint32_t* const d_out[3], uint32_t* d_rows_out,
                                uint32_t* d_count, void* d_work, uint64_t work_bytes, void* stream, bool parity,
                                const char* who) {
    last_error().clear();
    if (!parity && nwords < 2) return fail(FSS_EINVAL, "%s: records need the bit word and at least one word", who);
    if (nwords == 0) return fail(FSS_EINVAL, "%s: empty records", who);
    if (!d_table || !d_out || !seeds || !d_rows_out || !d_count) return fail(FSS_EINVAL, "%s: NULL argument", who);
    for (int i = 0; i < 3; i++)
        if (!d_table[i] || !d_out[i]) return fail(FSS_EINVAL, "%s: NULL share %d", who, i);
    if (ncand > 0x7FFFFFFFull) return fail(FSS_EUNSUPPORTED, "%s: more than 2^31 rows", who);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, (uint64_t)1, d_count);
    int rc = check_launch("k_zero");
    if (rc || ncand == 0) return rc;
    if (!d_work || work_bytes < rss_fetch_many_workspace_bytes(ncand, nwords))
        return fail(FSS_ENOMEM, "%s: workspace needs %llu bytes", who,
                    (unsigned long long)rss_fetch_many_workspace_bytes(ncand, nwords));
    Carve ws{(uint8_t*)d_work, work_bytes};
    const uint64_t tw = ncand * nwords;
    uint32_t* sh[3] = {ws.take<uint32_t>(tw), ws.take<uint32_t>(tw), ws.take<uint32_t>(tw)};
    uint32_t* flags = ws.take<uint32_t>(ncand);
    uint32_t* pos = ws.take<uint32_t>(ncand);
    size_t scan = 0;
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, scan, (const uint32_t*)nullptr, (uint32_t*)nullptr, (int)ncand);
    void* scan_tmp = ws.take<uint8_t>(scan);
    if (!ws.ok) return fail(FSS_ENOMEM, "%s: workspace too small", who);
    rc = run_shuffle(ncand, nwords, d_table, seeds, sh, ws, s);
    if (rc) return rc;
    if (parity)
        hipLaunchKernelGGL(k_open_parity, dim3((unsigned)((ncand + 255) / 256)), dim3(256), 0, s, ncand, nwords,
                           (uint32_t)((nwords & 3u) == 0 && aligned16(sh[0]) && aligned16(sh[1]) && aligned16(sh[2])),
                           sh[0], sh[1], sh[2], flags);
    else
        hipLaunchKernelGGL(k_open_flags, dim3((unsigned)((ncand + 255) / 256)), dim3(256), 0, s, ncand, nwords,
                           sh[0], sh[1], sh[2], flags);
    rc = check_launch("k_open");
    if (rc) return rc;
    if (hipcub::DeviceScan::ExclusiveSum(scan_tmp, scan, flags, pos, (int)ncand, s) != hipSuccess)
        return fail(FSS_EDEVICE, "%s: scan failed", who);
    hipLaunchKernelGGL(k_compact, dim3(grid_of(ncand * (nwords - (parity ? 0u : 1u)), 256)), dim3(256), 0, s, ncand, nwords,
                       parity ? 0u : 1u, flags, pos, sh[0], sh[1], sh[2], d_out[0], d_out[1], d_out[2], d_rows_out);
    rc = check_launch("k_compact");
    if (rc) return rc;
    hipLaunchKernelGGL(k_count, dim3(1), dim3(64), 0, s, ncand, flags, pos, d_count);
    return check_launch("k_count");
}

int rss_fetch_many(uint64_t ncand, uint32_t nwords, const uint32_t* const d_table[3], const uint64_t seeds[3],
                   uint32_t* const d_out[3], uint32_t* d_rows_out, uint32_t* d_count, void* d_work,
                   uint64_t work_bytes, void* stream) {
    return shuffle_open_compact(ncand, nwords, d_table, seeds, d_out, d_rows_out, d_count, d_work, work_bytes, stream,
                                false, "rss_fetch_many");
}

int rss_compact_valid(uint64_t nrec, uint32_t nwords, const uint32_t* const d_table[3], const uint64_t seeds[3],
                      uint32_t* const d_out[3], uint32_t* d_rows_out, uint32_t* d_count, void* d_work,
                      uint64_t work_bytes, void* stream) {
    return shuffle_open_compact(nrec, nwords, d_table, seeds, d_out, d_rows_out, d_count, d_work, work_bytes, stream,
                                true, "rss_compact_valid");
}

}  // extern "C"
