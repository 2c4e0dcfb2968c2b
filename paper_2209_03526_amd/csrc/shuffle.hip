// shuffle.hip -- three-party secret-shared shuffle (Alg. 5) and secure fetching
// of matched records (Alg. 4, Cases I and II), all three servers simulated.
//
// Tables are row-major: record r of a W-word table at words [r*W, r*W + W).
// Each pair of servers derives from its seed, with the counter-mode generator
// (domain 6), its permutations (stable sort of one 64-bit key per row) and
// mask tables (one AES block per four words); applying a permutation is the
// row gather out[i] = in[perm[i]].  The sequence of Alg. 5 is kept: X1, Y1
// and C1 are stored as the messages one server computes and sends; a message
// built with two permutations (X1, C2) is gathered through both in one pass,
// and C2 is folded into CS2's R3 = C1 ^ C2 as it is formed.

#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <stdint.h>

#include <mutex>

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

// Mask table `table` of the pair seed: word k = r*W + w is word (k mod 4) of
// block (6, table, W, 0, k div 4).  Block m gives words 4m .. 4m+3.
__global__ __launch_bounds__(kBlock) void k_mask_table(RoundKeys rk, uint32_t table, uint32_t nwords, uint64_t total,
                                                      uint32_t vec, uint32_t* __restrict__ out) {
    __shared__ uint32_t tab[kLdsTableWords];
    lds_table_fill(tab, g_tab.t0);
    __syncthreads();
    const LaneOff lo = lane_offset();
    const uint64_t nblk = (total + 3) / 4;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t m = (uint64_t)blockIdx.x * kBlock + threadIdx.x; m < nblk; m += stride) {
        const uint4 b = aes128_encrypt(make_uint4(6u | (table << 16), nwords, 0u, (uint32_t)m), ArgKey{rk}, tab, lo);
        if (vec && 4 * m + 4 <= total) {
            *(uint4*)(out + 4 * m) = b;
        } else {
            const uint32_t v[4] = {b.x, b.y, b.z, b.w};
            for (int q = 0; q < 4; q++)
                if (4 * m + q < total) out[4 * m + q] = v[q];
        }
    }
}

// Sort keys of permutation p: row r -> words 0-1 of block (6, 16 + p, 0, 0, r).
__global__ __launch_bounds__(kBlock) void k_perm_keys(RoundKeys rk, uint32_t p, uint64_t nrows,
                                                     uint64_t* __restrict__ keys, uint32_t* __restrict__ idx) {
    __shared__ uint32_t tab[kLdsTableWords];
    lds_table_fill(tab, g_tab.t0);
    __syncthreads();
    const LaneOff lo = lane_offset();
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t r = (uint64_t)blockIdx.x * kBlock + threadIdx.x; r < nrows; r += stride) {
        const uint4 b = aes128_encrypt(make_uint4(6u | ((16u + p) << 16), 0u, 0u, (uint32_t)r), ArgKey{rk}, tab, lo);
        keys[r] = (uint64_t)b.x | ((uint64_t)b.y << 32);
        idx[r] = (uint32_t)r;
    }
}

// out[i] = a[p] ^ b[p] ^ c[p] ^ post[i], p = perm[i] (absent tables skipped).
// With vec (record width a multiple of 4 words, every table 16-byte aligned)
// one thread moves 4 words with 16-byte loads and stores, else one word; row
// and word come from 32-bit division (rows < 2^31, checked by the callers).
__global__ void k_gather_xor(uint64_t nrows, uint32_t nwords, uint32_t vec, const uint32_t* __restrict__ perm,
                             const uint32_t* __restrict__ a, const uint32_t* __restrict__ b,
                             const uint32_t* __restrict__ c, const uint32_t* __restrict__ post,
                             uint32_t* __restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    if (vec) {
        const uint32_t q = nwords >> 2;                 // uint4 per record
        const uint64_t total = nrows * q;
        for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += stride) {
            const uint32_t i = (uint32_t)(k / q), w = (uint32_t)(k - (uint64_t)i * q);
            const uint64_t src = (uint64_t)perm[i] * q + w;
            uint4 v = ((const uint4*)a)[src];
            if (b) v = xor4(v, ((const uint4*)b)[src]);
            if (c) v = xor4(v, ((const uint4*)c)[src]);
            if (post) v = xor4(v, ((const uint4*)post)[k]);
            ((uint4*)out)[k] = v;
        }
        return;
    }
    const uint64_t total = nrows * nwords;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += stride) {
        const uint32_t i = (uint32_t)(k / nwords), w = (uint32_t)(k - (uint64_t)i * nwords);
        const uint64_t src = (uint64_t)perm[i] * nwords + w;
        uint32_t v = a[src];
        if (b) v ^= b[src];
        if (c) v ^= c[src];
        if (post) v ^= post[k];
        out[k] = v;
    }
}

// Two permutations in one pass: out[i] = A[q] ^ mid[p] ^ post[i] ^ post2[i]
// with p = p_out[i], q = p_in[p] and A = a ^ b ^ c (absent tables skipped):
// pi_out(pi_in(A) ^ mid) ^ post ^ post2 without writing pi_in(A) ^ mid.
// vec as in k_gather_xor.
__global__ void k_gather2_xor(uint64_t nrows, uint32_t nwords, uint32_t vec, const uint32_t* __restrict__ p_out,
                              const uint32_t* __restrict__ p_in, const uint32_t* __restrict__ a,
                              const uint32_t* __restrict__ b, const uint32_t* __restrict__ c,
                              const uint32_t* __restrict__ mid, const uint32_t* __restrict__ post,
                              const uint32_t* __restrict__ post2, uint32_t* __restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint32_t q = vec ? nwords >> 2 : nwords;       // units (uint4 or word) per record
    const uint64_t total = nrows * q;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += stride) {
        const uint32_t i = (uint32_t)(k / q), w = (uint32_t)(k - (uint64_t)i * q);
        const uint32_t p = p_out[i];
        const uint64_t sp = (uint64_t)p * q + w, sq = (uint64_t)p_in[p] * q + w;
        if (vec) {
            uint4 v = ((const uint4*)a)[sq];
            if (b) v = xor4(v, ((const uint4*)b)[sq]);
            if (c) v = xor4(v, ((const uint4*)c)[sq]);
            if (mid) v = xor4(v, ((const uint4*)mid)[sp]);
            if (post) v = xor4(v, ((const uint4*)post)[k]);
            if (post2) v = xor4(v, ((const uint4*)post2)[k]);
            ((uint4*)out)[k] = v;
        } else {
            uint32_t v = a[sq];
            if (b) v ^= b[sq];
            if (c) v ^= c[sq];
            if (mid) v ^= mid[sp];
            if (post) v ^= post[k];
            if (post2) v ^= post2[k];
            out[k] = v;
        }
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

size_t sort_temp_bytes(uint64_t nrows) {
    size_t b = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, b, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                             (const uint32_t*)nullptr, (uint32_t*)nullptr, (int)nrows);
    return b;
}

uint64_t shuffle_ws(uint64_t nrows, uint32_t nwords) {
    auto r = [](uint64_t b) { return (b + 255) & ~255ull; };
    const uint64_t tw = nrows * nwords * 4;
    // tables T12 T23 T31 X1 Y1 C1; three permutations; sort keys in and out;
    // the identity index; the sort's temporary storage
    return 6 * r(tw) + 3 * r(nrows * 4) + 2 * r(nrows * 8) + r(nrows * 4) + r(sort_temp_bytes(nrows)) + 4096;
}

// perm = stable argsort of the pair seed's row keys.
int make_perm(const RoundKeys& rk, uint32_t p, uint64_t nrows, uint64_t* keys, uint64_t* keys_sorted,
              uint32_t* idx, uint32_t* perm, void* temp, size_t temp_bytes, hipStream_t s) {
    hipLaunchKernelGGL(k_perm_keys, dim3(aes_grid(nrows)), dim3(kBlock), 0, s, rk, p, nrows, keys, idx);
    int rc = check_launch("k_perm_keys");
    if (rc) return rc;
    if (hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys, keys_sorted, idx, perm, (int)nrows, 0, 64, s) !=
        hipSuccess)
        return fail(FSS_EDEVICE, "rss_shuffle: radix sort failed");
    return FSS_OK;
}

int mask(const RoundKeys& rk, uint32_t table, uint64_t nrows, uint32_t nwords, uint32_t* out, hipStream_t s) {
    const uint64_t total = nrows * nwords;
    const uint64_t blocks = (total + 3) / 4;
    hipLaunchKernelGGL(k_mask_table, dim3(aes_grid(blocks)), dim3(kBlock), 0, s, rk, table, nwords, total,
                       (uint32_t)aligned16(out), out);
    return check_launch("k_mask_table");
}

int gather(uint64_t nrows, uint32_t nwords, const uint32_t* perm, const uint32_t* a, const uint32_t* b,
           const uint32_t* c, const uint32_t* post, uint32_t* out, hipStream_t s) {
    const bool vec = (nwords & 3u) == 0 && aligned16(a) && aligned16(b) && aligned16(c) && aligned16(post) &&
                     aligned16(out);
    hipLaunchKernelGGL(k_gather_xor, dim3(grid_of(vec ? nrows * nwords / 4 : nrows * nwords, 256)), dim3(256), 0, s,
                       nrows, nwords, (uint32_t)vec, perm, a, b, c, post, out);
    return check_launch("k_gather_xor");
}

int gather2(uint64_t nrows, uint32_t nwords, const uint32_t* p_out, const uint32_t* p_in, const uint32_t* a,
            const uint32_t* b, const uint32_t* c, const uint32_t* mid, const uint32_t* post, const uint32_t* post2,
            uint32_t* out, hipStream_t s) {
    const bool vec = (nwords & 3u) == 0 && aligned16(a) && aligned16(b) && aligned16(c) && aligned16(mid) &&
                     aligned16(post) && aligned16(post2) && aligned16(out);
    hipLaunchKernelGGL(k_gather2_xor, dim3(grid_of(vec ? nrows * nwords / 4 : nrows * nwords, 256)), dim3(256), 0, s,
                       nrows, nwords, (uint32_t)vec, p_out, p_in, a, b, c, mid, post, post2, out);
    return check_launch("k_gather2_xor");
}

// A second stream of the library's own (default priority, non-blocking) on
// which the mask tables are made while the permutations are sorted on the
// caller's stream: the first is AES work, the second memory-bound, and
// nothing joins them before the gathers.  Created once; ordered against the
// caller's stream with events only.
hipStream_t side_stream() {
    static hipStream_t side = nullptr;
    static std::once_flag once;
    std::call_once(once, [] {
        if (hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess) side = nullptr;
    });
    return side;
}

// Alg. 5 with all three servers simulated; out[0..2] = R1, R2, R3.
int run_shuffle(uint64_t nrows, uint32_t nwords, const uint32_t* const d[3], const uint64_t seeds[3],
                uint32_t* const out[3], Carve& ws, hipStream_t s) {
    const uint64_t tw = nrows * nwords;
    const RoundKeys k12 = seed_key(seeds[0]), k23 = seed_key(seeds[1]), k31 = seed_key(seeds[2]);
    uint32_t* t12 = ws.take<uint32_t>(tw);
    uint32_t* t23 = ws.take<uint32_t>(tw);
    uint32_t* t31 = ws.take<uint32_t>(tw);
    uint32_t* x1 = ws.take<uint32_t>(tw);
    uint32_t* y1 = ws.take<uint32_t>(tw);
    uint32_t* c1 = ws.take<uint32_t>(tw);
    uint32_t* p12 = ws.take<uint32_t>(nrows);
    uint32_t* p23 = ws.take<uint32_t>(nrows);
    uint32_t* p31 = ws.take<uint32_t>(nrows);
    uint64_t* keys = ws.take<uint64_t>(nrows);
    uint64_t* keys_sorted = ws.take<uint64_t>(nrows);
    uint32_t* idx = ws.take<uint32_t>(nrows);
    const size_t tb = sort_temp_bytes(nrows);
    void* temp = ws.take<uint8_t>(tb);
    if (!ws.ok) return fail(FSS_ENOMEM, "rss_shuffle: workspace too small");
    int rc = FSS_OK;
    // pair seeds: s12 -> pi12, T12, R2; s23 -> pi23, T23; s31 -> pi31, T31, R1.
    // Masks on the side stream (after everything already on s), permutations
    // on s; s waits for the masks before the first gather.
    hipStream_t ms = side_stream();
    hipEvent_t fork = nullptr, join = nullptr;
    bool forked = false;
    if (ms && hipEventCreateWithFlags(&fork, hipEventDisableTiming) == hipSuccess &&
        hipEventCreateWithFlags(&join, hipEventDisableTiming) == hipSuccess && hipEventRecord(fork, s) == hipSuccess &&
        hipStreamWaitEvent(ms, fork, 0) == hipSuccess)
        forked = true;
    const hipStream_t mstream = forked ? ms : s;       // without a side stream, all on s
    if (!rc) rc = mask(k12, kT12, nrows, nwords, t12, mstream);
    if (!rc) rc = mask(k12, kR2, nrows, nwords, out[1], mstream);       // R2
    if (!rc) rc = mask(k23, kT23, nrows, nwords, t23, mstream);
    if (!rc) rc = mask(k31, kT31, nrows, nwords, t31, mstream);
    if (!rc) rc = mask(k31, kR1, nrows, nwords, out[0], mstream);       // R1
    const bool recorded = forked && hipEventRecord(join, ms) == hipSuccess;
    // the permutations on the caller's stream, side by side with the masks
    if (!rc) rc = make_perm(k12, kP12, nrows, keys, keys_sorted, idx, p12, temp, tb, s);
    if (!rc) rc = make_perm(k23, kP23, nrows, keys, keys_sorted, idx, p23, temp, tb, s);
    if (!rc) rc = make_perm(k31, kP31, nrows, keys, keys_sorted, idx, p31, temp, tb, s);
    // the join is waited for whatever happened above, so that no work queued on
    // the side stream outlives the caller's view of this call
    const bool joined = !forked || (recorded && hipStreamWaitEvent(s, join, 0) == hipSuccess);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (!joined) {
        (void)hipStreamSynchronize(ms);       // the side stream drains before the failure is reported
        if (!rc) rc = fail(FSS_EDEVICE, "rss_shuffle: stream join failed");
    }
    // CS1: X1 = pi31[pi12(D1 ^ D2 ^ T12) ^ T31]  (both permutations in one pass)
    if (!rc) rc = gather2(nrows, nwords, p31, p12, d[0], d[1], t12, t31, nullptr, nullptr, x1, s);
    // CS2: Y1 = pi12(D3 ^ T12); C1 = pi23(X1 ^ T23) ^ R2
    if (!rc) rc = gather(nrows, nwords, p12, d[2], t12, nullptr, nullptr, y1, s);
    if (!rc) rc = gather(nrows, nwords, p23, x1, t23, nullptr, out[1], c1, s);
    // CS3: C2 = pi23[pi31(Y1 ^ T31) ^ T23] ^ R1, and CS2's R3 = C1 ^ C2, in one
    // pass (with the servers simulated together, C2 need not be stored)
    if (!rc) rc = gather2(nrows, nwords, p23, p31, y1, t31, nullptr, t23, out[0], c1, out[2], s);
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
