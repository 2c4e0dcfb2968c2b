// shuffle.hip -- three-party secret-shared shuffle (Alg. 5) and secure fetching
// of matched records (Alg. 4, Cases I and II), all three servers simulated.
//
// Tables are row-major: record r of a W-word table at words [r*W, r*W + W).
// Each pair of servers derives from its seed, with ChaCha12, its permutation
// (stable sort of one 64-bit key per row) and its mask tables; applying a
// permutation is the row gather out[i] = in[perm[i]].  A quad of lanes takes
// one 16-word slice of a record, which is one ChaCha block of every mask
// table (made by the four lanes together, chacha_gfx950.hpp), each lane one
// 16-byte quarter of it; so masks are made where they are XORed (VALU only,
// no table in LDS) and no mask table is stored.
//
// Two launches carry the five steps of Alg. 5.  The first reads the input
// shares in order and scatters each row through both inverse permutations
// (pi12, then pi31): it forms CS1's X1 (its pi12(D1 ^ D2 ^ T12) never leaves
// CS1) and CS3's pi31(Y1 ^ T31) (CS2's message Y1 met as it is formed), and
// draws R2 and R1.  The second, a gather through pi23 because its outputs
// are the result shares in order, forms C1 and C2 and R3 = C1 ^ C2.  Random
// 64-byte reads cost a whole 128-byte line and random writes only their
// bytes, hence scatters where the order allows.

#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <stdint.h>

#include <array>
#include <atomic>
#include <initializer_list>
#include <map>
#include <mutex>

#include "../../include/oblivgm_fss.h"
#include "chacha_gfx950.hpp"
#include "common.hpp"

using namespace ogm;

namespace {

constexpr int kBlock = 256;

enum { kT12 = 1, kR2 = 2, kT23 = 3, kT31 = 4, kR1 = 5 };
enum { kP12 = 0, kP23 = 1, kP31 = 2 };

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }   // NULL counts as aligned

unsigned slice_grid(uint64_t items) {
    uint64_t g = (items + kBlock - 1) / kBlock;
    if (g == 0) g = 1;
    if (g > (1u << 20)) g = 1u << 20;
    return (unsigned)g;
}

// How the permutations of tables above 1024 rows are made
// (rss_set_shuffle_tuning); every method gives the same permutation.
//   0: radix pass, exact comparisons in every run
//   1: radix pass, sorting networks where they apply
//   2: buckets (up to 2^23 rows, else method 1), sorting networks where they apply
//   3: buckets, exact comparisons in every run
//   4: buckets, every bucket ordered by comparing every pair
enum { kPermRadixExact = 0, kPermRadix = 1, kPermBuckets = 2, kPermBucketsExact = 3, kPermBucketsPairs = 4 };
std::atomic<uint32_t> g_perm_method{kPermBuckets};

// Pair keys: ChaCha key words (seed mod 2^32, seed div 2^32, 6, 0, 0, 0, 0, 0).
constexpr uint32_t kShuffleDomain = 6;

ChachaKey pair_key(uint64_t seed) { return chacha_key(seed, kShuffleDomain); }

// Sort keys of permutation p: the key of row r is slice words 2e (low) and
// 2e + 1 (high), e = r mod 8, of block (r div 8, 0, 16 + p, 0); a quad makes
// the keys of eight rows, lane c those of rows 2c and 2c + 1.  The key is
// stored rotated left by hb bits, so that its top hb bits (the row's run id)
// sit in bits 0 .. hb-1, the range the radix pass sorts, and the whole key
// travels with it; the row number goes beside it.
__global__ __launch_bounds__(kBlock) void k_perm_keys(ChachaKey pk, uint32_t p, uint64_t nrows, uint32_t hb,
                                                     uint64_t* __restrict__ keys, uint32_t* __restrict__ idx) {
    const uint64_t total = ((nrows + 7) >> 3) * 4;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x; t < total; t += stride) {
        const uint4 o = chacha_quad(pk, (uint32_t)(t >> 2), 0u, 16u + p, 0u);
        const uint64_t r0 = (t >> 2) * 8 + 2 * (t & 3);
        const uint64_t key[2] = {(uint64_t)o.x | ((uint64_t)o.y << 32), (uint64_t)o.z | ((uint64_t)o.w << 32)};
#pragma unroll
        for (int e = 0; e < 2; e++) {
            if (r0 + e < nrows) {
                keys[r0 + e] = hb ? (key[e] << hb) | (key[e] >> (64 - hb)) : key[e];
                idx[r0 + e] = (uint32_t)(r0 + e);
            }
        }
    }
}

// Small tables (at most kSmallPerm rows, as in secAccess, which shuffles one
// fetched posting list): the three permutations of a shuffle in one launch,
// one workgroup each.  The workgroup makes its rows' keys into LDS (the same
// keys as k_perm_keys, not rotated), then row i's position is its rank: the
// rows with a smaller key, or an equal key and a smaller row number -- the
// stable argsort, as the sort path makes it.  Every lane of the wave reads the
// same key at a time (an LDS broadcast).
constexpr uint32_t kSmallPerm = 1024;

struct SmallPerms {
    ChachaKey pk[3];
    uint32_t p[3];
    uint32_t inverse[3];
    uint32_t* out[3];
};

// One permutation of n <= kSmallPerm rows made by the whole workgroup: keys
// into `key` (LDS), then each row's rank; `out` gets the permutation (or its
// inverse).  Every thread of the workgroup calls it; `key` is free again when
// it returns.
__device__ __forceinline__ void small_perm(ChachaKey pk, uint32_t p, uint32_t inverse, uint32_t n, uint64_t* key,
                                           uint32_t* out) {
    const uint32_t lanes = (n + 7) / 8 * 4;              // whole quads: a quad makes the keys of 8 rows
    for (uint32_t t = threadIdx.x; t < lanes; t += blockDim.x) {
        const uint4 o = chacha_quad(pk, t >> 2, 0u, 16u + p, 0u);
        const uint32_t r0 = (t >> 2) * 8 + 2 * (t & 3);
        if (r0 < n) key[r0] = (uint64_t)o.x | ((uint64_t)o.y << 32);
        if (r0 + 1 < n) key[r0 + 1] = (uint64_t)o.z | ((uint64_t)o.w << 32);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint64_t ki = key[i];
        uint32_t rank = 0;
        for (uint32_t j = 0; j < n; j++) {
            const uint64_t kj = key[j];
            rank += (kj < ki || (kj == ki && j < i)) ? 1u : 0u;
        }
        if (inverse)
            out[i] = rank;
        else
            out[rank] = i;
    }
    __syncthreads();
}

__global__ __launch_bounds__(1024) void k_perm_small(uint32_t n, SmallPerms J) {
    __shared__ uint64_t key[kSmallPerm];
    const uint32_t q = blockIdx.x;
    small_perm(J.pk[q], J.p[q], J.inverse[q], n, key, J.out[q]);
}

// The permutation is the stable argsort of the 64-bit keys.  It is made in two
// steps: a stable radix sort of the rows by run id (the top hb key bits, hb =
// ceil(log2 n) - 6, so that a run holds 64 rows on average), then each run
// ordered by its full keys.  Inside a run the radix sort has kept the rows in
// their original order, so "equal key, earlier position" is "equal key,
// smaller row" and the result is the full stable argsort.

// starts[b] = first position of run b in the sorted keys, b = 0 .. 2^hb, and
// starts[2^hb] = n, in one coalesced pass: position i (0 <= i <= n, position n
// counting as id 2^hb) writes the entries of the ids after its predecessor's
// id up to its own.  Over sorted keys each entry is written once.  Whatever
// the sort returned, every write stays in [0, 2^hb] and each thread's loop is
// bounded by 2^hb + 1; the ranking clamps the starts to [0, n], so it stays in
// bounds too.
__global__ void k_run_starts(uint64_t n, uint32_t hb, const uint64_t* __restrict__ keys,
                             uint32_t* __restrict__ starts) {
    const uint64_t nruns = 1ull << hb;
    const uint64_t id_mask = nruns - 1;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride) {
        const uint64_t lo = i == 0 ? 0 : (keys[i - 1] & id_mask) + 1;
        const uint64_t hi = i == n ? nruns : keys[i] & id_mask;
        for (uint64_t b = lo; b <= hi; b++) starts[b] = (uint32_t)i;
    }
}

// Broadcast of lane t's 64-bit value to the whole wavefront (t uniform).
__device__ __forceinline__ uint64_t lane_value(uint64_t v, uint32_t t) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, (int)t);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)t);
    return ((uint64_t)hi << 32) | lo;
}

// Lane l's copy of the value of lane l ^ J (every lane of the wavefront
// active): DPP quad permutations for J = 1, 2, a swizzle inside each half of
// the wavefront for J = 4, 8, 16, a permute across the halves for J = 32.
template <int J>
__device__ __forceinline__ uint32_t from_lane_xor(uint32_t v, uint32_t lane) {
    if constexpr (J == 1)
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1, 0, 3, 2]
    else if constexpr (J == 2)
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2, 3, 0, 1]
    else if constexpr (J < 32)
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (J << 10));     // and 31, or 0, xor J
    else
        return (uint32_t)__builtin_amdgcn_ds_bpermute((int)((lane ^ 32u) << 2), (int)v);
}

// Bitonic sorting network over the wavefront, element i in lane i (register
// a) or lane i - 64 (register b).  In the stage (K, J) element i meets element
// i ^ J and keeps the smaller value when bits J and K of i agree, the larger
// one otherwise; after the stages K = 2, 4, .., N (J = K/2 .. 1 in each) the N
// elements are in ascending order.
template <int K, int J>
__device__ __forceinline__ uint32_t bitonic_stage(uint32_t v, uint32_t i, uint32_t lane) {
    const uint32_t o = from_lane_xor<J>(v, lane);
    return (((i / J) ^ (i / K)) & 1u) ? max(o, v) : min(o, v);
}

template <int K, int J>
__device__ __forceinline__ void merge64(uint32_t& a, uint32_t lane) {
    a = bitonic_stage<K, J>(a, lane, lane);
    if constexpr (J > 1) merge64<K, J / 2>(a, lane);
}

template <int K>
__device__ __forceinline__ void sort64(uint32_t& a, uint32_t lane) {
    merge64<K, K / 2>(a, lane);
    if constexpr (K < 64) sort64<2 * K>(a, lane);
}

template <int K, int J>
__device__ __forceinline__ void merge128(uint32_t& a, uint32_t& b, uint32_t lane) {
    if constexpr (J == 64) {             // K = 128: the partners share a lane
        const uint32_t lo = min(a, b), hi = max(a, b);
        a = lo, b = hi;
    } else {
        a = bitonic_stage<K, J>(a, lane, lane);
        b = bitonic_stage<K, J>(b, lane + 64u, lane);
    }
    if constexpr (J > 1) merge128<K, J / 2>(a, b, lane);
}

template <int K>
__device__ __forceinline__ void sort128(uint32_t& a, uint32_t& b, uint32_t lane) {
    merge128<K, K / 2>(a, b, lane);
    if constexpr (K < 128) sort128<2 * K>(a, b, lane);
}

__device__ __forceinline__ uint32_t lane_read(uint32_t v, uint32_t src) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src << 2), (int)v);
}

// One wavefront per run: row e of the run goes to position start + rank(e),
// rank = number of rows of the run with a smaller key, or an equal key at an
// earlier position (inside a run the radix pass kept the original row order).
// With `inverse` the kernel writes the inverse permutation instead:
// out[row] = its position.
//
// Sorting-network path (runs of at most 128 rows, when `fast`): each row
// becomes the 32-bit value (the 25 key bits after the run id) << 7 | e, with
// 2^32 - 1 for the lanes past the run; the network sorts the run in the lanes
// (64 or 128 values), and e is read back from the low bits.  When no two
// neighbours in that order share their 25 key bits, it is the order of the
// full keys.  Otherwise -- and for longer runs -- the run takes the exact
// path.
//
// Exact path: the run's keys are taken 64 at a time into the lanes and
// broadcast with readlane, so any run length is ordered exactly (the cost
// grows as the square of the length).  All keys of a run share their id bits
// (bits 0 .. hb-1 of the rotated key); when the run has at most 2^hb rows
// those bits are replaced by the row's position in the run, which makes every
// key of the run distinct and ordered as (key, position), so one compare per
// row does.
__global__ __launch_bounds__(256) void k_rank_runs(uint64_t n, uint32_t hb, uint32_t inverse, uint32_t fast,
                                                   const uint32_t* __restrict__ starts,
                                                   const uint64_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ rows, uint32_t* __restrict__ perm) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t nruns = 1u << hb;
    const uint64_t id_mask = (uint64_t)(nruns - 1u);
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    // the run number is the same on every lane of the wavefront; saying so
    // keeps the run bounds and loop counters in scalar registers
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t n32 = (uint32_t)n;
    for (uint32_t b = blockIdx.x * (blockDim.x >> 6) + wave; b < nruns; b += waves) {
        const uint32_t s = min(starts[b], n32), e_end = min(starts[b + 1], n32);
        const uint32_t m = e_end > s ? e_end - s : 0u;
        if (m == 0) continue;
        bool exact = !fast || m > 128;
        if (!exact) {
            const uint32_t pb = lane + 64u;
            uint32_t a = 0xFFFFFFFFu, bb = 0xFFFFFFFFu, ra = 0u, rb = 0u;
            if (lane < m) {
                a = ((uint32_t)(keys[s + lane] >> 39) << 7) | lane;
                ra = rows[s + lane];
            }
            if (pb < m) {
                bb = ((uint32_t)(keys[s + pb] >> 39) << 7) | pb;
                rb = rows[s + pb];
            }
            if (m <= 64)
                sort64<2>(a, lane);
            else
                sort128<2>(a, bb, lane);
            // neighbours in sorted order: position lane - 1 for register a
            // (lane 0 has none), and for register b the last of a at lane 0
            const uint32_t prev_a = lane_read(a, (lane - 1u) & 63u);
            const uint32_t prev_b_lane = lane_read(bb, (lane - 1u) & 63u);
            const uint32_t prev_b = lane == 0 ? prev_a : prev_b_lane;
            const bool tie = (lane >= 1 && lane < m && (a >> 7) == (prev_a >> 7)) ||
                             (pb < m && (bb >> 7) == (prev_b >> 7));
            if (__ballot(tie) != 0) {
                exact = true;
            } else {
                const uint32_t qa = a & 127u, qb = bb & 127u;
                const uint32_t ya = lane_read(ra, qa & 63u), za = lane_read(rb, qa & 63u);
                const uint32_t yb = lane_read(ra, qb & 63u), zb = lane_read(rb, qb & 63u);
                const uint32_t row_a = qa < 64 ? ya : za, row_b = qb < 64 ? yb : zb;
                if (lane < m) {
                    if (!inverse)
                        perm[s + lane] = row_a;
                    else if (row_a < n32)
                        perm[row_a] = s + lane;
                }
                if (pb < m) {
                    if (!inverse)
                        perm[s + pb] = row_b;
                    else if (row_b < n32)
                        perm[row_b] = s + pb;
                }
            }
        }
        if (!exact) continue;
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
                const uint32_t row = rows[s + e];
                if (!inverse)
                    perm[s + rank] = row;
                else if (row < n32)
                    perm[row] = s + rank;
            }
        }
    }
}

// ---------------------------------------------------------------- permutations by buckets
//
// Tables of 1025 .. 2^23 rows take the stable argsort of their keys in four
// launches and no sort library: with hb run-id bits as above, the top
// d1 = ceil(log2 n) - 12 key bits (at least 0) name the row's bucket (2^11 ..
// 2^12 rows on average), the next d2 = hb - d1 bits its run in the bucket.
//   count: each workgroup makes the keys of 8192 rows and counts them per
//          bucket in LDS: counts[bucket][workgroup];
//   scan:  per bucket, the workgroups' exclusive offsets and the total; then
//          the buckets' starts;
//   place: the workgroups make their keys again, group them by bucket in
//          LDS and store each row (key and row number) in its bucket's range
//          (the order inside a bucket follows LDS counters: arbitrary);
//   rank:  one workgroup per bucket loads it into LDS, groups it by run (LDS
//          counters again), and orders each run by (key, row number) as the
//          radix path's ranking does: a sorting network over the wavefront
//          for runs of at most 128 rows whose leading 25 bits after the run
//          id differ, exact comparisons otherwise.  A bucket of more than
//          kBucketCap rows (about 50 standard deviations above the mean for
//          keys drawn by ChaCha12) is ordered by comparing every pair.
// Row r's position is its bucket's start + its run's start in the bucket +
// its rank in the run, and (key, row number) orders bucket, run and rank:
// the result is the stable argsort whatever order the placing left.
constexpr uint32_t kChunkRows = 8192;        // rows per counting / placing workgroup
constexpr uint32_t kMaxBuckets = 2048;       // 2^(23 - 12)
constexpr uint32_t kBucketCap = 7168;        // rows of a bucket held in LDS
constexpr uint64_t kBucketMaxRows = 1ull << 23;

// The three permutations of a shuffle, made together: blockIdx.y picks one.
struct BucketSet {
    ChachaKey pk[3];
    uint32_t p[3], inverse[3];
    uint32_t* perm[3];          // output: the permutation or its inverse
    uint64_t* skeys[3];         // keys placed by bucket
    uint32_t* srows[3];         // their row numbers
    uint32_t* counts[3];        // per bucket and counting workgroup
    uint32_t* totals[3];        // per bucket
    uint32_t* starts[3];        // bucket starts, nb + 1
};

__device__ __forceinline__ uint32_t bucket_of(uint64_t key, uint32_t d1) {
    return d1 ? (uint32_t)(key >> (64 - d1)) : 0u;
}

// The keys of the block's rows, two per lane (all lanes of each quad active):
// f(row, key) for every row below n.
template <class F>
__device__ __forceinline__ void chunk_keys(ChachaKey pk, uint32_t p, uint64_t n, F f) {
    const uint64_t q0 = (uint64_t)blockIdx.x * (kChunkRows / 8);
    for (uint32_t t = threadIdx.x; t < kChunkRows / 2; t += blockDim.x) {
        const uint64_t q = q0 + (t >> 2);
        const uint4 o = chacha_quad(pk, (uint32_t)q, 0u, 16u + p, 0u);
        const uint64_t r0 = q * 8 + 2 * (t & 3);
        if (r0 < n) f(r0, (uint64_t)o.x | ((uint64_t)o.y << 32));
        if (r0 + 1 < n) f(r0 + 1, (uint64_t)o.z | ((uint64_t)o.w << 32));
    }
}

__global__ __launch_bounds__(1024) void k_perm_count(uint64_t n, uint32_t d1, uint32_t nblk, BucketSet S) {
    __shared__ uint32_t hist[kMaxBuckets];
    const uint32_t q = blockIdx.y;
    const ChachaKey pk = S.pk[q];
    const uint32_t p = S.p[q];
    uint32_t* __restrict__ counts = S.counts[q];
    const uint32_t nb = 1u << d1;
    for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    chunk_keys(pk, p, n, [&](uint64_t, uint64_t key) { atomicAdd(&hist[bucket_of(key, d1)], 1u); });
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x) counts[(uint64_t)i * nblk + blockIdx.x] = hist[i];
}

// Exclusive scan of 256 values in LDS (blockDim.x = 256); returns this
// thread's exclusive prefix, *total the sum.
__device__ __forceinline__ uint32_t block_scan256(uint32_t v, uint32_t* sh, uint32_t* total) {
    const uint32_t t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (uint32_t d = 1; d < 256; d <<= 1) {
        const uint32_t x = t >= d ? sh[t - d] : 0u;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    *total = sh[255];
    return sh[t] - v;
}

// One workgroup (256 threads) per bucket: counts[bucket][w] becomes the
// number of the bucket's rows in workgroups before w; totals[bucket] = all.
__global__ __launch_bounds__(256) void k_bucket_offsets(uint32_t nblk, BucketSet S) {
    __shared__ uint32_t sh[256];
    uint32_t* __restrict__ totals = S.totals[blockIdx.y];
    uint32_t* c = S.counts[blockIdx.y] + (uint64_t)blockIdx.x * nblk;
    const uint32_t per = (nblk + 255) / 256;       // at most 4 (nblk <= 1024)
    const uint32_t b0 = threadIdx.x * per;
    uint32_t v[4] = {0, 0, 0, 0}, sum = 0;
    for (uint32_t k = 0; k < per; k++) {
        v[k] = b0 + k < nblk ? c[b0 + k] : 0u;
        sum += v[k];
    }
    uint32_t total = 0;
    uint32_t run = block_scan256(sum, sh, &total);
    for (uint32_t k = 0; k < per; k++) {
        if (b0 + k < nblk) c[b0 + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = total;
}

// One workgroup (256 threads): starts[b] = rows in buckets before b, b = 0 .. nb.
__global__ __launch_bounds__(256) void k_bucket_starts(uint32_t nb, BucketSet S) {
    __shared__ uint32_t sh[256];
    const uint32_t* __restrict__ totals = S.totals[blockIdx.y];
    uint32_t* __restrict__ starts = S.starts[blockIdx.y];
    const uint32_t per = (nb + 255) / 256;         // at most 8 (nb <= 2048)
    const uint32_t b0 = threadIdx.x * per;
    uint32_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0}, sum = 0;
    for (uint32_t k = 0; k < per; k++) {
        v[k] = b0 + k < nb ? totals[b0 + k] : 0u;
        sum += v[k];
    }
    uint32_t total = 0;
    uint32_t run = block_scan256(sum, sh, &total);
    for (uint32_t k = 0; k < per; k++) {
        if (b0 + k < nb) starts[b0 + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) starts[nb] = total;
}

// Placing: the workgroup's keys (eight per thread, kept in registers) are
// counted per bucket and grouped by bucket in LDS first, so that each thread
// then stores consecutive positions of a bucket's range: the stores of a
// wavefront cover a few contiguous segments instead of 64 scattered words.
__global__ __launch_bounds__(1024) void k_perm_place(uint64_t n, uint32_t d1, uint32_t nblk, BucketSet S) {
    const uint32_t q = blockIdx.y;
    const ChachaKey pk = S.pk[q];
    const uint32_t p = S.p[q];
    const uint32_t* __restrict__ counts = S.counts[q];
    const uint32_t* __restrict__ starts = S.starts[q];
    uint64_t* __restrict__ skeys = S.skeys[q];
    uint32_t* __restrict__ srows = S.srows[q];
    __shared__ uint64_t lkeys[kChunkRows];
    __shared__ uint32_t lrows[kChunkRows];
    __shared__ uint32_t loff[kMaxBuckets];     // the bucket's first slot in the workgroup's group
    __shared__ uint32_t lcur[kMaxBuckets];     // counts, then slot cursors
    __shared__ uint32_t gpos[kMaxBuckets];     // the bucket's first position for this workgroup
    __shared__ uint32_t scan[1024];
    const uint32_t nb = 1u << d1, tid = threadIdx.x;
    for (uint32_t i = tid; i < nb; i += 1024) lcur[i] = 0;
    __syncthreads();
    uint64_t key[8], row0[4];
    const uint64_t q0 = (uint64_t)blockIdx.x * (kChunkRows / 8);
    // the rows and keys of chunk_keys (which k_perm_count counts), unrolled
    // so that the eight keys stay in registers
#pragma unroll
    for (uint32_t it = 0; it < 4; it++) {         // kChunkRows / 2 lanes' worth: 4 x 1024
        const uint32_t t = tid + 1024u * it;
        const uint64_t q = q0 + (t >> 2);
        const uint4 o = chacha_quad(pk, (uint32_t)q, 0u, 16u + p, 0u);
        row0[it] = q * 8 + 2 * (t & 3);
        key[2 * it] = (uint64_t)o.x | ((uint64_t)o.y << 32);
        key[2 * it + 1] = (uint64_t)o.z | ((uint64_t)o.w << 32);
        if (row0[it] < n) atomicAdd(&lcur[bucket_of(key[2 * it], d1)], 1u);
        if (row0[it] + 1 < n) atomicAdd(&lcur[bucket_of(key[2 * it + 1], d1)], 1u);
    }
    __syncthreads();
    {   // exclusive scan of the counts, two buckets per thread (nb <= 2048)
        const uint32_t a = 2 * tid < nb ? lcur[2 * tid] : 0u, b = 2 * tid + 1 < nb ? lcur[2 * tid + 1] : 0u;
        scan[tid] = a + b;
        __syncthreads();
        for (uint32_t d = 1; d < 1024; d <<= 1) {
            const uint32_t x = tid >= d ? scan[tid - d] : 0u;
            __syncthreads();
            scan[tid] += x;
            __syncthreads();
        }
        const uint32_t ex = scan[tid] - (a + b);
        if (2 * tid < nb) loff[2 * tid] = lcur[2 * tid] = ex;
        if (2 * tid + 1 < nb) loff[2 * tid + 1] = lcur[2 * tid + 1] = ex + a;
    }
    for (uint32_t i = tid; i < nb; i += 1024) gpos[i] = starts[i] + counts[(uint64_t)i * nblk + blockIdx.x];
    __syncthreads();
#pragma unroll
    for (uint32_t it = 0; it < 4; it++)
#pragma unroll
        for (uint32_t e = 0; e < 2; e++)
            if (row0[it] + e < n) {
                const uint32_t slot = atomicAdd(&lcur[bucket_of(key[2 * it + e], d1)], 1u);
                lkeys[slot] = key[2 * it + e];
                lrows[slot] = (uint32_t)(row0[it] + e);
            }
    __syncthreads();
    const uint64_t first = (uint64_t)blockIdx.x * kChunkRows;
    const uint32_t rows_here = (uint32_t)(n - first < kChunkRows ? n - first : kChunkRows);
    for (uint32_t i = tid; i < rows_here; i += 1024) {
        const uint64_t k = lkeys[i];
        const uint32_t bk = bucket_of(k, d1);
        const uint32_t dst = gpos[bk] + (i - loff[bk]);
        if (dst < n) {                            // always, with counts from k_perm_count
            skeys[dst] = k;
            srows[dst] = lrows[i];
        }
    }
}

// perm entry of the row at position pos (or its inverse).
__device__ __forceinline__ void put_position(uint32_t* perm, uint32_t inverse, uint32_t n, uint32_t pos, uint32_t row) {
    if (!inverse)
        perm[pos] = row;
    else if (row < n)
        perm[row] = pos;
}

// Bucket ranking; `mode` 0: networks where they apply, 1: exact comparisons
// for every run, 2: every bucket ordered by comparing every pair.
__global__ __launch_bounds__(1024) void k_bucket_rank(uint64_t n, uint32_t hb, uint32_t d1, uint32_t mode,
                                                      BucketSet S) {
    const uint32_t q = blockIdx.y;
    const uint32_t inverse = S.inverse[q];
    const uint32_t* __restrict__ starts = S.starts[q];
    const uint64_t* __restrict__ skeys = S.skeys[q];
    const uint32_t* __restrict__ srows = S.srows[q];
    uint32_t* __restrict__ perm = S.perm[q];
    __shared__ uint32_t part[kBucketCap];     // 25 key bits after the run id << 7 | slot in the run
    __shared__ uint32_t lrow[kBucketCap];     // row number
    __shared__ uint16_t sidx[kBucketCap];     // index in the bucket's range
    __shared__ uint32_t rcount[64];
    __shared__ uint32_t rstart[65];
    constexpr uint32_t kPer = (kBucketCap + 1023) / 1024;
    const uint32_t n32 = (uint32_t)n;
    const uint32_t s = min(starts[blockIdx.x], n32), e = min(starts[blockIdx.x + 1], n32);
    const uint32_t size = e > s ? e - s : 0u;
    if (size == 0) return;
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tid >> 6));
    if (size > kBucketCap || mode == 2) {
        // every pair: position = rows of the bucket with a smaller (key, row)
        for (uint32_t i = tid; i < size; i += blockDim.x) {
            const uint64_t ki = skeys[s + i];
            const uint32_t ri = srows[s + i];
            uint32_t rank = 0;
            for (uint32_t j = 0; j < size; j++) {
                const uint64_t kj = skeys[s + j];
                const uint32_t rj = srows[s + j];
                rank += (uint32_t)(kj < ki) | ((uint32_t)(kj == ki) & (uint32_t)(rj < ri));
            }
            put_position(perm, inverse, n32, s + rank, ri);
        }
        return;
    }
    const uint32_t d2 = hb - d1, nr = 1u << d2;
    const uint32_t run_mask = nr - 1u;
    for (uint32_t i = tid; i < nr; i += blockDim.x) rcount[i] = 0;
    __syncthreads();
    uint64_t key[kPer];
    uint32_t slot[kPer], row[kPer];
#pragma unroll
    for (uint32_t k = 0; k < kPer; k++) {
        const uint32_t i = tid + 1024u * k;
        key[k] = 0;
        row[k] = 0;
        if (i < size) {
            key[k] = skeys[s + i];
            row[k] = srows[s + i];
        }
    }
#pragma unroll
    for (uint32_t k = 0; k < kPer; k++) {
        slot[k] = 0;
        if (tid + 1024u * k < size) slot[k] = atomicAdd(&rcount[(uint32_t)(key[k] >> (64 - hb)) & run_mask], 1u);
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t acc = 0;
        for (uint32_t r = 0; r < nr; r++) {
            rstart[r] = acc;
            acc += rcount[r];
        }
        rstart[nr] = acc;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kPer; k++) {
        const uint32_t i = tid + 1024u * k;
        if (i < size) {
            const uint32_t pos = rstart[(uint32_t)(key[k] >> (64 - hb)) & run_mask] + slot[k];
            part[pos] = (((uint32_t)(key[k] >> (39 - hb)) & 0x1FFFFFFu) << 7) | (slot[k] & 127u);
            lrow[pos] = row[k];
            sidx[pos] = (uint16_t)i;
        }
    }
    __syncthreads();
    for (uint32_t r = wave; r < nr; r += blockDim.x >> 6) {
        const uint32_t rs = rstart[r], m = rstart[r + 1] - rs;
        if (m == 0) continue;
        const uint32_t base = s + rs;              // the run's first position
        bool exact = mode == 1 || m > 128;
        if (!exact) {
            const uint32_t pb = lane + 64u;
            uint32_t a = lane < m ? part[rs + lane] : 0xFFFFFFFFu;
            uint32_t bb = pb < m ? part[rs + pb] : 0xFFFFFFFFu;
            if (m <= 64)
                sort64<2>(a, lane);
            else
                sort128<2>(a, bb, lane);
            const uint32_t prev_a = lane_read(a, (lane - 1u) & 63u);
            const uint32_t prev_b_lane = lane_read(bb, (lane - 1u) & 63u);
            const uint32_t prev_b = lane == 0 ? prev_a : prev_b_lane;
            const bool tie = (lane >= 1 && lane < m && (a >> 7) == (prev_a >> 7)) ||
                             (pb < m && (bb >> 7) == (prev_b >> 7));
            if (__ballot(tie) != 0) {
                exact = true;
            } else {
                if (lane < m) put_position(perm, inverse, n32, base + lane, lrow[rs + (a & 127u)]);
                if (pb < m) put_position(perm, inverse, n32, base + pb, lrow[rs + (bb & 127u)]);
            }
        }
        if (!exact) continue;
        // exact: rank = members with a smaller (key, row), keys from the
        // bucket's range, 64 at a time broadcast with readlane
        for (uint32_t c0 = 0; c0 < m; c0 += 64) {
            const uint32_t ei = c0 + lane;
            const bool has = ei < m;
            const uint64_t ke = has ? skeys[s + sidx[rs + ei]] : 0ull;
            const uint32_t re = has ? lrow[rs + ei] : 0u;
            uint32_t rank = 0;
            for (uint32_t j0 = 0; j0 < m; j0 += 64) {
                const bool hj = j0 + lane < m;
                const uint64_t kj = hj ? skeys[s + sidx[rs + j0 + lane]] : 0ull;
                const uint32_t rj = hj ? lrow[rs + j0 + lane] : 0u;
                const uint32_t cnt = (uint32_t)__builtin_amdgcn_readfirstlane((int)(m - j0 < 64 ? m - j0 : 64));
                for (uint32_t t = 0; t < cnt; t++) {
                    const uint64_t kt = lane_value(kj, t);
                    const uint32_t rt = (uint32_t)__builtin_amdgcn_readlane((int)rj, (int)t);
                    rank += (uint32_t)(kt < ke) | ((uint32_t)(kt == ke) & (uint32_t)(rt < re));
                }
            }
            if (has) put_position(perm, inverse, n32, base + rank, re);
        }
    }
}

// A slice is words [16b, 16b + L) of record r, L = min(16, W - 16b): block
// (r, b, table, W) of each mask table covers it, and lane c of a quad moves
// its words 4c .. 4c + 3 (those below L).  VEC: W a multiple of 4 words and
// every table 16-byte aligned, so a quarter is one 16-byte access.
template <bool VEC>
__device__ __forceinline__ uint4 load_quarter(const uint32_t* __restrict__ t, uint64_t base, uint32_t c, uint32_t len) {
    if (VEC) return 4 * c < len ? *(const uint4*)(t + base + 4 * c) : make_uint4(0u, 0u, 0u, 0u);
    uint32_t v[4];
#pragma unroll
    for (uint32_t k = 0; k < 4; k++) v[k] = 4 * c + k < len ? t[base + 4 * c + k] : 0u;
    return make_uint4(v[0], v[1], v[2], v[3]);
}

template <bool VEC>
__device__ __forceinline__ void store_quarter(uint32_t* __restrict__ t, uint64_t base, uint32_t c, uint32_t len,
                                              uint4 v) {
    if (VEC) {
        if (4 * c < len) *(uint4*)(t + base + 4 * c) = v;
        return;
    }
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (uint32_t k = 0; k < 4; k++)
        if (4 * c + k < len) t[base + 4 * c + k] = w[k];
}

// An empty asm statement that the words pass through: it keeps the compiler
// from cancelling the mask T23 that C1 and C2 share (each server forms its
// own message with it).
__device__ __forceinline__ void pin(uint4& v) {
    asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w));
}

// Rounds pi12 and pi31 in one pass, as scatters through both inverse
// permutations: input row i goes to row j = inv12[i] after pi12 and to row
// l = inv31[j] after pi31, so
//   o0[l] = (g0 ^ g1 ^ T12)[i] ^ T31[j]   (CS1's X1)
//   o1[l] = (g2 ^ T12)[i] ^ T31[j]        (CS3's pi31(Y1 ^ T31), Y1 = CS2's pi12(D3 ^ T12))
//   r12[i] = R2, r31[i] = R1.
// The masks are indexed by the row they are XORed at: T12 before pi12, T31
// before pi31.  A quad of lanes takes one slice.
template <bool VEC>
__device__ __forceinline__ void first_slice(uint64_t t, uint64_t nrows, uint32_t nwords, ChachaKey k12, ChachaKey k31,
                                            const uint32_t* __restrict__ inv12, const uint32_t* __restrict__ inv31,
                                            const uint32_t* __restrict__ g0, const uint32_t* __restrict__ g1,
                                            const uint32_t* __restrict__ g2, uint32_t* __restrict__ o0,
                                            uint32_t* __restrict__ o1, uint32_t* __restrict__ r12,
                                            uint32_t* __restrict__ r31) {
    const uint32_t nb = (nwords + 15) >> 4;
    const uint32_t c = threadIdx.x & 3u;
    const uint64_t sl = t >> 2;
    const uint32_t i = (uint32_t)(sl / nb), b = (uint32_t)(sl - (uint64_t)i * nb);
    const uint32_t len = nwords - 16 * b < 16 ? nwords - 16 * b : 16;
    // The blocks that do not need the load in flight are drawn while it is:
    // T12 while inv12[i] is, R2 and R1 while inv31[j] is.  A quad shares its
    // record, so the exits keep quads whole; they only matter for
    // permutations that were not made by this library, and then leave the
    // row unwritten.
    const uint64_t src = (uint64_t)i * nwords + 16 * b;
    const uint32_t j = inv12[i];
    const uint4 x = load_quarter<VEC>(g0, src, c, len), y = load_quarter<VEC>(g1, src, c, len);
    const uint4 z = load_quarter<VEC>(g2, src, c, len);
    const uint4 t12 = chacha_quad(k12, i, b, kT12, nwords);
    if (j >= nrows) return;
    const uint32_t l = inv31[j];
    const uint4 r2 = chacha_quad(k12, i, b, kR2, nwords), r1 = chacha_quad(k31, i, b, kR1, nwords);
    const uint4 m = xor4(t12, chacha_quad(k31, j, b, kT31, nwords));
    if (l >= nrows) return;
    const uint64_t dst = (uint64_t)l * nwords + 16 * b;
    store_quarter<VEC>(r12, src, c, len, r2);
    store_quarter<VEC>(r31, src, c, len, r1);
    store_quarter<VEC>(o0, dst, c, len, xor4(xor4(x, y), m));
    store_quarter<VEC>(o1, dst, c, len, xor4(z, m));
}

template <bool VEC>
__global__ __launch_bounds__(kBlock) void k_shuffle_first(uint64_t nrows, uint32_t nwords, ChachaKey k12, ChachaKey k31,
                                                        const uint32_t* __restrict__ inv12,
                                                        const uint32_t* __restrict__ inv31,
                                                        const uint32_t* __restrict__ g0,
                                                        const uint32_t* __restrict__ g1,
                                                        const uint32_t* __restrict__ g2, uint32_t* __restrict__ o0,
                                                        uint32_t* __restrict__ o1, uint32_t* __restrict__ r12,
                                                        uint32_t* __restrict__ r31) {
    const uint64_t total = nrows * ((nwords + 15) >> 4) * 4;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x; t < total; t += stride)
        first_slice<VEC>(t, nrows, nwords, k12, k31, inv12, inv31, g0, g1, g2, o0, o1, r12, r31);
}

// Round pi23 as a gather (its outputs are the result shares, written in
// order): with p = perm[i],
//   out[i] = C1 ^ C2, C1 = (g0 ^ T23)[p] ^ R2[i], C2 = (g1 ^ T23)[p] ^ R1[i]
// (CS2's C1 = pi23(X1 ^ T23) ^ R2, CS3's C2 = pi23(pi31(Y1 ^ T31) ^ T23) ^ R1
// and CS2's R3 = C1 ^ C2; with the servers simulated together C1 and C2 are
// not stored).  R1 and R2 are made again from their pairs' keys rather than
// read back.
// open: 0 none; 1 secFetch's flag of each record (bit 0 of word 0); 2 the
// secAccess filter's flag (parity of all bits) of records of at most 16
// words (one slice).  The opened record is R1 ^ R2 ^ R3 = x ^ y, which the
// three servers' exchange reconstructs; the flag of output row i goes to
// flags[i].
template <bool VEC>
__device__ __forceinline__ void final_slice(uint64_t t, uint64_t nrows, uint32_t nwords, ChachaKey k12, ChachaKey k23,
                                            ChachaKey k31, const uint32_t* __restrict__ perm,
                                            const uint32_t* __restrict__ g0, const uint32_t* __restrict__ g1,
                                            uint32_t* __restrict__ out, uint32_t open = 0,
                                            uint32_t* __restrict__ flags = nullptr) {
    const uint32_t nb = (nwords + 15) >> 4;
    const uint32_t c = threadIdx.x & 3u;
    const uint64_t sl = t >> 2;
    const uint32_t i = (uint32_t)(sl / nb), b = (uint32_t)(sl - (uint64_t)i * nb);
    const uint32_t len = nwords - 16 * b < 16 ? nwords - 16 * b : 16;
    const uint32_t p = perm[i];
    // R2 and R1 (indexed by the output row) while the load of p is in flight
    const uint4 r2 = chacha_quad(k12, i, b, kR2, nwords), r1 = chacha_quad(k31, i, b, kR1, nwords);
    if (p >= nrows) {                // as in first_slice
        if (open && b == 0 && c == 0) flags[i] = 0u;
        return;
    }
    const uint64_t src = (uint64_t)p * nwords + 16 * b, dst = (uint64_t)i * nwords + 16 * b;
    const uint4 x = load_quarter<VEC>(g0, src, c, len), y = load_quarter<VEC>(g1, src, c, len);
    const uint4 m = chacha_quad(k23, p, b, kT23, nwords);
    uint4 c1 = xor4(x, m);
    pin(c1);
    c1 = xor4(c1, r2);
    const uint4 c2 = xor4(xor4(y, m), r1);
    store_quarter<VEC>(out, dst, c, len, xor4(c1, c2));
    if (open == 1) {
        if (b == 0 && c == 0) flags[i] = (x.x ^ y.x) & 1u;
    } else if (open == 2) {
        uint32_t acc = (x.x ^ y.x) ^ (x.y ^ y.y) ^ (x.z ^ y.z) ^ (x.w ^ y.w);
        acc ^= quad_from<1>(acc);
        acc ^= quad_from<2>(acc);
        if (c == 0) flags[i] = __builtin_popcount(acc) & 1u;
    }
}

template <bool VEC>
__global__ __launch_bounds__(kBlock) void k_shuffle_final(uint64_t nrows, uint32_t nwords, ChachaKey k12, ChachaKey k23,
                                                        ChachaKey k31, const uint32_t* __restrict__ perm,
                                                        const uint32_t* __restrict__ g0,
                                                        const uint32_t* __restrict__ g1, uint32_t* __restrict__ out,
                                                        uint32_t open, uint32_t* __restrict__ flags) {
    const uint64_t total = nrows * ((nwords + 15) >> 4) * 4;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x; t < total; t += stride)
        final_slice<VEC>(t, nrows, nwords, k12, k23, k31, perm, g0, g1, out, open, flags);
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

// secAccess filter: flag of shuffled record i = parity of all bits of R1 ^ R2 ^ R3
// (1 for a one-hot ID, 0 for a dummy all-zero ID).  A quad of lanes takes a
// record, lane c its 16-byte quarters c, c + 4, ... (with vec: width a
// multiple of 4 words, tables 16-byte aligned; else its words c, c + 4, ...),
// so a wavefront reads 16 consecutive 64-byte records in one access; the
// quad's partial XORs meet through DPP quad moves.
__global__ void k_open_parity(uint64_t nrows, uint32_t nwords, uint32_t vec, const uint32_t* __restrict__ a,
                              const uint32_t* __restrict__ b, const uint32_t* __restrict__ c,
                              uint32_t* __restrict__ flags) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t i = t >> 2;
    if (i >= nrows) return;                         // whole quads leave together
    const uint32_t lane = (uint32_t)t & 3u;
    uint32_t acc = 0;
    if (vec) {
        const uint32_t nq = nwords >> 2;
        const uint64_t base = i * nq;
        for (uint32_t q = lane; q < nq; q += 4) {
            const uint4 v = xor4(xor4(((const uint4*)a)[base + q], ((const uint4*)b)[base + q]),
                                 ((const uint4*)c)[base + q]);
            acc ^= v.x ^ v.y ^ v.z ^ v.w;
        }
    } else {
        for (uint32_t w = lane; w < nwords; w += 4) acc ^= a[i * nwords + w] ^ b[i * nwords + w] ^ c[i * nwords + w];
    }
    acc ^= quad_from<1>(acc);
    acc ^= quad_from<2>(acc);
    if (lane == 0) flags[i] = __builtin_popcount(acc) & 1u;
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

// k_compact for whole records (first = 0) of a width that is a multiple of 4
// words, every table 16-byte aligned: one thread per 16-byte quarter.
__global__ void k_compact_vec(uint64_t nrows, uint32_t nwords, const uint32_t* __restrict__ flags,
                              const uint32_t* __restrict__ pos, const uint4* __restrict__ s0,
                              const uint4* __restrict__ s1, const uint4* __restrict__ s2, uint4* __restrict__ o0,
                              uint4* __restrict__ o1, uint4* __restrict__ o2, uint32_t* __restrict__ rows_out) {
    const uint32_t nq = nwords >> 2;
    const uint64_t total = nrows * nq;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += stride) {
        const uint32_t i = (uint32_t)(k / nq), q = (uint32_t)(k - (uint64_t)i * nq);
        if (!flags[i]) continue;
        const uint64_t d = (uint64_t)pos[i] * nq + q;
        o0[d] = s0[k];
        o1[d] = s1[k];
        o2[d] = s2[k];
        if (q == 0) rows_out[pos[i]] = i;
    }
}

// Tables of at most kSmallPerm records (secAccess shuffles one posting list):
// the open, the exclusive scan of the flags, the compaction and the count in
// one workgroup of 1024 threads.  A wavefront opens a record at a time, its
// lanes over the record's words (the parity of all bits for the secAccess
// filter, bit 0 of word 0 for secFetch); then the kept records' words
// [first, nwords) go to their positions in shuffled order.
__device__ __forceinline__ void open_compact_block(uint32_t n, uint32_t nwords, uint32_t parity,
                                                   const uint32_t* __restrict__ a, const uint32_t* __restrict__ b,
                                                   const uint32_t* __restrict__ c, uint32_t* __restrict__ o0,
                                                   uint32_t* __restrict__ o1, uint32_t* __restrict__ o2,
                                                   uint32_t* __restrict__ rows_out, uint32_t* __restrict__ count,
                                                   uint32_t* flag, uint32_t* incl) {
    const uint32_t t = threadIdx.x, lane = t & 63u, wave = t >> 6;
    flag[t] = 0;
    __syncthreads();
    for (uint32_t i = wave; i < n; i += blockDim.x >> 6) {
        const uint64_t base = (uint64_t)i * nwords;
        uint32_t acc = 0;
        if (parity) {
            for (uint32_t w = lane; w < nwords; w += 64) acc ^= a[base + w] ^ b[base + w] ^ c[base + w];
            for (uint32_t d = 32; d > 0; d >>= 1) acc ^= (uint32_t)__shfl_xor((int)acc, (int)d);
            acc = __builtin_popcount(acc) & 1u;
        } else {
            acc = (a[base] ^ b[base] ^ c[base]) & 1u;
        }
        if (lane == 0) flag[i] = acc;
    }
    __syncthreads();
    const uint32_t f = flag[t];
    incl[t] = f;
    __syncthreads();
    for (uint32_t d = 1; d < kSmallPerm; d <<= 1) {
        const uint32_t x = t >= d ? incl[t - d] : 0u;
        __syncthreads();
        incl[t] += x;
        __syncthreads();
    }
    if (t < n && f) rows_out[incl[t] - 1] = t;
    if (t == 0) *count = incl[kSmallPerm - 1];
    const uint32_t first = parity ? 0u : 1u, ow = nwords - first;
    const uint64_t total = (uint64_t)n * ow;
    for (uint64_t k = t; k < total; k += blockDim.x) {
        const uint32_t i = (uint32_t)(k / ow), w = (uint32_t)(k - (uint64_t)i * ow);
        if (!flag[i]) continue;
        const uint64_t src = (uint64_t)i * nwords + first + w, dst = (uint64_t)(incl[i] - 1) * ow + w;
        o0[dst] = a[src];
        o1[dst] = b[src];
        o2[dst] = c[src];
    }
}

__global__ __launch_bounds__(1024) void k_open_compact_small(uint32_t n, uint32_t nwords, uint32_t parity,
                                                             const uint32_t* __restrict__ a,
                                                             const uint32_t* __restrict__ b,
                                                             const uint32_t* __restrict__ c, uint32_t* __restrict__ o0,
                                                             uint32_t* __restrict__ o1, uint32_t* __restrict__ o2,
                                                             uint32_t* __restrict__ rows_out,
                                                             uint32_t* __restrict__ count) {
    __shared__ uint32_t flag[kSmallPerm];
    __shared__ uint32_t incl[kSmallPerm];
    open_compact_block(n, nwords, parity, a, b, c, o0, o1, o2, rows_out, count, flag, incl);
}

// A whole shuffle of a small table (at most kSmallPerm records and
// kFusedSlices 16-word slices) in one workgroup: the three permutations into
// LDS, the first round (first_slice), the final round (final_slice), and,
// with compact = 1 (secFetch: bit 0 of word 0) or 2 (secAccess filter: parity
// of all bits), the open and compaction of the shuffled table.  The same
// per-slice code as the multi-workgroup launches, so the same shares; the
// rounds meet through global memory (x1, v, out) behind workgroup barriers.
constexpr uint32_t kFusedSlices = 1024;

struct SmallShuffle {
    ChachaKey k12, k23, k31;
    const uint32_t* g[3];
    uint32_t* x1;
    uint32_t* v;
    uint32_t* out[3];              // R1, R2, R3
    uint32_t compact;
    uint32_t* kept[3];
    uint32_t* rows_out;
    uint32_t* count;
};

template <bool VEC>
__global__ __launch_bounds__(1024) void k_shuffle_small(uint32_t n, uint32_t nwords, SmallShuffle A) {
    __shared__ uint64_t key[kSmallPerm];
    __shared__ uint32_t perm[3][kSmallPerm];     // inverse of pi12, inverse of pi31, pi23
    __shared__ uint32_t flag[kSmallPerm];
    __shared__ uint32_t incl[kSmallPerm];
    small_perm(A.k12, kP12, 1u, n, key, perm[0]);
    small_perm(A.k31, kP31, 1u, n, key, perm[1]);
    small_perm(A.k23, kP23, 0u, n, key, perm[2]);
    const uint64_t total = (uint64_t)n * ((nwords + 15) >> 4) * 4;
    for (uint64_t t = threadIdx.x; t < total; t += blockDim.x)
        first_slice<VEC>(t, n, nwords, A.k12, A.k31, perm[0], perm[1], A.g[0], A.g[1], A.g[2], A.x1, A.v, A.out[1],
                         A.out[0]);
    __syncthreads();
    for (uint64_t t = threadIdx.x; t < total; t += blockDim.x)
        final_slice<VEC>(t, n, nwords, A.k12, A.k23, A.k31, perm[2], A.x1, A.v, A.out[2]);
    if (!A.compact) return;
    __syncthreads();
    open_compact_block(n, nwords, A.compact == 2, A.out[0], A.out[1], A.out[2], A.kept[0], A.kept[1], A.kept[2],
                       A.rows_out, A.count, flag, incl);
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

// Workspace of the permutations' scratch: for each of the three (they are
// made side by side) rotated keys in and out, row numbers in and out, run
// starts and the sort's temporary storage.
uint64_t perm_scratch_bytes(uint64_t nrows) {
    auto r = [](uint64_t b) { return (b + 255) & ~255ull; };
    return 3 * (2 * r(nrows * 8) + 2 * r(nrows * 4) + r(((1ull << run_bits(nrows)) + 1) * 4) +
                r(sort_temp_bytes(nrows)));
}

// rss_shuffle: X1 and pi31(Y1 ^ T31), three permutations and their scratch.
uint64_t shuffle_ws(uint64_t nrows, uint32_t nwords) {
    auto r = [](uint64_t b) { return (b + 255) & ~255ull; };
    return 2 * r(nrows * nwords * 4) + 3 * r(nrows * 4) + perm_scratch_bytes(nrows) + 4096;
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

// One permutation in four steps (keys, radix pass, run starts, ranking), so
// that the three permutations of a shuffle can be enqueued step by step on
// their streams: each stream then has work as soon as possible, instead of
// after the host has enqueued the whole of the ones before it.
struct PermJob {
    ChachaKey pk;
    uint32_t p;
    bool inverse;
    uint32_t* perm;
    PermScratch w;
    hipStream_t s;
};

uint32_t ceil_log2(uint64_t n) {
    uint32_t lg = 0;
    while ((1ull << lg) < n) lg++;
    return lg;
}

// Bucket bits d1 of the bucket method: 2^11 .. 2^12 rows per bucket on average.
uint32_t bucket_bits(uint64_t nrows) {
    const uint32_t lg = ceil_log2(nrows);
    return lg > 12 ? lg - 12 : 0;
}

// The method a permutation of nrows rows takes (tables of at most 1024 rows
// take k_perm_small whatever it is).
uint32_t perm_method(uint64_t nrows, uint32_t m) {
    if (m >= kPermBuckets && nrows > kBucketMaxRows) return kPermRadix;
    return m;
}

// The bucket method for all three permutations at once, five launches on
// stream s (blockIdx.y picks the permutation).
int bucket_perms(uint64_t nrows, const PermJob (&jobs)[3], uint32_t method, hipStream_t s) {
    const uint32_t hb = run_bits(nrows), d1 = bucket_bits(nrows), nb = 1u << d1;
    const uint32_t nblk = (uint32_t)((nrows + kChunkRows - 1) / kChunkRows);
    // scratch of each permutation: keys and rows placed by bucket in keys /
    // idx, per-workgroup counts in keys_sorted, bucket totals and starts in
    // idx_sorted; they fit for every table the method takes
    if ((uint64_t)nb * nblk > 2 * nrows || 2ull * nb + 1 > nrows || nblk > 1024)
        return fail(FSS_EDEVICE, "rss_shuffle: bucket scratch does not fit");
    BucketSet S{};
    for (int q = 0; q < 3; q++) {
        const PermScratch& w = jobs[q].w;
        S.pk[q] = jobs[q].pk;
        S.p[q] = jobs[q].p;
        S.inverse[q] = jobs[q].inverse ? 1u : 0u;
        S.perm[q] = jobs[q].perm;
        S.skeys[q] = w.keys;
        S.srows[q] = w.idx;
        S.counts[q] = (uint32_t*)w.keys_sorted;
        S.totals[q] = w.idx_sorted;
        S.starts[q] = w.idx_sorted + nb;
    }
    hipLaunchKernelGGL(k_perm_count, dim3(nblk, 3), dim3(1024), 0, s, nrows, d1, nblk, S);
    if (int rc = check_launch("k_perm_count")) return rc;
    hipLaunchKernelGGL(k_bucket_offsets, dim3(nb, 3), dim3(256), 0, s, nblk, S);
    if (int rc = check_launch("k_bucket_offsets")) return rc;
    hipLaunchKernelGGL(k_bucket_starts, dim3(1, 3), dim3(256), 0, s, nb, S);
    if (int rc = check_launch("k_bucket_starts")) return rc;
    hipLaunchKernelGGL(k_perm_place, dim3(nblk, 3), dim3(1024), 0, s, nrows, d1, nblk, S);
    if (int rc = check_launch("k_perm_place")) return rc;
    hipLaunchKernelGGL(k_bucket_rank, dim3(nb, 3), dim3(1024), 0, s, nrows, hb, d1, method - kPermBuckets, S);
    return check_launch("k_bucket_rank");
}

int perm_step(int step, uint64_t nrows, const PermJob& j, uint32_t method) {
    const uint32_t hb = run_bits(nrows);
    const PermScratch& w = j.w;
    // with no run-id bits there is one run, already in row order: no sort
    const uint64_t* keys = hb ? w.keys_sorted : w.keys;
    const uint32_t* rows = hb ? w.idx_sorted : w.idx;
    const uint64_t nruns = 1ull << hb;
    switch (step) {
        case 0:
            hipLaunchKernelGGL(k_perm_keys, dim3(slice_grid((nrows + 7) / 8 * 4)), dim3(kBlock), 0, j.s, j.pk, j.p,
                               nrows, hb, w.keys, w.idx);
            return check_launch("k_perm_keys");
        case 1: {
            if (!hb) return 0;
            size_t temp_bytes = w.temp_bytes;
            if (hipcub::DeviceRadixSort::SortPairs(w.temp, temp_bytes, w.keys, w.keys_sorted, w.idx, w.idx_sorted,
                                                   (int)nrows, 0, (int)hb, j.s) != hipSuccess)
                return fail(FSS_EDEVICE, "rss_shuffle: radix sort failed");
            return 0;
        }
        case 2:
            hipLaunchKernelGGL(k_run_starts, dim3(grid_of(nrows + 1, 256)), dim3(256), 0, j.s, nrows, hb, keys,
                               w.starts);
            return check_launch("k_run_starts");
        default:
            hipLaunchKernelGGL(k_rank_runs, dim3(grid_of(nruns * 64, 256)), dim3(256), 0, j.s, nrows, hb,
                               (uint32_t)j.inverse, (uint32_t)(method == kPermRadix), w.starts, keys, rows, j.perm);
            return check_launch("k_rank_runs");
    }
}

// The 16-byte path needs the width a multiple of 4 words and every table
// 16-byte aligned.
bool vec_quarters(uint32_t nwords, std::initializer_list<const void*> tables) {
    if (nwords & 3u) return false;
    for (const void* t : tables)
        if (!aligned16(t)) return false;
    return true;
}

int shuffle_first(uint64_t nrows, uint32_t nwords, ChachaKey k12, ChachaKey k31, const uint32_t* inv12,
                  const uint32_t* inv31, const uint32_t* g0, const uint32_t* g1, const uint32_t* g2, uint32_t* o0,
                  uint32_t* o1, uint32_t* r12, uint32_t* r31, hipStream_t s) {
    const unsigned grid = slice_grid(nrows * ((nwords + 15) / 16) * 4);
    if (vec_quarters(nwords, {g0, g1, g2, o0, o1, r12, r31}))
        hipLaunchKernelGGL(k_shuffle_first<true>, dim3(grid), dim3(kBlock), 0, s, nrows, nwords, k12, k31, inv12,
                           inv31, g0, g1, g2, o0, o1, r12, r31);
    else
        hipLaunchKernelGGL(k_shuffle_first<false>, dim3(grid), dim3(kBlock), 0, s, nrows, nwords, k12, k31, inv12,
                           inv31, g0, g1, g2, o0, o1, r12, r31);
    return check_launch("k_shuffle_first");
}

int shuffle_final(uint64_t nrows, uint32_t nwords, ChachaKey k12, ChachaKey k23, ChachaKey k31, const uint32_t* perm,
                  const uint32_t* g0, const uint32_t* g1, uint32_t* out, uint32_t open, uint32_t* flags,
                  hipStream_t s) {
    const unsigned grid = slice_grid(nrows * ((nwords + 15) / 16) * 4);
    if (vec_quarters(nwords, {g0, g1, out}))
        hipLaunchKernelGGL(k_shuffle_final<true>, dim3(grid), dim3(kBlock), 0, s, nrows, nwords, k12, k23, k31, perm,
                           g0, g1, out, open, flags);
    else
        hipLaunchKernelGGL(k_shuffle_final<false>, dim3(grid), dim3(kBlock), 0, s, nrows, nwords, k12, k23, k31, perm,
                           g0, g1, out, open, flags);
    return check_launch("k_shuffle_final");
}

// Two streams of the library's own per device (default priority,
// non-blocking) on which the permutations pi31 and pi23 are made while pi12
// is made on the caller's stream: the permutations are independent, and most
// of their kernels are small or latency-bound.  Ordered against the caller's
// stream with events only; nullptr if they cannot be created (then all runs
// on the caller's stream).
std::mutex g_stream_mu;
std::map<int, std::array<hipStream_t, 2>> g_streams;

hipStream_t perm_stream(int i) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lock(g_stream_mu);
    auto it = g_streams.find(dev);
    if (it == g_streams.end()) {
        std::array<hipStream_t, 2> st{nullptr, nullptr};
        for (auto& x : st)
            if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) x = nullptr;
        it = g_streams.emplace(dev, st).first;
    }
    return it->second[i];
}

// The three permutations of a shuffle.  pi12 and pi31 are written as their
// inverses (the first launch scatters through them), pi23 as is (the final
// launch gathers through it).  The bucket method makes all three in one
// launch sequence on the caller's stream.  The radix methods make them side
// by side: pi12 on the caller's stream, pi31 and pi23 on the library's two
// streams (after everything already on the caller's stream); join(i) makes
// the caller's stream wait for pi31 (i = 0) or pi23 (i = 1), every join is
// enqueued whatever happened before it, and finish() must follow, so that no
// work on the library's streams outlives the caller's view of the call.
struct PermSet {
    hipStream_t s;
    hipStream_t side[2] = {nullptr, nullptr};
    hipEvent_t fork = nullptr, done[2] = {nullptr, nullptr};
    bool forked = false, recorded[2] = {true, true};
    int rc = 0;

    void begin(uint64_t nrows, const uint64_t seeds[3], uint32_t* inv12, uint32_t* inv31, uint32_t* p23, Carve& ws) {
        PermScratch pw[3];
        for (PermScratch& w : pw) {
            w.keys = ws.take<uint64_t>(nrows);
            w.keys_sorted = ws.take<uint64_t>(nrows);
            w.idx = ws.take<uint32_t>(nrows);
            w.idx_sorted = ws.take<uint32_t>(nrows);
            w.starts = ws.take<uint32_t>((1ull << run_bits(nrows)) + 1);
            w.temp_bytes = sort_temp_bytes(nrows);
            w.temp = ws.take<uint8_t>(w.temp_bytes);
        }
        if (!ws.ok) {
            rc = fail(FSS_ENOMEM, "rss_shuffle: workspace too small");
            return;
        }
        if (nrows <= kSmallPerm) {
            // one launch on the caller's stream: no sort, no side streams
            SmallPerms J{};
            const uint64_t sd[3] = {seeds[0], seeds[2], seeds[1]};
            const uint32_t pid[3] = {kP12, kP31, kP23}, inv[3] = {1, 1, 0};
            uint32_t* outs[3] = {inv12, inv31, p23};
            for (int q = 0; q < 3; q++) {
                J.pk[q] = pair_key(sd[q]);
                J.p[q] = pid[q];
                J.inverse[q] = inv[q];
                J.out[q] = outs[q];
            }
            hipLaunchKernelGGL(k_perm_small, dim3(3), dim3(1024), 0, s, (uint32_t)nrows, J);
            rc = check_launch("k_perm_small");
            return;
        }
        const uint32_t method = perm_method(nrows, g_perm_method.load());
        // pair seeds: s12 -> pi12, T12, R2; s23 -> pi23, T23; s31 -> pi31, T31, R1
        if (method >= kPermBuckets) {
            // the three permutations together, on the caller's stream (so also
            // under stream capture: no sort library, no memset nodes)
            const PermJob jobs[3] = {{pair_key(seeds[0]), kP12, true, inv12, pw[0], s},
                                     {pair_key(seeds[2]), kP31, true, inv31, pw[1], s},
                                     {pair_key(seeds[1]), kP23, false, p23, pw[2], s}};
            rc = bucket_perms(nrows, jobs, method, s);
            return;
        }
        // the radix methods: one permutation per stream, the caller's and the
        // library's two; not under stream capture (their radix passes clear
        // buffers with memset operations)
        hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
        if (s && hipStreamIsCapturing(s, &capture) == hipSuccess && capture != hipStreamCaptureStatusNone) {
            rc = fail(FSS_EUNSUPPORTED, "rss_shuffle: under stream capture at most 2^23 rows (bucket permutations)");
            return;
        }
        side[0] = perm_stream(0), side[1] = perm_stream(1);
        forked = side[0] && side[1] && hipEventCreateWithFlags(&fork, hipEventDisableTiming) == hipSuccess &&
                 hipEventCreateWithFlags(&done[0], hipEventDisableTiming) == hipSuccess &&
                 hipEventCreateWithFlags(&done[1], hipEventDisableTiming) == hipSuccess &&
                 hipEventRecord(fork, s) == hipSuccess && hipStreamWaitEvent(side[0], fork, 0) == hipSuccess &&
                 hipStreamWaitEvent(side[1], fork, 0) == hipSuccess;
        const hipStream_t s31 = forked ? side[0] : s, s23 = forked ? side[1] : s;
        const PermJob jobs[3] = {{pair_key(seeds[0]), kP12, true, inv12, pw[0], s},
                                 {pair_key(seeds[2]), kP31, true, inv31, pw[1], s31},
                                 {pair_key(seeds[1]), kP23, false, p23, pw[2], s23}};
        int prc[3] = {0, 0, 0};
        for (int step = 0; step < 4; step++)
            for (int q = 0; q < 3; q++)
                if (!prc[q]) prc[q] = perm_step(step, nrows, jobs[q], method);
        if (forked) {
            recorded[0] = hipEventRecord(done[0], s31) == hipSuccess;
            recorded[1] = hipEventRecord(done[1], s23) == hipSuccess;
        }
        rc = prc[0] ? prc[0] : prc[1] ? prc[1] : prc[2];
    }

    void join(int i) {
        if (!forked) return;
        if (recorded[i] && hipStreamWaitEvent(s, done[i], 0) == hipSuccess) return;
        (void)hipStreamSynchronize(side[i]);
        if (!rc) rc = fail(FSS_EDEVICE, "rss_shuffle: stream join failed");
    }

    void finish() {
        for (hipEvent_t e : {fork, done[0], done[1]})
            if (e) (void)hipEventDestroy(e);
    }
};

// The data-dependent part of Alg. 5 (all three servers simulated), given the
// permutations: out[0..2] = R1, R2, R3.  x1 and v are workspace tables.
// open / flags: the final round's optional open (final_slice).
int shuffle_rounds(uint64_t nrows, uint32_t nwords, const uint32_t* const d[3], const uint64_t seeds[3],
                   const uint32_t* inv12, const uint32_t* inv31, const uint32_t* p23, uint32_t* x1, uint32_t* v,
                   uint32_t* const out[3], hipStream_t s, PermSet* pending, uint32_t open = 0,
                   uint32_t* flags = nullptr) {
    const ChachaKey k12 = pair_key(seeds[0]), k23 = pair_key(seeds[1]), k31 = pair_key(seeds[2]);
    // pi12 then pi31: CS1's X1, CS3's pi31(Y1 ^ T31); R2 and R1 drawn
    if (pending) pending->join(0);
    int rc = pending ? pending->rc : 0;
    if (!rc) rc = shuffle_first(nrows, nwords, k12, k31, inv12, inv31, d[0], d[1], d[2], x1, v, out[1], out[0], s);
    // pi23: CS2's C1 = pi23(X1 ^ T23) ^ R2, CS3's C2 = pi23(pi31(Y1 ^ T31) ^ T23) ^ R1,
    // R3 = C1 ^ C2
    if (pending) {
        pending->join(1);
        if (!rc) rc = pending->rc;
    }
    if (!rc) rc = shuffle_final(nrows, nwords, k12, k23, k31, p23, x1, v, out[2], open, flags, s);
    return rc;
}

// Alg. 5 with all three servers simulated; out[0..2] = R1, R2, R3.  The
// permutation pi23 is still being made while the first launch runs.
// Whether a shuffle runs in one workgroup (k_shuffle_small).
bool fused_shuffle(uint64_t nrows, uint32_t nwords) {
    return nrows <= kSmallPerm && nrows * ((nwords + 15) / 16) <= kFusedSlices;
}

// The one-workgroup shuffle; compact: 0 none, 1 secFetch's open, 2 the
// secAccess filter's (then kept / rows_out / count receive the compaction).
int launch_fused(uint64_t nrows, uint32_t nwords, const uint32_t* const d[3], const uint64_t seeds[3],
                 uint32_t* const out[3], uint32_t* x1, uint32_t* v, uint32_t compact, uint32_t* const kept[3],
                 uint32_t* rows_out, uint32_t* count, hipStream_t s) {
    SmallShuffle A{};
    A.k12 = pair_key(seeds[0]), A.k23 = pair_key(seeds[1]), A.k31 = pair_key(seeds[2]);
    for (int i = 0; i < 3; i++) {
        A.g[i] = d[i];
        A.out[i] = out[i];
        A.kept[i] = kept ? kept[i] : nullptr;
    }
    A.x1 = x1, A.v = v, A.compact = compact, A.rows_out = rows_out, A.count = count;
    if (vec_quarters(nwords, {d[0], d[1], d[2], x1, v, out[0], out[1], out[2]}))
        hipLaunchKernelGGL(k_shuffle_small<true>, dim3(1), dim3(1024), 0, s, (uint32_t)nrows, nwords, A);
    else
        hipLaunchKernelGGL(k_shuffle_small<false>, dim3(1), dim3(1024), 0, s, (uint32_t)nrows, nwords, A);
    return check_launch("k_shuffle_small");
}

int run_shuffle(uint64_t nrows, uint32_t nwords, const uint32_t* const d[3], const uint64_t seeds[3],
                uint32_t* const out[3], Carve& ws, hipStream_t s, uint32_t open = 0, uint32_t* flags = nullptr) {
    const uint64_t tw = nrows * nwords;
    uint32_t* x1 = ws.take<uint32_t>(tw);      // CS1 -> CS2: X1
    uint32_t* v = ws.take<uint32_t>(tw);       // CS3: pi31(Y1 ^ T31)
    uint32_t* inv12 = ws.take<uint32_t>(nrows);
    uint32_t* inv31 = ws.take<uint32_t>(nrows);
    uint32_t* p23 = ws.take<uint32_t>(nrows);
    if (!ws.ok) return fail(FSS_ENOMEM, "rss_shuffle: workspace too small");
    if (fused_shuffle(nrows, nwords)) return launch_fused(nrows, nwords, d, seeds, out, x1, v, 0, nullptr, nullptr, nullptr, s);
    PermSet ps{s};
    ps.begin(nrows, seeds, inv12, inv31, p23, ws);
    const int rc = shuffle_rounds(nrows, nwords, d, seeds, inv12, inv31, p23, x1, v, out, s, &ps, open, flags);
    ps.finish();
    return rc;
}

}  // namespace

namespace ogm {

// The shuffle's own streams, for fss_shutdown: each is drained, then
// destroyed; the next shuffle creates them again.
int shuffle_release() {
    std::lock_guard<std::mutex> lock(g_stream_mu);
    int rc = FSS_OK;
    for (auto& kv : g_streams)
        for (hipStream_t& st : kv.second) {
            if (st && (hipStreamSynchronize(st) != hipSuccess || hipStreamDestroy(st) != hipSuccess)) rc = FSS_EDEVICE;
            st = nullptr;
        }
    g_streams.clear();
    return rc;
}

}  // namespace ogm

namespace {

// secFetch's table {x || id || d} (Alg. 4): record c of share i is the
// predicate bit c of share i in bit 0 of word 0, then id record c (wi words),
// then value record c (wv words).  One thread per output word.
struct FetchTableArgs {
    const uint32_t* bits[3];
    const uint32_t* ids[3];
    const uint32_t* vals[3];
    uint32_t* out[3];
};

__global__ void k_fetch_table(uint64_t ncand, uint32_t wi, uint32_t wv, FetchTableArgs A) {
    const uint64_t W = 1ull + wi + wv, total = ncand * W;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
        const uint64_t c = g / W;
        const uint32_t w = (uint32_t)(g - c * W);
#pragma unroll
        for (int i = 0; i < 3; i++) {
            uint32_t v;
            if (w == 0)
                v = (A.bits[i][c >> 5] >> (c & 31u)) & 1u;
            else if (w <= wi)
                v = A.ids[i][c * wi + (w - 1)];
            else
                v = A.vals[i][c * wv + (w - 1 - wi)];
            A.out[i][g] = v;
        }
    }
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

uint64_t rss_shuffle_prepare_workspace_bytes(uint64_t nrows) {
    if (nrows == 0) return 0;
    return perm_scratch_bytes(nrows) + 4096;
}

int rss_shuffle_prepare(uint64_t nrows, const uint64_t seeds[3], uint32_t* d_perms, void* d_work, uint64_t work_bytes,
                        void* stream) {
    last_error().clear();
    if (nrows == 0) return FSS_OK;
    if (nrows > 0x7FFFFFFFull) return fail(FSS_EUNSUPPORTED, "rss_shuffle_prepare: more than 2^31 rows");
    if (!seeds || !d_perms) return fail(FSS_EINVAL, "rss_shuffle_prepare: NULL argument");
    if (!d_work || work_bytes < rss_shuffle_prepare_workspace_bytes(nrows))
        return fail(FSS_ENOMEM, "rss_shuffle_prepare: workspace needs %llu bytes",
                    (unsigned long long)rss_shuffle_prepare_workspace_bytes(nrows));
    Carve ws{(uint8_t*)d_work, work_bytes};
    PermSet ps{(hipStream_t)stream};
    ps.begin(nrows, seeds, d_perms, d_perms + nrows, d_perms + 2 * nrows, ws);
    ps.join(0);
    ps.join(1);
    ps.finish();
    return ps.rc;
}

uint64_t rss_shuffle_prepared_workspace_bytes(uint64_t nrows, uint32_t nwords) {
    if (nrows == 0 || nwords == 0) return 0;
    return 2 * ((nrows * nwords * 4 + 255) & ~255ull) + 4096;
}

int rss_shuffle_prepared(uint64_t nrows, uint32_t nwords, const uint32_t* const d_in[3], const uint64_t seeds[3],
                         const uint32_t* d_perms, uint32_t* const d_out[3], void* d_work, uint64_t work_bytes,
                         void* stream) {
    last_error().clear();
    if (nrows == 0 || nwords == 0) return FSS_OK;
    if (nrows > 0x7FFFFFFFull) return fail(FSS_EUNSUPPORTED, "rss_shuffle_prepared: more than 2^31 rows");
    if (!d_in || !d_out || !seeds || !d_perms) return fail(FSS_EINVAL, "rss_shuffle_prepared: NULL argument");
    for (int i = 0; i < 3; i++)
        if (!d_in[i] || !d_out[i]) return fail(FSS_EINVAL, "rss_shuffle_prepared: NULL share %d", i);
    if (!d_work || work_bytes < rss_shuffle_prepared_workspace_bytes(nrows, nwords))
        return fail(FSS_ENOMEM, "rss_shuffle_prepared: workspace needs %llu bytes",
                    (unsigned long long)rss_shuffle_prepared_workspace_bytes(nrows, nwords));
    Carve ws{(uint8_t*)d_work, work_bytes};
    const uint64_t tw = nrows * nwords;
    uint32_t* x1 = ws.take<uint32_t>(tw);
    uint32_t* v = ws.take<uint32_t>(tw);
    if (!ws.ok) return fail(FSS_ENOMEM, "rss_shuffle_prepared: workspace too small");
    return shuffle_rounds(nrows, nwords, d_in, seeds, d_perms, d_perms + nrows, d_perms + 2 * nrows, x1, v, d_out,
                          (hipStream_t)stream, nullptr);
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

int rss_fetch_table(uint64_t ncand, const uint32_t* const d_bits[3], uint32_t id_words, const uint32_t* const d_ids[3],
                    uint32_t val_words, const uint32_t* const d_vals[3], uint32_t* const d_out[3], void* stream) {
    last_error().clear();
    if (ncand == 0) return FSS_OK;
    if (!d_bits || !d_out || (id_words && !d_ids) || (val_words && !d_vals))
        return fail(FSS_EINVAL, "rss_fetch_table: NULL argument");
    if ((uint64_t)id_words + val_words + 1 > 65535)
        return fail(FSS_EUNSUPPORTED, "rss_fetch_table: more than 65535 words per record");
    if (ncand > 0xFFFFFFFFull) return fail(FSS_EUNSUPPORTED, "rss_fetch_table: more than 2^32 candidates");
    FetchTableArgs A{};
    for (int i = 0; i < 3; i++) {
        if (!d_bits[i] || !d_out[i] || (id_words && !d_ids[i]) || (val_words && !d_vals[i]))
            return fail(FSS_EINVAL, "rss_fetch_table: NULL share %d", i);
        A.bits[i] = d_bits[i];
        A.ids[i] = id_words ? d_ids[i] : nullptr;
        A.vals[i] = val_words ? d_vals[i] : nullptr;
        A.out[i] = d_out[i];
    }
    const uint64_t total = ncand * (1ull + id_words + val_words);
    hipLaunchKernelGGL(k_fetch_table, dim3(grid_of(total, 256)), dim3(256), 0, (hipStream_t)stream, ncand, id_words,
                       val_words, A);
    return check_launch("k_fetch_table");
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
    int rc = 0;
    if (ncand == 0) {
        hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, (uint64_t)1, d_count);
        return check_launch("k_zero");
    }
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
    if (fused_shuffle(ncand, nwords)) {
        // the shuffle, the open and the compaction in one workgroup
        const uint64_t tw = ncand * nwords;
        uint32_t* x1 = ws.take<uint32_t>(tw);
        uint32_t* v = ws.take<uint32_t>(tw);
        if (!ws.ok) return fail(FSS_ENOMEM, "%s: workspace too small", who);
        return launch_fused(ncand, nwords, d_table, seeds, sh, x1, v, parity ? 2u : 1u, d_out, d_rows_out, d_count, s);
    }
    const bool small = ncand <= kSmallPerm;
    // the final round opens secFetch's bit, and the secAccess filter's parity
    // of records of one slice; wider records are opened by k_open_parity
    const uint32_t open = small ? 0u : !parity ? 1u : nwords <= 16 ? 2u : 0u;
    rc = run_shuffle(ncand, nwords, d_table, seeds, sh, ws, s, open, flags);
    if (rc) return rc;
    if (small) {
        hipLaunchKernelGGL(k_open_compact_small, dim3(1), dim3(kSmallPerm), 0, s, (uint32_t)ncand, nwords,
                           (uint32_t)parity, sh[0], sh[1], sh[2], d_out[0], d_out[1], d_out[2], d_rows_out, d_count);
        return check_launch("k_open_compact_small");
    }
    if (!open) {
        hipLaunchKernelGGL(k_open_parity, dim3((unsigned)((4 * ncand + 255) / 256)), dim3(256), 0, s, ncand, nwords,
                           (uint32_t)((nwords & 3u) == 0 && aligned16(sh[0]) && aligned16(sh[1]) && aligned16(sh[2])),
                           sh[0], sh[1], sh[2], flags);
        rc = check_launch("k_open_parity");
        if (rc) return rc;
    }
    if (hipcub::DeviceScan::ExclusiveSum(scan_tmp, scan, flags, pos, (int)ncand, s) != hipSuccess)
        return fail(FSS_EDEVICE, "%s: scan failed", who);
    if (parity && (nwords & 3u) == 0 && aligned16(sh[0]) && aligned16(sh[1]) && aligned16(sh[2]) &&
        aligned16(d_out[0]) && aligned16(d_out[1]) && aligned16(d_out[2]))
        hipLaunchKernelGGL(k_compact_vec, dim3(grid_of(ncand * (nwords >> 2), 256)), dim3(256), 0, s, ncand, nwords,
                           flags, pos, (const uint4*)sh[0], (const uint4*)sh[1], (const uint4*)sh[2],
                           (uint4*)d_out[0], (uint4*)d_out[1], (uint4*)d_out[2], d_rows_out);
    else
        hipLaunchKernelGGL(k_compact, dim3(grid_of(ncand * (nwords - (parity ? 0u : 1u)), 256)), dim3(256), 0, s,
                           ncand, nwords, parity ? 0u : 1u, flags, pos, sh[0], sh[1], sh[2], d_out[0], d_out[1],
                           d_out[2], d_rows_out);
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

int rss_set_shuffle_tuning(uint32_t perm_method) {
    last_error().clear();
    if (perm_method > kPermBucketsPairs) return fail(FSS_EINVAL, "rss_set_shuffle_tuning: perm_method is 0 .. 4");
    g_perm_method.store(perm_method);
    return FSS_OK;
}

int rss_get_shuffle_tuning(uint32_t* perm_method) {
    last_error().clear();
    if (perm_method) *perm_method = g_perm_method.load();
    return FSS_OK;
}

}  // extern "C"
