// access.hip -- the paper's graph encoding with k-groups (Alg. 1) and secure
// neighbouring-vertex access (Alg. 6) over it.
//
//   rss_group_k            host: Alg. 1's degree protection (padded lengths)
//   k_place_ids,
//   k_split_records        one-hot posting records in CSR order, split into
//                          binary RSS with the ChaCha12 PRF     (HBM stream)
//   k_csr_select           P_m[l] = XOR_c id_m[c] AND id_{c,l}  (HBM stream, 16-byte loads, XOR atomics)
//   k_attr_select          d = XOR_x id[x] AND d_x per kept ID  (HBM stream, XOR atomics)
// rss_sec_access chains the selection, the RSS re-share, the shuffle with the
// parity open and compaction (shuffle.hip) and the attribute selection.
//
// Selections: a block takes a run of candidates and a tile of record words on
// consecutive threads (coalesced); the partials of one word meet in LDS and
// one atomicXor per word and share goes to the zeroed output.  XOR is
// order-free, so results do not depend on scheduling.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "../../include/oblivgm_fss.h"
#include "chacha_gfx950.hpp"
#include "common.hpp"

using namespace ogm;

namespace {

constexpr int kSelBlock = 256;

unsigned blocks_for(uint64_t n, unsigned block, uint64_t cap) {
    uint64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

__global__ void k_fill(uint64_t n, uint32_t v, uint32_t* __restrict__ p) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) p[k] = v;
}

// rec_id[off[v] + slot[e]] = adj[e] for the true IDs e of vertex v (a slot
// outside the padded list, or an ID outside [0, x_bits), is skipped).
__global__ void k_place_ids(uint64_t n, uint32_t x_bits, const uint32_t* __restrict__ adj_off,
                            const uint32_t* __restrict__ adj, const uint32_t* __restrict__ slot,
                            const uint32_t* __restrict__ off, uint32_t* __restrict__ rec_id) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const uint32_t len = off[v + 1] - off[v];
        for (uint32_t e = adj_off[v]; e < adj_off[v + 1]; e++)
            if (slot[e] < len && adj[e] < x_bits) rec_id[off[v] + slot[e]] = adj[e];
    }
}

// Thread m owns words 4m .. 4m+3 of the record table (row-major), lane m & 3
// of the quad that makes PRF block m / 4 of both split keys; share 1 and 2
// are those PRF words, share 3 the one-hot record ^ both.  VEC: the record
// width is a multiple of four words and the shares are 16-byte aligned, so a
// thread's four words lie in one record (one division, one ID read) and go
// out as one 16-byte store per share.
template <bool VEC>
__global__ __launch_bounds__(256) void k_split_records(uint64_t nwords_total, uint32_t wx,
                                                       const uint32_t* __restrict__ rec_id, ChachaKey ka,
                                                       ChachaKey kb, uint32_t counter, uint32_t* __restrict__ s0,
                                                       uint32_t* __restrict__ s1, uint32_t* __restrict__ s2) {
    const uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint4 fa = chacha_quad(ka, (uint32_t)(m >> 2), counter, 0u, 0u);
    const uint4 fb = chacha_quad(kb, (uint32_t)(m >> 2), counter, 0u, 0u);
    if constexpr (VEC) {
        if (4 * m >= nwords_total) return;
        const uint64_t r = 4 * m / wx;
        const uint32_t w0 = (uint32_t)(4 * m - r * wx), x = rec_id[r];
        const uint32_t d = (x >> 5) - w0, bit = x != 0xFFFFFFFFu && d < 4u ? 1u << (x & 31u) : 0u;
        const uint4 plain = make_uint4(d == 0 ? bit : 0u, d == 1 ? bit : 0u, d == 2 ? bit : 0u, d == 3 ? bit : 0u);
        ((uint4*)s0)[m] = fa;
        ((uint4*)s1)[m] = fb;
        ((uint4*)s2)[m] = make_uint4(plain.x ^ fa.x ^ fb.x, plain.y ^ fa.y ^ fb.y, plain.z ^ fa.z ^ fb.z,
                                     plain.w ^ fa.w ^ fb.w);
    } else {
        const uint32_t a[4] = {fa.x, fa.y, fa.z, fa.w}, b[4] = {fb.x, fb.y, fb.z, fb.w};
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const uint64_t g = 4 * m + q;
            if (g >= nwords_total) break;
            const uint64_t r = g / wx;
            const uint32_t w = (uint32_t)(g - r * wx), x = rec_id[r];
            const uint32_t plain = (x != 0xFFFFFFFFu && (x >> 5) == w) ? 1u << (x & 31u) : 0u;
            s0[g] = a[q];
            s1[g] = b[q];
            s2[g] = plain ^ a[q] ^ b[q];
        }
    }
}

// Three-out-of-three product of one word: x_i r_i ^ x_i r_j ^ x_j r_i, j = i + 1.
__device__ __forceinline__ void rss_product(const uint32_t m[3], const uint32_t r[3], uint32_t acc[3]) {
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const int j = (i + 1) % 3;
        acc[i] ^= (r[i] & m[i]) ^ (r[j] & m[i]) ^ (r[i] & m[j]);
    }
}

// Partials of the threads of a tile (tw words, `lanes` candidate lanes) meet
// in LDS; one atomicXor per word and share.
__device__ __forceinline__ void reduce_out(uint32_t (*part)[kSelBlock], const uint32_t acc[3], uint32_t tw,
                                           uint32_t lanes, uint32_t* const out[3], uint64_t base) {
    const uint32_t t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 3; i++) part[i][t] = acc[i];
    __syncthreads();
    if (t < tw) {
#pragma unroll
        for (int i = 0; i < 3; i++) {
            uint32_t v = 0;
            for (uint32_t k = 0; k < lanes; k++) v ^= part[i][k * tw + t];
            if (v) atomicXor(&out[i][base + t], v);
        }
    }
    __syncthreads();
}

struct Shares3 {
    const uint32_t* p[3];
};
struct Out3 {
    uint32_t* p[3];
};

// Zeroes n words of each of three buffers (one launch for the three shares).
__global__ void k_zero3(uint64_t n, Out3 o) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        o.p[0][k] = 0u;
        o.p[1][k] = 0u;
        o.p[2][k] = 0u;
    }
}

// Slot l = blockIdx.y of the fetched list: XOR over this block's candidates c
// with l < len_c of id_m[c] AND record (off_c + l), into out[.][l * wx + w].
// First the block lists in LDS the candidates whose (public, padded) list
// reaches slot l, with their three mask bits; then its threads stream those
// records, V words (16 bytes for V = 4) per load and two records per step, so
// that each lane keeps six loads in flight.  At most kSelCand candidates per
// block (the host sizes the grid for it).
constexpr uint32_t kSelCand = 512;

template <int V>
struct SelVec;
template <>
struct SelVec<1> {
    using T = uint32_t;
    static __device__ __forceinline__ T zero() { return 0u; }
    static __device__ __forceinline__ void prod(const uint32_t m[3], const T r[3], T acc[3]) { rss_product(m, r, acc); }
    static __device__ __forceinline__ uint32_t word(const T& v, int) { return v; }
};
template <>
struct SelVec<4> {
    using T = uint4;
    static __device__ __forceinline__ T zero() { return make_uint4(0u, 0u, 0u, 0u); }
    static __device__ __forceinline__ void prod(const uint32_t m[3], const T r[3], T acc[3]) {
#pragma unroll
        for (int i = 0; i < 3; i++) {
            const int j = (i + 1) % 3;
            acc[i].x ^= (r[i].x & m[i]) ^ (r[j].x & m[i]) ^ (r[i].x & m[j]);
            acc[i].y ^= (r[i].y & m[i]) ^ (r[j].y & m[i]) ^ (r[i].y & m[j]);
            acc[i].z ^= (r[i].z & m[i]) ^ (r[j].z & m[i]) ^ (r[i].z & m[j]);
            acc[i].w ^= (r[i].w & m[i]) ^ (r[j].w & m[i]) ^ (r[i].w & m[j]);
        }
    }
    static __device__ __forceinline__ uint32_t word(const T& v, int q) {
        return q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w;
    }
};

template <int V>
__global__ __launch_bounds__(kSelBlock) void k_csr_select(uint64_t ncand, uint32_t wx, Shares3 idm,
                                                          const uint32_t* __restrict__ off, Shares3 post, Out3 out) {
    using S = SelVec<V>;
    using T = typename S::T;
    __shared__ uint32_t rec[kSelCand];
    __shared__ uint32_t msk[kSelCand];
    __shared__ uint32_t nsel;
    __shared__ T part[3][kSelBlock];
    const uint32_t l = blockIdx.y;
    const uint64_t per = (ncand + gridDim.x - 1) / gridDim.x;
    const uint64_t c0 = (uint64_t)blockIdx.x * per;
    const uint64_t c1 = c0 + per < ncand ? c0 + per : ncand;
    const uint32_t t = threadIdx.x;
    if (t == 0) nsel = 0;
    __syncthreads();
    for (uint64_t c = c0 + t; c < c1; c += kSelBlock) {
        const uint32_t o = off[c];
        if (l >= off[c + 1] - o) continue;              // the list ends before slot l
        uint32_t m = 0;
#pragma unroll
        for (int i = 0; i < 3; i++) m |= ((idm.p[i][c >> 5] >> (c & 31)) & 1u) << i;
        const uint32_t k = atomicAdd(&nsel, 1u);         // order-free: the products are XORed
        if (k < kSelCand) {
            rec[k] = o + l;
            msk[k] = m;
        }
    }
    __syncthreads();
    const uint32_t n = nsel < kSelCand ? nsel : kSelCand;
    const uint32_t nv = wx / V;                          // loads per record
    const T* src[3] = {(const T*)post.p[0], (const T*)post.p[1], (const T*)post.p[2]};
    for (uint32_t v0 = 0; v0 < nv; v0 += kSelBlock) {
        const uint32_t tw = nv - v0 < kSelBlock ? nv - v0 : kSelBlock;
        const uint32_t lanes = kSelBlock / tw;
        const uint32_t w = t % tw, g = t / tw;
        T acc[3] = {S::zero(), S::zero(), S::zero()};
        if (g < lanes) {
            uint32_t k = g;
            for (; k + lanes < n; k += 2 * lanes) {
                const uint64_t a = (uint64_t)rec[k] * nv + v0 + w, b = (uint64_t)rec[k + lanes] * nv + v0 + w;
                T ra[3], rb[3];
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    ra[i] = src[i][a];
                    rb[i] = src[i][b];
                }
                uint32_t ma[3], mb[3];
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    ma[i] = 0u - ((msk[k] >> i) & 1u);
                    mb[i] = 0u - ((msk[k + lanes] >> i) & 1u);
                }
                S::prod(ma, ra, acc);
                S::prod(mb, rb, acc);
            }
            if (k < n) {
                const uint64_t a = (uint64_t)rec[k] * nv + v0 + w;
                T ra[3];
                uint32_t ma[3];
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    ra[i] = src[i][a];
                    ma[i] = 0u - ((msk[k] >> i) & 1u);
                }
                S::prod(ma, ra, acc);
            }
        }
#pragma unroll
        for (int i = 0; i < 3; i++) part[i][t] = acc[i];
        __syncthreads();
        if (t < tw) {
#pragma unroll
            for (int i = 0; i < 3; i++) {
                T v = S::zero();
                for (uint32_t k = 0; k < lanes; k++) {
                    const T p = part[i][k * tw + t];
                    if constexpr (V == 4) {
                        v.x ^= p.x; v.y ^= p.y; v.z ^= p.z; v.w ^= p.w;
                    } else {
                        v ^= p;
                    }
                }
#pragma unroll
                for (int q = 0; q < V; q++) {
                    const uint32_t x = S::word(v, q);
                    if (x) atomicXor(&out.p[i][(uint64_t)l * wx + (uint64_t)(v0 + t) * V + q], x);
                }
            }
        }
        __syncthreads();
    }
}

// Kept ID k = blockIdx.y (exits when k >= *count): XOR over this block's
// attribute rows x < x_bits of bit x of the kept record AND row x.
__global__ __launch_bounds__(kSelBlock) void k_attr_select(uint32_t x_bits, uint32_t wx, uint32_t wd,
                                                           const uint32_t* __restrict__ count, Shares3 ids,
                                                           Shares3 attr, Out3 out) {
    __shared__ uint32_t part[3][kSelBlock];
    const uint32_t k = blockIdx.y;
    if (k >= *count) return;                                      // uniform over the block
    const uint64_t per = ((uint64_t)x_bits + gridDim.x - 1) / gridDim.x;
    const uint64_t x0 = (uint64_t)blockIdx.x * per;
    const uint64_t x1 = x0 + per < x_bits ? x0 + per : x_bits;
    const uint32_t t = threadIdx.x;
    for (uint32_t w0 = 0; w0 < wd; w0 += kSelBlock) {
        const uint32_t tw = wd - w0 < kSelBlock ? wd - w0 : kSelBlock;
        const uint32_t lanes = kSelBlock / tw;
        const uint32_t w = t % tw, g = t / tw;
        uint32_t acc[3] = {0, 0, 0};
        if (g < lanes) {
            for (uint64_t x = x0 + g; x < x1; x += lanes) {
                uint32_t m[3], r[3];
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    m[i] = 0u - ((ids.p[i][(uint64_t)k * wx + (x >> 5)] >> (x & 31)) & 1u);
                    r[i] = attr.p[i][x * wd + w0 + w];
                }
                rss_product(m, r, acc);
            }
        }
        reduce_out(part, acc, tw, lanes, out.p, (uint64_t)k * wd + w0);
    }
}

struct Carve {
    uint8_t* base;
    uint64_t size, used = 0;
    bool ok = true;
    uint32_t* take(uint64_t words) {
        const uint64_t bytes = (words * 4 + 255) & ~255ull;
        if (used + bytes > size) {
            ok = false;
            return nullptr;
        }
        uint32_t* p = (uint32_t*)(base + used);
        used += bytes;
        return p;
    }
};

uint64_t rnd(uint64_t words) { return (words * 4 + 255) & ~255ull; }

}  // namespace

extern "C" {

int rss_group_k_lists(uint64_t n, uint32_t nlists, const uint32_t* lengths, const uint32_t* types, uint32_t k,
                      uint32_t* padded, uint32_t* group) {
    last_error().clear();
    if (n == 0) return FSS_OK;
    if (!lengths || !types || !padded) return fail(FSS_EINVAL, "rss_group_k: NULL argument");
    if (k == 0) return fail(FSS_EINVAL, "rss_group_k: k must be at least 1");
    if (nlists == 0) return fail(FSS_EINVAL, "rss_group_k: no list types");
    auto len = [&](uint32_t l, uint64_t v) { return lengths[(uint64_t)l * n + v]; };
    std::vector<uint64_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    // by type, then the vector of list lengths (list type 0 first), then vertex ID
    std::sort(order.begin(), order.end(), [&](uint64_t a, uint64_t b) {
        if (types[a] != types[b]) return types[a] < types[b];
        for (uint32_t l = 0; l < nlists; l++)
            if (len(l, a) != len(l, b)) return len(l, a) < len(l, b);
        return a < b;
    });
    uint32_t gid = 0;
    for (uint64_t s = 0; s < n;) {
        uint64_t e = s;
        while (e < n && types[order[e]] == types[order[s]]) e++;     // [s, e): one type
        const uint64_t m = e - s;
        const uint64_t ngroups = m / k > 0 ? m / k : 1;
        for (uint64_t g = 0; g < ngroups; g++) {
            const uint64_t lo = s + g * k, hi = g + 1 < ngroups ? lo + k : e;   // the last takes the rest
            for (uint32_t l = 0; l < nlists; l++) {
                uint32_t mx = 0;
                for (uint64_t i = lo; i < hi; i++) mx = std::max(mx, len(l, order[i]));
                for (uint64_t i = lo; i < hi; i++) padded[(uint64_t)l * n + order[i]] = mx;
            }
            if (group)
                for (uint64_t i = lo; i < hi; i++) group[order[i]] = gid;
            gid++;
        }
        s = e;
    }
    return FSS_OK;
}

int rss_group_k(uint64_t n, const uint32_t* lengths, const uint32_t* types, uint32_t k, uint32_t* padded,
                uint32_t* group) {
    return rss_group_k_lists(n, 1, lengths, types, k, padded, group);
}

int rss_enc_posting_lists(uint64_t n, uint32_t x_bits, const uint32_t* d_adj_off, const uint32_t* d_adj,
                          const uint32_t* d_slot, const uint32_t* d_off, uint64_t nrec, const uint64_t split_keys[2],
                          uint32_t counter, uint32_t* const d_out[3], void* d_work, uint64_t work_bytes,
                          void* stream) {
    last_error().clear();
    if (x_bits == 0) return fail(FSS_EINVAL, "rss_enc_posting_lists: x_bits is 0");
    if (n == 0 || nrec == 0) return FSS_OK;
    if (!d_adj_off || !d_adj || !d_slot || !d_off || !split_keys || !d_out || !d_out[0] || !d_out[1] || !d_out[2])
        return fail(FSS_EINVAL, "rss_enc_posting_lists: NULL argument");
    const uint32_t wx = (x_bits + 31) / 32;
    if (nrec > 0xFFFFFFFFull || nrec * wx / 16 > 0xFFFFFFFFull)
        return fail(FSS_EUNSUPPORTED, "rss_enc_posting_lists: table too large");
    if (!d_work || work_bytes < nrec * 4)
        return fail(FSS_ENOMEM, "rss_enc_posting_lists: workspace needs %llu bytes", (unsigned long long)(nrec * 4));
    hipStream_t s = (hipStream_t)stream;
    uint32_t* rec_id = (uint32_t*)d_work;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(nrec, 256, 4096)), dim3(256), 0, s, nrec, 0xFFFFFFFFu, rec_id);
    hipLaunchKernelGGL(k_place_ids, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, n, x_bits, d_adj_off, d_adj,
                       d_slot, d_off, rec_id);
    const uint64_t total = nrec * wx, quads = (total + 3) / 4;
    const bool vec = wx % 4 == 0 && ((uintptr_t)d_out[0] | (uintptr_t)d_out[1] | (uintptr_t)d_out[2]) % 16 == 0;
    const ChachaKey ka = chacha_key(split_keys[0], 5), kb = chacha_key(split_keys[1], 5);
    if (vec)
        hipLaunchKernelGGL(k_split_records<true>, dim3((unsigned)((quads + 255) / 256)), dim3(256), 0, s, total, wx,
                           rec_id, ka, kb, counter, d_out[0], d_out[1], d_out[2]);
    else
        hipLaunchKernelGGL(k_split_records<false>, dim3((unsigned)((quads + 255) / 256)), dim3(256), 0, s, total, wx,
                           rec_id, ka, kb, counter, d_out[0], d_out[1], d_out[2]);
    return check_launch("rss_enc_posting_lists");
}

uint64_t rss_sec_access_workspace_bytes(uint32_t lmax, uint32_t x_bits, uint32_t attr_words) {
    const uint64_t wx = (x_bits + 31) / 32, l = lmax ? lmax : 1;
    return 6 * rnd(l * wx) + 3 * rnd(l * attr_words) + rss_fetch_many_workspace_bytes(l, (uint32_t)wx) + 256;
}

int rss_sec_access(uint64_t ncand, uint32_t x_bits, const uint32_t* const d_idm[3], const uint32_t* d_off,
                   uint32_t lmax, const uint32_t* const d_post[3], uint32_t attr_words,
                   const uint32_t* const d_attr[3], const uint64_t prf_keys[3], uint32_t counter,
                   const uint64_t seeds[3], uint32_t* const d_ids[3], uint32_t* const d_attrs[3],
                   uint32_t* d_rows_out, uint32_t* d_count, void* d_work, uint64_t work_bytes, void* stream) {
    last_error().clear();
    const char* who = "rss_sec_access";
    if (x_bits == 0 || attr_words == 0) return fail(FSS_EINVAL, "%s: empty IDs or attribute records", who);
    if (lmax == 0 || lmax > 65535) return fail(FSS_EINVAL, "%s: lmax %u outside 1..65535", who, lmax);
    if (!d_idm || !d_off || !d_post || !d_attr || !prf_keys || !seeds || !d_ids || !d_attrs || !d_rows_out || !d_count)
        return fail(FSS_EINVAL, "%s: NULL argument", who);
    for (int i = 0; i < 3; i++)
        if (!d_idm[i] || !d_post[i] || !d_attr[i] || !d_ids[i] || !d_attrs[i])
            return fail(FSS_EINVAL, "%s: NULL share %d", who, i);
    if (ncand > 0xFFFFFFFFull) return fail(FSS_EUNSUPPORTED, "%s: more than 2^32 candidates", who);
    const uint32_t wx = (x_bits + 31) / 32, wd = attr_words;
    if (!d_work || work_bytes < rss_sec_access_workspace_bytes(lmax, x_bits, wd))
        return fail(FSS_ENOMEM, "%s: workspace needs %llu bytes", who,
                    (unsigned long long)rss_sec_access_workspace_bytes(lmax, x_bits, wd));
    hipStream_t s = (hipStream_t)stream;
    Carve ws{(uint8_t*)d_work, work_bytes};
    const uint64_t tw = (uint64_t)lmax * wx, ta = (uint64_t)lmax * wd;
    uint32_t* add[3] = {ws.take(tw), ws.take(tw), ws.take(tw)};
    uint32_t* rss[3] = {ws.take(tw), ws.take(tw), ws.take(tw)};
    uint32_t* att[3] = {ws.take(ta), ws.take(ta), ws.take(ta)};
    const uint64_t cws = rss_fetch_many_workspace_bytes(lmax, wx);
    uint8_t* cwork = (uint8_t*)ws.take((cws + 3) / 4);
    if (!ws.ok) return fail(FSS_ENOMEM, "%s: workspace too small", who);
    // 1. P_m[l] = XOR_c id_m[c] AND id_{c,l}: additive shares
    hipLaunchKernelGGL(k_zero3, dim3(blocks_for(tw, 256, 4096)), dim3(256), 0, s, tw, Out3{{add[0], add[1], add[2]}});
    if (ncand) {
        // enough chunks to fill the chip over lmax slots, and at most kSelCand candidates per chunk
        const uint64_t chunks = std::max<uint64_t>((ncand + kSelCand - 1) / kSelCand,
                                                   std::min<uint64_t>((ncand + 63) / 64, 4096 / lmax + 1));
        const Shares3 idm{{d_idm[0], d_idm[1], d_idm[2]}}, post{{d_post[0], d_post[1], d_post[2]}};
        const Out3 o{{add[0], add[1], add[2]}};
        bool vec = wx % 4 == 0;
        for (int i = 0; i < 3; i++) vec = vec && ((uintptr_t)d_post[i] & 15) == 0;
        if (vec)
            hipLaunchKernelGGL(k_csr_select<4>, dim3((unsigned)chunks, lmax), dim3(kSelBlock), 0, s, ncand, wx, idm,
                               d_off, post, o);
        else
            hipLaunchKernelGGL(k_csr_select<1>, dim3((unsigned)chunks, lmax), dim3(kSelBlock), 0, s, ncand, wx, idm,
                               d_off, post, o);
    }
    int rc = check_launch("k_csr_select");
    if (rc) return rc;
    // ... re-shared into RSS
    const uint32_t* a3[3] = {add[0], add[1], add[2]};
    rc = rss_reshare(32 * tw, a3, prf_keys, counter, rss, stream);
    if (rc) return rc;
    // 2. shuffle, open the parity of each record, keep the valid IDs
    const uint32_t* r3[3] = {rss[0], rss[1], rss[2]};
    rc = rss_compact_valid(lmax, wx, r3, seeds, d_ids, d_rows_out, d_count, cwork, cws, stream);
    if (rc) return rc;
    // 3. the attribute record of every kept ID, then one re-share of them all
    hipLaunchKernelGGL(k_zero3, dim3(blocks_for(ta, 256, 4096)), dim3(256), 0, s, ta, Out3{{att[0], att[1], att[2]}});
    const uint64_t xchunks = std::max<uint64_t>(1, std::min<uint64_t>((x_bits + 255) / 256, 2048 / lmax + 1));
    hipLaunchKernelGGL(k_attr_select, dim3((unsigned)xchunks, lmax), dim3(kSelBlock), 0, s, x_bits, wx, wd, d_count,
                       Shares3{{d_ids[0], d_ids[1], d_ids[2]}}, Shares3{{d_attr[0], d_attr[1], d_attr[2]}},
                       Out3{{att[0], att[1], att[2]}});
    rc = check_launch("k_attr_select");
    if (rc) return rc;
    const uint32_t* t3[3] = {att[0], att[1], att[2]};
    return rss_reshare(32 * ta, t3, prf_keys, counter + 1, d_attrs, stream);
}

int rss_sec_access_batch(uint32_t count, uint64_t ncand, uint32_t x_bits, const uint32_t* const* d_idm,
                         const uint32_t* d_off, uint32_t lmax, const uint32_t* const d_post[3], uint32_t attr_words,
                         const uint32_t* const d_attr[3], const uint64_t prf_keys[3], const uint32_t* counters,
                         const uint64_t* seeds, uint32_t* const d_ids[3], uint32_t* const d_attrs[3],
                         uint32_t* d_rows_out, uint32_t* d_count, void* d_work, uint64_t work_bytes, void* stream) {
    last_error().clear();
    const char* who = "rss_sec_access_batch";
    if (count == 0) return FSS_OK;
    if (!d_idm || !counters || !seeds || !d_ids || !d_attrs || !d_rows_out || !d_count)
        return fail(FSS_EINVAL, "%s: NULL argument", who);
    for (uint64_t k = 0; k < 3ull * count; k++)
        if (!d_idm[k]) return fail(FSS_EINVAL, "%s: NULL matched-ID share %llu", who, (unsigned long long)k);
    for (int i = 0; i < 3; i++)
        if (!d_ids[i] || !d_attrs[i]) return fail(FSS_EINVAL, "%s: NULL output share %d", who, i);
    const uint64_t wx = (x_bits + 31) / 32;
    for (uint32_t c = 0; c < count; c++) {
        uint32_t* ids[3];
        uint32_t* attrs[3];
        for (int i = 0; i < 3; i++) {
            ids[i] = d_ids[i] + (uint64_t)c * lmax * wx;
            attrs[i] = d_attrs[i] + (uint64_t)c * lmax * attr_words;
        }
        // the shared arguments are checked by the first call; the rest differ
        // only in pointers checked above
        const int rc = rss_sec_access(ncand, x_bits, d_idm + 3ull * c, d_off, lmax, d_post, attr_words, d_attr,
                                      prf_keys, counters[c], seeds + 3ull * c, ids, attrs,
                                      d_rows_out + (uint64_t)c * lmax, d_count + c, d_work, work_bytes, stream);
        if (rc) return rc;
    }
    return FSS_OK;
}

}  // extern "C"
