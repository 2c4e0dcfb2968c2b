// aes_gfx950.hpp -- AES-128 encryption for gfx950 wavefronts, T-table in LDS.
//
// The tree hash of the FSS keys is fixed-key AES-128 made circular
// correlation-robust, H(x) = AES_K(sigma(x)) ^ sigma(x) (lambda = 128,
// Sec. VII-A); the dealer's randomness is AES-128 in counter mode under a
// per-call key.  Both run through aes128_encrypt() below.
//
// Table layout.  T0[x] = (2S(x), S(x), S(x), 3S(x)) (bytes 0..3: the
// MixColumns image of S(x) in row 0) and T1 = rotl8(T0) sit in LDS as 256 rows
// of 256 bytes: row x holds 32 copies of T0[x], then 32 copies of T1[x].  Lane
// l reads copy (l mod 32), i.e. byte address (x << 8) | (t << 7) | ((l & 31) << 2):
// within each half-wave every lane reads its own bank whatever the data, so
// the lookups are free of bank conflicts (measured: zero).  The address of
// "byte k of state word w in table t" is one v_perm_b32 -- byte 1 of the result
// is byte k of w, byte 0 the lane's offset for table t, bytes 2..3 zero.
// With T2 = rotl16(T0) and T3 = rotl16(T1), a round column is
//   T0[a] ^ T1[b] ^ rotl16(T0[c] ^ T1[d] ^ rotr16(k)),
// i.e. 4 perms, 4 ds_read_b32, 2 three-input XORs and one rotate.  The last
// round takes S(x) = byte 1 of T0[x] and assembles a column with two perms.
// 64 KiB of LDS per workgroup.  At 160 lookups per block this round function
// keeps the LDS pipe (32 dwords per clock per CU) nearly saturated; the VALU
// has some slack.
//
// Tables and the fixed key schedule are generated at compile time from GF(2^8)
// arithmetic (log/antilog tables over the generator 3) and FIPS-197's affine
// map; nothing is pasted.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ogm {

// ----------------------------------------------------------------- compile-time tables

constexpr uint8_t xtime(uint8_t a) { return (uint8_t)((a << 1) ^ ((a & 0x80) ? 0x1b : 0x00)); }

struct GfLogExp {
    uint8_t exp[256];
    uint8_t log[256];
};

constexpr GfLogExp make_log_exp() {
    GfLogExp t{};
    uint8_t v = 1;
    for (int i = 0; i < 255; i++) {
        t.exp[i] = v;
        t.log[v] = (uint8_t)i;
        v = (uint8_t)(v ^ xtime(v));  // multiply by the generator 3
    }
    t.exp[255] = t.exp[0];
    return t;
}

constexpr GfLogExp kLogExp = make_log_exp();

constexpr uint8_t gf_inverse(uint8_t x) {
    return x == 0 ? 0 : kLogExp.exp[(255 - kLogExp.log[x]) % 255];
}

constexpr uint8_t rot8(uint8_t x, int k) { return (uint8_t)((x << k) | (x >> (8 - k))); }

constexpr uint8_t sub_byte(uint8_t x) {
    uint8_t b = gf_inverse(x);
    return (uint8_t)(b ^ rot8(b, 1) ^ rot8(b, 2) ^ rot8(b, 3) ^ rot8(b, 4) ^ 0x63);
}

struct AesTables {
    uint8_t sbox[256];
    uint32_t t0[256];
};

constexpr AesTables make_tables() {
    AesTables t{};
    for (int x = 0; x < 256; x++) {
        uint8_t s = sub_byte((uint8_t)x);
        uint8_t s2 = xtime(s);
        uint8_t s3 = (uint8_t)(s2 ^ s);
        t.sbox[x] = s;
        t.t0[x] = (uint32_t)s2 | ((uint32_t)s << 8) | ((uint32_t)s << 16) | ((uint32_t)s3 << 24);
    }
    return t;
}

constexpr AesTables kTables = make_tables();

// Round keys as 44 little-endian words, word 4r + c = column c of round r,
// each kept in the form the cipher consumes it: the first (whitening) and last
// round keys as they are, the keys of rounds 1..9 rotated right by 16 bits
// (round_col folds them in before its rotate).  A per-call schedule then costs
// no rotate in the kernel and 44 scalar registers.
struct RoundKeys {
    uint32_t w[44];
};

constexpr bool kRotatedRoundKey(int i) { return i >= 4 && i < 40; }

constexpr RoundKeys expand_key(const uint8_t (&key)[16]) {
    RoundKeys rk{};
    uint8_t b[176] = {};
    for (int i = 0; i < 16; i++) b[i] = key[i];
    uint8_t rcon = 1;
    for (int i = 4; i < 44; i++) {
        uint8_t t[4] = {b[4 * i - 4], b[4 * i - 3], b[4 * i - 2], b[4 * i - 1]};
        if (i % 4 == 0) {
            uint8_t first = t[0];
            t[0] = (uint8_t)(kTables.sbox[t[1]] ^ rcon);
            t[1] = kTables.sbox[t[2]];
            t[2] = kTables.sbox[t[3]];
            t[3] = kTables.sbox[first];
            rcon = xtime(rcon);
        }
        for (int k = 0; k < 4; k++) b[4 * i + k] = (uint8_t)(b[4 * i - 16 + k] ^ t[k]);
    }
    for (int i = 0; i < 44; i++) {
        rk.w[i] = (uint32_t)b[4 * i] | ((uint32_t)b[4 * i + 1] << 8) | ((uint32_t)b[4 * i + 2] << 16) |
                  ((uint32_t)b[4 * i + 3] << 24);
        if (kRotatedRoundKey(i)) rk.w[i] = (rk.w[i] >> 16) | (rk.w[i] << 16);
    }
    return rk;
}

constexpr uint8_t kHashKeyBytes[16] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15};
constexpr RoundKeys kHashKeys = expand_key(kHashKeyBytes);

// Key sources: k[i] is word i for the whitening (i < 4) and last (i >= 40)
// round keys, k.mid(i) a word of rounds 1..9, already rotated.
//
// The fixed tree-hash key schedule, folded into instruction constants after unrolling.
struct FixedHashKey {
    __device__ __forceinline__ constexpr uint32_t operator[](int i) const { return kHashKeys.w[i]; }
    __device__ __forceinline__ constexpr uint32_t mid(int i) const { return kHashKeys.w[i]; }
};

// A per-call key schedule held in kernel arguments (scalar registers).
struct ArgKey {
    const RoundKeys& rk;
    __device__ __forceinline__ uint32_t operator[](int i) const { return rk.w[i]; }
    __device__ __forceinline__ uint32_t mid(int i) const { return rk.w[i]; }
};

// ----------------------------------------------------------------- LDS table

constexpr int kLdsTableWords = 256 * 64;  // 64 KiB

__device__ __forceinline__ uint32_t rotl32(uint32_t x, int k) { return (x << k) | (x >> (32 - k)); }

// Fills the replicated tables; every thread of the workgroup takes part.  The
// caller synchronises the workgroup before the first lookup.
__device__ __forceinline__ void lds_table_fill(uint32_t* tab, const uint32_t* g_t0) {
    for (int i = threadIdx.x; i < kLdsTableWords; i += blockDim.x) {
        const uint32_t v = g_t0[i >> 6];
        tab[i] = (i & 32) ? rotl32(v, 8) : v;     // word i: row i >> 6, table (i >> 5) & 1
    }
}

// This lane's byte offsets into row x of T0 and of T1.
struct LaneOff {
    uint32_t t0, t1;
};

__device__ __forceinline__ LaneOff lane_offset() {
    const uint32_t c = (threadIdx.x & 31u) << 2;
    return LaneOff{c, 128u | c};
}

__device__ __forceinline__ uint32_t lds_word(const uint32_t* tab, uint32_t byte_addr) {
    return *(const uint32_t*)((const char*)tab + byte_addr);
}

// Lookup of T[byte k of w] in this lane's copy of the table whose lane offset is `off`.
template <int K>
__device__ __forceinline__ uint32_t tlook(const uint32_t* tab, uint32_t w, uint32_t off) {
    constexpr uint32_t sel = 0x0C0C0000u | ((uint32_t)(4 + K) << 8);
    return lds_word(tab, __builtin_amdgcn_perm(w, off, sel));
}

// a ^ b ^ c in one v_bitop3_b32 (truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// One full round: out_c = T0[b0(s_c)] ^ T1[b1(s_c+1)] ^ T2[b2(s_c+2)] ^ T3[b3(s_c+3)] ^ rk_c
// with T2[y] = rotl16(T0[y]), T3[y] = rotl16(T1[y]); kr = rotr16(rk_c).
__device__ __forceinline__ uint32_t round_col(const uint32_t* tab, LaneOff lo, uint32_t a, uint32_t b,
                                              uint32_t c, uint32_t d, uint32_t kr) {
    const uint32_t t0 = tlook<0>(tab, a, lo.t0);
    const uint32_t t1 = tlook<1>(tab, b, lo.t1);
    const uint32_t t2 = tlook<2>(tab, c, lo.t0);
    const uint32_t t3 = tlook<3>(tab, d, lo.t1);
    return xor3(t0, t1, rotl32(xor3(t2, t3, kr), 16));
}

// Last round: out_c = S(b0(s_c)) | S(b1(s_c+1)) << 8 | S(b2(s_c+2)) << 16 | S(b3(s_c+3)) << 24, ^ rk.
__device__ __forceinline__ uint32_t final_col(const uint32_t* tab, LaneOff lo, uint32_t a, uint32_t b,
                                              uint32_t c, uint32_t d, uint32_t k) {
    const uint32_t t0 = tlook<0>(tab, a, lo.t0);
    const uint32_t t1 = tlook<1>(tab, b, lo.t0);
    const uint32_t t2 = tlook<2>(tab, c, lo.t0);
    const uint32_t t3 = tlook<3>(tab, d, lo.t0);
    const uint32_t low = __builtin_amdgcn_perm(t1, t0, 0x0C0C0501u);   // (S(b), S(a)) in bytes 1, 0
    const uint32_t high = __builtin_amdgcn_perm(t3, t2, 0x05010C0Cu);  // (S(d), S(c)) in bytes 3, 2
    return xor3(low, high, k);
}

// Rounds 2..10 from the state after round 1.
template <class RK>
__device__ __forceinline__ uint4 aes128_rounds_2_10(uint32_t s0, uint32_t s1, uint32_t s2, uint32_t s3, const RK& rk,
                                                    const uint32_t* tab, LaneOff lo) {
#pragma unroll
    for (int r = 2; r < 10; r++) {
        const uint32_t n0 = round_col(tab, lo, s0, s1, s2, s3, rk.mid(4 * r + 0));
        const uint32_t n1 = round_col(tab, lo, s1, s2, s3, s0, rk.mid(4 * r + 1));
        const uint32_t n2 = round_col(tab, lo, s2, s3, s0, s1, rk.mid(4 * r + 2));
        const uint32_t n3 = round_col(tab, lo, s3, s0, s1, s2, rk.mid(4 * r + 3));
        s0 = n0; s1 = n1; s2 = n2; s3 = n3;
    }
    uint4 out;
    out.x = final_col(tab, lo, s0, s1, s2, s3, rk[40]);
    out.y = final_col(tab, lo, s1, s2, s3, s0, rk[41]);
    out.z = final_col(tab, lo, s2, s3, s0, s1, rk[42]);
    out.w = final_col(tab, lo, s3, s0, s1, s2, rk[43]);
    return out;
}

template <class RK>
__device__ __forceinline__ uint4 aes128_encrypt(uint4 in, const RK& rk, const uint32_t* tab, LaneOff lo) {
    const uint32_t s0 = in.x ^ rk[0], s1 = in.y ^ rk[1], s2 = in.z ^ rk[2], s3 = in.w ^ rk[3];
    const uint32_t n0 = round_col(tab, lo, s0, s1, s2, s3, rk.mid(4));
    const uint32_t n1 = round_col(tab, lo, s1, s2, s3, s0, rk.mid(5));
    const uint32_t n2 = round_col(tab, lo, s2, s3, s0, s1, rk.mid(6));
    const uint32_t n3 = round_col(tab, lo, s3, s0, s1, s2, rk.mid(7));
    return aes128_rounds_2_10(n0, n1, n2, n3, rk, tab, lo);
}

__device__ __forceinline__ uint4 xor4(uint4 a, uint4 b) {
    return make_uint4(a.x ^ b.x, a.y ^ b.y, a.z ^ b.z, a.w ^ b.w);
}

__device__ __forceinline__ uint4 and4(uint4 a, uint32_t m) {
    return make_uint4(a.x & m, a.y & m, a.z & m, a.w & m);
}

// The linear orthomorphism sigma(a || b) = (a ^ b) || a on the two 64-bit
// halves of a block (a = bytes 0..7, words x and y).
__device__ __forceinline__ uint4 sigma(uint4 s) { return make_uint4(s.x ^ s.z, s.y ^ s.w, s.x, s.y); }

// H(s) = AES_K(sigma(s)) ^ sigma(s) under the fixed key K = 00 01 .. 0f: one
// hash per tree node (Guo, Katz, Wang, Yu, IEEE S&P 2020 show fixed-key AES in
// this form is circular correlation-robust, the property a half-tree needs).
__device__ __forceinline__ uint4 tree_hash(uint4 s, const uint32_t* tab, LaneOff lo) {
    const uint4 u = sigma(s);
    return xor4(aes128_encrypt(u, FixedHashKey{}, tab, lo), u);
}

}  // namespace ogm
