// chacha_gfx950.hpp -- the ChaCha block function (Bernstein 2008; RFC 8439
// gives the 20-round form) with 12 rounds, made by four lanes together on
// CDNA4.  The shuffle's pairwise tables and keys and the RSS zero-sharing PRF
// draw from it.
//
// A key is a 64-bit seed and a domain: key words (seed mod 2^32, seed div
// 2^32, domain, 0, 0, 0, 0, 0); state words 12-15 name the block.  Lane c of
// each aligned quad of lanes holds column c of the state (words c, 4 + c,
// 8 + c, 12 + c) and applies the column round's quarter round to it; for the
// diagonal round rows 1-3 rotate across the quad by 1, 2 and 3 lanes (DPP
// quad permutations), and back afterwards.  A block's words are read column
// by column (slice word 4c + k is state word 4k + c), so lane c ends holding
// slice words 4c .. 4c + 3: four lanes hold one 64-byte slice, 16 contiguous
// bytes each.  All four lanes of a quad must be active.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ogm {

constexpr int kChachaRounds = 12;

struct ChachaKey {
    uint32_t lo, hi, domain;
};

inline ChachaKey chacha_key(uint64_t seed, uint32_t domain) {
    return ChachaKey{(uint32_t)seed, (uint32_t)(seed >> 32), domain};
}

__device__ __forceinline__ void chacha_quarter(uint32_t& a, uint32_t& b, uint32_t& c, uint32_t& d) {
    a += b; d = __builtin_rotateleft32(d ^ a, 16);
    c += d; b = __builtin_rotateleft32(b ^ c, 12);
    a += b; d = __builtin_rotateleft32(d ^ a, 8);
    c += d; b = __builtin_rotateleft32(b ^ c, 7);
}

// lane c of the quad takes the value of lane (c + S) mod 4.  Callers keep
// every quad whole (all four lanes active), so every source lane is valid and
// the bound control never applies; in this form (old value 0, bound control
// on) the compiler folds the permutation into the add or XOR that consumes
// it as a DPP operand (a separate v_mov_b32_dpp adds 6 instructions to the
// 24 of each double round: 186 per block and lane instead of 151).
template <int S>
__device__ __forceinline__ uint32_t quad_from(uint32_t v) {
    constexpr int ctrl = ((0 + S) & 3) | (((1 + S) & 3) << 2) | (((2 + S) & 3) << 4) | (((3 + S) & 3) << 6);
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ctrl, 0xF, 0xF, true);
}

// Lane c = threadIdx.x & 3 of each quad: returns slice words 4c .. 4c + 3 of
// block (w12, w13, w14, w15) under key k.
__device__ __forceinline__ uint4 chacha_quad(ChachaKey k, uint32_t w12, uint32_t w13, uint32_t w14, uint32_t w15) {
    const uint32_t c = threadIdx.x & 3u;
    const uint32_t a0 = c == 0 ? 0x61707865u : c == 1 ? 0x3320646eu : c == 2 ? 0x79622d32u : 0x6b206574u;
    const uint32_t b0 = c == 0 ? k.lo : c == 1 ? k.hi : c == 2 ? k.domain : 0u;   // key words c; 4 + c are 0
    const uint32_t d0 = c == 0 ? w12 : c == 1 ? w13 : c == 2 ? w14 : w15;
    uint32_t x0 = a0, x1 = b0, x2 = 0u, x3 = d0;
#pragma unroll
    for (int r = 0; r < kChachaRounds / 2; r++) {
        chacha_quarter(x0, x1, x2, x3);
        x1 = quad_from<1>(x1), x2 = quad_from<2>(x2), x3 = quad_from<3>(x3);
        chacha_quarter(x0, x1, x2, x3);
        x1 = quad_from<3>(x1), x2 = quad_from<2>(x2), x3 = quad_from<1>(x3);
    }
    return make_uint4(x0 + a0, x1 + b0, x2, x3 + d0);
}

}  // namespace ogm
