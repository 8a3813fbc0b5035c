// philox.hpp -- Philox4x64-10 counter-based generator (Salmon, Moraes, Dror,
// Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), written from
// its published definition: 10 rounds, each two 64x64->128-bit products of
// counter words with fixed multipliers, xor-ed with the other counter words
// and the round key; the key advances by a Weyl sequence between rounds.
#pragma once
#include "common.hpp"

namespace agn {

struct u64x4 { uint64_t v[4]; };

AGN_DEV u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                            uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    u64x4 o; o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// Uniform #k of stream `stream` for (seed, curve): key (seed, stream<<32 | curve),
// counter (k/4, 0, 0, 0), word k%4, mapped to ((w >> 12) + 1/2) * 2^-52 in (0, 1).
AGN_DEV double philox_uniform(uint64_t seed, uint32_t stream, uint32_t curve, uint64_t k) {
    u64x4 o = philox4x64_10(k >> 2, 0, 0, 0, seed, ((uint64_t)stream << 32) | curve);
    uint64_t w = o.v[k & 3];
    return ((double)(w >> 12) + 0.5) * 0x1.0p-52;
}

// Uniform #k of chain `chain` of a stream: counter (k/4, chain, 0, 0), same
// key and mapping as philox_uniform (which is chain 0).
AGN_DEV double philox_uniform_chain(uint64_t seed, uint32_t stream, uint32_t curve, uint64_t chain, uint64_t k) {
    u64x4 o = philox4x64_10(k >> 2, chain, 0, 0, seed, ((uint64_t)stream << 32) | curve);
    uint64_t w = o.v[k & 3];
    return ((double)(w >> 12) + 0.5) * 0x1.0p-52;
}

}  // namespace agn
