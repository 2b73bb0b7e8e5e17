// philox.hpp -- Philox4x32-10 for gfx950 device code.
//
// Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC'11): ten rounds of a keyed bijection on four 32-bit words.  A round
// forms the full 64-bit products of counter words 0 and 2 with two fixed odd
// multipliers, xors each high half with the opposite word pair and a round key
// word, and reorders the four results; the two key words advance by the two
// Weyl increments between rounds.  The key is uniform across a launch, so the
// ten round keys are computed once by the caller (scalar registers) and the
// lanes spend only the two 32x32->64 products and two three-way xors per round.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spinlat {

struct PhiloxKey {
    uint32_t k0[10];
    uint32_t k1[10];
};

__host__ __device__ inline PhiloxKey philox_schedule(uint32_t key0, uint32_t key1)
{
    PhiloxKey ks;
    for (int r = 0; r < 10; ++r) {
        ks.k0[r] = key0 + (uint32_t)r * 0x9E3779B9u;
        ks.k1[r] = key1 + (uint32_t)r * 0xBB67AE85u;
    }
    return ks;
}

struct Words4 {
    uint32_t w[4];
};

// a ^ b ^ c in one VALU instruction (gfx950 three-input bitwise op, truth
// table 0x96); the round key operand is wave-uniform and stays in a scalar
// register.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Counter (c0, c1, c2, c3) -> four uniform 32-bit words.  Rounds 0 and 1 are
// left to the compiler: when counter words 1-3 are uniform across the wave
// (colour, sweep, tag) it evaluates their products on the scalar unit.  From
// round 2 on every word varies per lane and each round is two 32x32->64
// multiply-adds and two three-way xors.
__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, const PhiloxKey& ks)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0, n2;
        if (r < 2) {
            n0 = (uint32_t)(p1 >> 32) ^ c1 ^ ks.k0[r];
            n2 = (uint32_t)(p0 >> 32) ^ c3 ^ ks.k1[r];
        } else {
            n0 = xor3((uint32_t)(p1 >> 32), c1, ks.k0[r]);
            n2 = xor3((uint32_t)(p0 >> 32), c3, ks.k1[r]);
        }
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    Words4 out;
    out.w[0] = c0;
    out.w[1] = c1;
    out.w[2] = c2;
    out.w[3] = c3;
    return out;
}

}  // namespace spinlat
