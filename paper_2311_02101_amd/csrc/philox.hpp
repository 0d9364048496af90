// Philox4x32-10 counter-based generator for gfx950 device code.
//
// Definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11): ten rounds over a 4x32-bit counter with a 2x32-bit
// key.  A round multiplies words 0 and 2 by the constants M0 and M1 into
// 64-bit products; the new words are (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0).
// The key is advanced by the Weyl increments between rounds.
//
// The key is uniform across a wavefront (it depends only on the seed and the
// formula), so the key schedule stays in scalar registers.  Each round is
// four VALU instructions per lane: two 32x32->64 multiplies and two
// three-input XORs (gfx950's v_bitop3_b32 with truth table 0x96 = a^b^c,
// the key taken straight from its scalar register).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hp {

struct Key2 {
    uint32_t k0, k1;
};

__device__ __forceinline__ uint4 philox4x32_10(uint4 x, Key2 key) {
    uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            // keep the key schedule as two live scalar registers: without
            // this the compiler hoists all 20 round keys out of the caller's
            // loops and spills them into vector lanes
            asm volatile("" : "+s"(k0), "+s"(k1));
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x.z;
        x = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), x.y, k0, 0x96), (uint32_t)p1,
                       __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), x.w, k1, 0x96), (uint32_t)p0);
    }
    return x;
}

// Two counters under one key, round by round: the two chains of dependent
// multiplies interleave and the key schedule is computed once.
__device__ __forceinline__ void philox4x32_10_pair(uint4 &x, uint4 &y, Key2 key) {
    uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            asm volatile("" : "+s"(k0), "+s"(k1));
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x.z;
        const uint64_t q0 = (uint64_t)0xD2511F53u * (uint64_t)y.x;
        const uint64_t q1 = (uint64_t)0xCD9E8D57u * (uint64_t)y.z;
        x = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), x.y, k0, 0x96), (uint32_t)p1,
                       __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), x.w, k1, 0x96), (uint32_t)p0);
        y = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(q1 >> 32), y.y, k0, 0x96), (uint32_t)q1,
                       __builtin_amdgcn_bitop3_b32((uint32_t)(q0 >> 32), y.w, k1, 0x96), (uint32_t)q0);
    }
}

// Same generator for a key that differs between lanes (kept in vector
// registers; no scalar-register pinning).
__device__ __forceinline__ uint4 philox4x32_10_lane_key(uint4 x, Key2 key) {
    uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x.z;
        x = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), x.y, k0, 0x96), (uint32_t)p1,
                       __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), x.w, k1, 0x96), (uint32_t)p0);
    }
    return x;
}

// Counter word 2: phase in the top bit, block index below it.
constexpr uint32_t kPhaseHidden = 0u;
constexpr uint32_t kPhaseVisible = 0x80000000u;

}  // namespace hp
