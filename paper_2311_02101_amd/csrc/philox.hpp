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

// Counters (tlo, chain, w, thi) of one sweep of one chain differ only in
// word w, so in the first two rounds the products of the other words are the
// same for every call of the sweep: round 1 maps the counter to
// (hi(M1 w) ^ chain ^ k0, lo(M1 w), u2, u3) with u2 = hi(M0 tlo) ^ thi ^ k1
// and u3 = lo(M0 tlo), and round 2 (key k + W) multiplies u2 by M1.  Word 1
// after round 2, lo(M1 u2), is the same for every call too; round 3 only
// XORs it with its key, so that XOR is done here (one scalar operand left
// in the lane's three-input XOR, which takes at most one).
struct PhiloxSweep {
    uint32_t c1;   // chain ^ k0
    uint32_t a2;   // hi(M1 u2) ^ (k0 + W0)
    uint32_t b2k;  // lo(M1 u2) ^ (k0 + 2 W0)
    uint32_t d2;   // u3 ^ (k1 + W1)
};

__device__ __forceinline__ PhiloxSweep philox_sweep_consts(uint32_t tlo, uint32_t chain, uint32_t thi, Key2 key) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)tlo;
    const uint32_t u2 = (uint32_t)(p0 >> 32) ^ thi ^ key.k1;
    const uint64_t v = (uint64_t)0xCD9E8D57u * (uint64_t)u2;
    return PhiloxSweep{chain ^ key.k0, (uint32_t)(v >> 32) ^ (key.k0 + 0x9E3779B9u),
                       (uint32_t)v ^ (key.k0 + 2u * 0x9E3779B9u), (uint32_t)p0 ^ (key.k1 + 0xBB67AE85u)};
}

// Philox4x32-10 of the counters (tlo, chain, w[i], thi) of one sweep: the
// first two rounds from the sweep constants (5 lane instructions instead of
// 8), round 3 with a two-input XOR for word 0, then seven full rounds, the
// NS chains interleaved round by round.
// (philox_sweep_from takes round 1's products M1 w[i] already made.)
template <int NS>
__device__ __forceinline__ void philox_sweep_from(uint4 (&x)[NS], const uint64_t (&p1)[NS], const PhiloxSweep &u,
                                                  Key2 key) {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const uint32_t a = (uint32_t)(p1[i] >> 32) ^ u.c1;         // word 0 after round 1
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)a;
        x[i] = make_uint4(u.a2 ^ (uint32_t)p1[i], 0u, (uint32_t)(p0 >> 32) ^ u.d2, (uint32_t)p0);
    }
    uint32_t k0 = key.k0 + 2u * 0x9E3779B9u, k1 = key.k1 + 2u * 0xBB67AE85u;   // round 3's key
#pragma unroll
    for (int i = 0; i < NS; ++i) {           // round 3: word 1 is lo(M1 u2), folded with k0 into b2k
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x[i].x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x[i].z;
        x[i] = make_uint4((uint32_t)(p1 >> 32) ^ u.b2k, (uint32_t)p1,
                          __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), x[i].w, k1, 0x96), (uint32_t)p0);
    }
#pragma unroll
    for (int r = 3; r < 10; ++r) {
        asm volatile("" : "+s"(k0), "+s"(k1));
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x[i].x;
            const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x[i].z;
            x[i] = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), x[i].y, k0, 0x96), (uint32_t)p1,
                              __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), x[i].w, k1, 0x96), (uint32_t)p0);
        }
    }
}

template <int NS>
__device__ __forceinline__ void philox_sweep_multi(uint4 (&x)[NS], const uint32_t (&w)[NS], const PhiloxSweep &u,
                                                   Key2 key) {
    uint64_t p1[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) p1[i] = (uint64_t)0xCD9E8D57u * (uint64_t)w[i];
    philox_sweep_from<NS>(x, p1, u, key);
}

// The blocks w and w + 1 (w + 1 < 2^32, so M1 (w + 1) = M1 w + M1 without a
// carry out of 64 bits): the second product is one multiply-add from w
// instead of an add and a multiply.  Written as asm with M1 in a vector
// register and the addend in a scalar pair (one scalar operand per
// instruction), which the compiler's own form would move into vector
// registers on every call.
__device__ __forceinline__ void philox_sweep_pair(uint4 (&x)[2], uint32_t w, const PhiloxSweep &u, Key2 key) {
    const uint32_t m1 = 0xCD9E8D57u;
    uint64_t q;
    asm("v_mad_u64_u32 %0, vcc, %1, %2, %3" : "=v"(q) : "v"(w), "v"(m1), "s"((uint64_t)m1) : "vcc");
    const uint64_t p1[2] = {(uint64_t)m1 * (uint64_t)w, q};
    philox_sweep_from<2>(x, p1, u, key);
}

__device__ __forceinline__ uint4 philox_sweep(uint32_t w, const PhiloxSweep &u, Key2 key) {
    uint4 x[1];
    const uint32_t ws[1] = {w};
    philox_sweep_multi<1>(x, ws, u, key);
    return x[0];
}

// Counter word 2: phase in the top bit, block index below it.
constexpr uint32_t kPhaseHidden = 0u;
constexpr uint32_t kPhaseVisible = 0x80000000u;

}  // namespace hp
