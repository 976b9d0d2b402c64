// Philox4x32-10 counter-based random numbers on the device, written from
// Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC'11): ten rounds of two 32x32->64 multiplications (multipliers
// 0xD2511F53 and 0xCD9E8D57) with the key bumped by 0x9E3779B9 / 0xBB67AE85
// (golden ratio and sqrt(3)-1 Weyl increments) between rounds.
//
// Stream layout of the method (the paper only says "random"): key = the
// 64-bit seed, counter = (block, iteration, member index in swarm, swarm).
// Element e of a stream is word e & 3 of block e >> 2.
//   iteration t >= 1:  element 0 -> r2, element 1 -> r3 (eq. velocity);
//                      element 4 + i -> tie-break of SecondTarget selection i
//   iteration 0:       elements 0..n-2 -> Fisher-Yates draws,
//                      element 256 + r*n + c -> V(0) cell (r, c)
//   migration after t: member 0xFFFFFFFF, swarm 0, element k -> k-th donor
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qap {

struct Philox4 {
    uint32_t w[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo0 = 0xD2511F53u * c0;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t y0 = hi1 ^ c1 ^ k0;
        const uint32_t y2 = hi0 ^ c3 ^ k1;
        c0 = y0;
        c1 = lo1;
        c2 = y2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Philox4 r;
    r.w[0] = c0; r.w[1] = c1; r.w[2] = c2; r.w[3] = c3;
    return r;
}

// One element of a particle's stream.
__device__ __forceinline__ uint32_t stream_word(uint64_t seed, uint32_t element, uint32_t iter,
                                                uint32_t member, uint32_t swarm)
{
    const Philox4 b = philox4x32_10(element >> 2, iter, member, swarm, (uint32_t)seed,
                                    (uint32_t)(seed >> 32));
    const uint32_t e = element & 3u;
    return e == 0 ? b.w[0] : e == 1 ? b.w[1] : e == 2 ? b.w[2] : b.w[3];
}

// [0,1) from the top 24 bits (exact in binary32).
__device__ __forceinline__ float unit_float(uint32_t w) { return (float)(w >> 8) * 5.9604644775390625e-8f; }

// [0, m) by the high word of w*m.
__device__ __forceinline__ uint32_t bounded_u32(uint32_t w, uint32_t m) { return __umulhi(w, m); }

}  // namespace qap
