// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
// as easy as 1, 2, 3", SC'11), usable on host and device.
//
// Ten rounds on a 128-bit counter with a 64-bit key.  A round multiplies counter words 0 and 2 by
// the two Philox multipliers, splits each 64-bit product into high and low halves, and forms the
// new counter (hi(w2*M1) ^ w1 ^ key0, lo(w2*M1), hi(w0*M0) ^ w3 ^ key1, lo(w0*M0)).  The key is
// advanced by the two Weyl constants between rounds.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssqa {

struct Philox4 {
    uint32_t v[4];
};

constexpr uint32_t kPhiloxMul0 = 0xD2511F53u;
constexpr uint32_t kPhiloxMul1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxWeyl0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxWeyl1 = 0xBB67AE85u;

__host__ __device__ inline Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                  uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += kPhiloxWeyl0;
            k1 += kPhiloxWeyl1;
        }
        // one 32 x 32 -> 64-bit product per multiplier (a single v_mad_u64_u32 on the GPU)
        const uint64_t p0 = (uint64_t)kPhiloxMul0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxMul1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return Philox4{{c0, c1, c2, c3}};
}

}  // namespace ssqa
