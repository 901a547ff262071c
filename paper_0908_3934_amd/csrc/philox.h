// Counter-based random numbers for the device code of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace geonet {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64-bit multiplies with
// the Weyl key schedule.  Counter x, key (k0, k1).
__device__ __forceinline__ uint4 philox4x32_10(uint4 x, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // each 32 x 32 -> 64-bit product in one v_mad_u64_u32
        const uint64_t pa = static_cast<uint64_t>(x.x) * 0xD2511F53u;
        const uint64_t pc = static_cast<uint64_t>(x.z) * 0xCD9E8D57u;
        x = make_uint4(static_cast<uint32_t>(pc >> 32) ^ x.y ^ k0, static_cast<uint32_t>(pc),
                       static_cast<uint32_t>(pa >> 32) ^ x.w ^ k1, static_cast<uint32_t>(pa));
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return x;
}

}  // namespace geonet
