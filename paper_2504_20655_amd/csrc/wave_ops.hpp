// Wave-wide helpers for CDNA's 64-lane wavefronts: 64-bit broadcasts and
// reductions.  Reductions run within rows of 16 lanes through DPP moves
// (lane xor 1, xor 2, then the half-row and row mirrors, each of which pairs
// a lane with one in the other half of its group) and combine the four rows
// through readlane; every lane of the wave must be active.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wr {

__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x >> 32));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t x, uint32_t l) {
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(x), l);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(x >> 32), l);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t x) {
    const uint32_t lo = __builtin_amdgcn_update_dpp(0u, static_cast<uint32_t>(x), CTRL, 0xF, 0xF, false);
    const uint32_t hi = __builtin_amdgcn_update_dpp(0u, static_cast<uint32_t>(x >> 32), CTRL, 0xF, 0xF, false);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

constexpr int DPP_XOR1 = 0xB1;          // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;          // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <-> 7 - i within 8
constexpr int DPP_MIRROR = 0x140;       // lane i <-> 15 - i within 16

// minimum over the wave, returned uniform
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
    uint64_t o;
    o = dpp64<DPP_XOR1>(x), x = o < x ? o : x;
    o = dpp64<DPP_XOR2>(x), x = o < x ? o : x;
    o = dpp64<DPP_HALF_MIRROR>(x), x = o < x ? o : x;
    o = dpp64<DPP_MIRROR>(x), x = o < x ? o : x;
    uint64_t r = readlane64(x, 0);
    for (uint32_t l = 16; l < 64; l += 16) {
        o = readlane64(x, l);
        r = o < r ? o : r;
    }
    return r;
}

// maximum over the wave, returned uniform
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t x) {
    uint64_t o;
    o = dpp64<DPP_XOR1>(x), x = o > x ? o : x;
    o = dpp64<DPP_XOR2>(x), x = o > x ? o : x;
    o = dpp64<DPP_HALF_MIRROR>(x), x = o > x ? o : x;
    o = dpp64<DPP_MIRROR>(x), x = o > x ? o : x;
    uint64_t r = readlane64(x, 0);
    for (uint32_t l = 16; l < 64; l += 16) {
        o = readlane64(x, l);
        r = o > r ? o : r;
    }
    return r;
}

}  // namespace wr
