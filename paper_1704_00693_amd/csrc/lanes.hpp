// Cross-lane moves inside one 64-lane wavefront through DPP (wave_shr:1 and
// wave_shl:1): a VALU move with no LDS traffic.  lane_prev gives every lane
// the value of the lane below it (lane 0 receives 0), lane_next the value of
// the lane above it (lane 63 receives 0).  Two moves make a shift by two.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tc {

__device__ __forceinline__ int dpp_prev(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int dpp_next(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }

__device__ __forceinline__ double lane_prev(double v) {
    const int64_t u = __builtin_bit_cast(int64_t, v);
    const int lo = dpp_prev((int)u), hi = dpp_prev((int)(u >> 32));
    return __builtin_bit_cast(double, (int64_t)(uint32_t)lo | ((int64_t)hi << 32));
}
__device__ __forceinline__ double lane_next(double v) {
    const int64_t u = __builtin_bit_cast(int64_t, v);
    const int lo = dpp_next((int)u), hi = dpp_next((int)(u >> 32));
    return __builtin_bit_cast(double, (int64_t)(uint32_t)lo | ((int64_t)hi << 32));
}
__device__ __forceinline__ float lane_prev(float v) {
    return __builtin_bit_cast(float, dpp_prev(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ float lane_next(float v) {
    return __builtin_bit_cast(float, dpp_next(__builtin_bit_cast(int, v)));
}

}  // namespace tc
