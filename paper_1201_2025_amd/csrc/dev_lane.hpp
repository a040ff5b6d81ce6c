// dev_lane.hpp -- FP64 exchanges between the lanes of a wavefront without the LDS
// crossbar: DPP moves within rows of 16 lanes and scalar reads of one lane.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hsad {

// An FP64 value from another lane by DPP (both 32-bit halves); CTRL is the DPP control.
template <int CTRL> __device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// The FP64 value of lane l (l uniform): a scalar read, no LDS round trip.
__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum over the 64 lanes of a wavefront (all active), the same value in every lane: pairs,
// quads, half rows and rows of 16 by DPP (quad_perm [1,0,3,2] and [2,3,0,1], row_half_mirror,
// row_mirror), then the four row sums by scalar reads.  Shuffles would take six LDS
// crossbar round trips in a row.
__device__ __forceinline__ double wave_sum64(double v)
{
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    v += dpp_f64<0x140>(v);
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

}  // namespace hsad
