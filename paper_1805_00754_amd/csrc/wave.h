// Wavefront-level helpers for 64-lane waves on gfx950.
//
// The reductions use DPP lane permutations inside each row of 16 lanes and
// then read the four row totals with v_readlane, so they stay on the vector
// ALU (no LDS crossbar traffic) and the result is uniform across the wave.
// The order of the additions is fixed, so every call with the same inputs
// gives the same bits.  They must be called with all 64 lanes active.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zs {

// DPP controls (GFX9 encoding)
constexpr int kDppQuadXor1 = 0xB1;     // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v)
{
    const int64_t b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Value of v in lane l (l uniform), as a wave-uniform value.
__device__ __forceinline__ double readlane_d(double v, int l)
{
    const int64_t b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Sum over the 16 lanes of each row; every lane of the row gets the row total.
// Each stage adds a lane's value to its partner's, and both partners compute
// the same sum (addition is commutative), so the row total is exact-identical
// in all 16 lanes.
__device__ __forceinline__ double row16_sum(double v)
{
    v += dpp_mov<kDppQuadXor1>(v);
    v += dpp_mov<kDppQuadXor2>(v);
    v += dpp_mov<kDppRowHalfMirror>(v);
    v += dpp_mov<kDppRowMirror>(v);
    return v;
}

// Sum over all 64 lanes, returned uniform.
__device__ __forceinline__ double wave_sum64(double v)
{
    v = row16_sum(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

}  // namespace zs
