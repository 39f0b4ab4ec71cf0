// Sum over the 64 lanes of a wave in a fixed order, for the row-per-wave
// kernels of the smallest n.
#pragma once

#include <hip/hip_runtime.h>

namespace nbody {

// v plus v of the lane that DPP control CTRL names (all 64 lanes active).
template <int CTRL>
__device__ __forceinline__ float dpp_swap_add(float v)
{
    const int o = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false);
    return v + __builtin_bit_cast(float, o);
}

// Every lane gets the same bits: each step adds lane pairs that exchange
// values, and a + b rounds as b + a.  Call with all 64 lanes active.
__device__ __forceinline__ float wave_sum(float v)
{
    v = dpp_swap_add<0xB1>(v);   // quad_perm [1,0,3,2]: lane l ^ 1
    v = dpp_swap_add<0x4E>(v);   // quad_perm [2,3,0,1]: lane l ^ 2
    v = dpp_swap_add<0x141>(v);  // row_half_mirror: the other quad of 8 lanes
    v = dpp_swap_add<0x140>(v);  // row_mirror: the other half of 16 lanes
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

}  // namespace nbody
