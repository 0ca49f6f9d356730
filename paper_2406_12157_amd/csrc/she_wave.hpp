// Wave-level reductions over the 64 lanes with DPP moves (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace she {

// One DPP move of a double (both halves with the same control); lanes with
// no source, or outside the row / bank masks, receive 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v)
{
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(u & 0xffffffffLL), CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(u >> 32), CTRL, ROWS, 0xf, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// Inclusive prefix sum over the 64 lanes of a wave: shifts by 1, 2, 4, 8
// within rows of 16, then the last lane of row 0 / 2 into row 1 / 3 and lane
// 31 into rows 2 and 3.
__device__ __forceinline__ double wave_inclusive_sum(double v)
{
    v += dpp_move<0x111, 0xf>(v);  // row_shr:1
    v += dpp_move<0x112, 0xf>(v);  // row_shr:2
    v += dpp_move<0x114, 0xf>(v);  // row_shr:4
    v += dpp_move<0x118, 0xf>(v);  // row_shr:8
    v += dpp_move<0x142, 0xa>(v);  // row_bcast:15
    v += dpp_move<0x143, 0xc>(v);  // row_bcast:31
    return v;
}

// Sum over the wave, the same value in every lane (lane 63 of the scan).
__device__ __forceinline__ double wave_total(double v)
{
    const long long u = __double_as_longlong(wave_inclusive_sum(v));
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(u & 0xffffffffLL), 63);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(u >> 32), 63);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

}  // namespace she
