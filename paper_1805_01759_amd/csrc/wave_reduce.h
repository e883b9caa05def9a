// Wave-level FP64 helpers shared by the FP64 kernels (refinement, certificate).
#pragma once
#include <hip/hip_runtime.h>

namespace l1ls {
namespace wr {

// value of v held by lane i (i uniform across the wave)
__device__ __forceinline__ double lane_value(double v, int i)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), i);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), i);
    return __hiloint2double(hi, lo);
}

// Wave reductions over DPP lane moves (register to register, no LDS round
// trip): a row-wise inclusive scan with row_shr 1, 2, 4, 8 leaves each 16-lane
// row's total in its lane 15; row_bcast 15 and 31 carry the row totals into
// lane 63, which is broadcast.  Lanes whose source falls outside the row read
// 0, so the max form is for non-negative values.  All 64 lanes must be active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wsum(double v)
{
    v += dpp_move<0x111, 0xF>(v);  // row_shr:1
    v += dpp_move<0x112, 0xF>(v);  // row_shr:2
    v += dpp_move<0x114, 0xF>(v);  // row_shr:4
    v += dpp_move<0x118, 0xF>(v);  // row_shr:8
    v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 -> rows 1, 3
    v += dpp_move<0x143, 0xC>(v);  // row_bcast:31 -> rows 2, 3
    return lane_value(v, 63);
}
__device__ __forceinline__ double wmax(double v)  // v >= 0
{
    v = fmax(v, dpp_move<0x111, 0xF>(v));
    v = fmax(v, dpp_move<0x112, 0xF>(v));
    v = fmax(v, dpp_move<0x114, 0xF>(v));
    v = fmax(v, dpp_move<0x118, 0xF>(v));
    v = fmax(v, dpp_move<0x142, 0xA>(v));
    v = fmax(v, dpp_move<0x143, 0xC>(v));
    return lane_value(v, 63);
}

}  // namespace wr
}  // namespace l1ls
