// Cross-lane moves of doubles within a 64-lane wavefront (DPP, lane reads),
// shared by the forward and the adjoint kernels.
#pragma once
#include <hip/hip_runtime.h>

// Cross-lane move of a double with a DPP pattern (two 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int l2 = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
    const int h2 = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
    return __hiloint2double(h2, l2);
}

// Row broadcast of a double (DPP row_bcast:15 / row_bcast:31): rows whose
// bit is set in ROWS receive the named lane's value, the others 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_bcast(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWS, 0xF, false);
    const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWS, 0xF, false);
    return __hiloint2double(h2, l2);
}

__device__ __forceinline__ double read_lane(double v, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Sum of v over each aligned group of N lanes (N = 1, 2, 4, 8 or 16), in
// every lane of the group: the pairwise tree of a lane-xor butterfly
// (partners 1, 2, 4, 8 apart).  Once every lane of a block holds the block's
// sum, a mirror within the row pairs it with the same neighbouring block as
// the xor would, and a + b == b + a, so the bits are the butterfly's.
template <int N>
__device__ __forceinline__ double lane_sum(double v) {
    static_assert(N == 1 || N == 2 || N == 4 || N == 8 || N == 16, "groups within a row of 16 lanes");
    if (N >= 2) v = v + dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
    if (N >= 4) v = v + dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
    if (N >= 8) v = v + dpp_mov<0x141>(v);   // row_half_mirror
    if (N >= 16) v = v + dpp_mov<0x140>(v);  // row_mirror
    return v;
}
