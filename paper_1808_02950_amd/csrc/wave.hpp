// Wave-wide reductions on the DPP lane crossbar (no LDS, no address registers).
#pragma once

namespace adct {

// Sum over the 64 lanes: quad swaps, then rotations by 4 and 8 lanes, leave
// every lane with its 16-lane row's sum; the row broadcasts add row 0 into
// row 1 and row 2 into row 3, then lane 31 into rows 2 and 3 (lanes of the
// disabled rows keep their value), so lane 63 holds the total, which
// readlane returns to every lane.  Unsigned addition: the total is exact
// modulo 2^32.
__device__ __forceinline__ unsigned wave_sum_u32(unsigned v) {
    v += unsigned(__builtin_amdgcn_update_dpp(0, int(v), 0xb1, 0xf, 0xf, false));    // quad_perm [1,0,3,2]
    v += unsigned(__builtin_amdgcn_update_dpp(0, int(v), 0x4e, 0xf, 0xf, false));    // quad_perm [2,3,0,1]
    v += unsigned(__builtin_amdgcn_update_dpp(0, int(v), 0x124, 0xf, 0xf, false));   // row_ror:4
    v += unsigned(__builtin_amdgcn_update_dpp(0, int(v), 0x128, 0xf, 0xf, false));   // row_ror:8
    v += unsigned(__builtin_amdgcn_update_dpp(0, int(v), 0x142, 0xa, 0xf, false));   // row_bcast:15
    v += unsigned(__builtin_amdgcn_update_dpp(0, int(v), 0x143, 0xc, 0xf, false));   // row_bcast:31
    return unsigned(__builtin_amdgcn_readlane(int(v), 63));
}

}  // namespace adct
