// Workgroup renumbering for the 8 XCDs of the chip.
#pragma once

namespace adct {

// Workgroups are dealt to the XCDs in turn (workgroup b runs on XCD b % 8),
// each with its own L2.  xcd_swizzle(b, nb) is a bijection of [0, nb) that
// gives every XCD one contiguous run of the logical numbering, so work items
// that are neighbours in that numbering (and share cache lines at their
// seams) run on the same L2 at about the same time.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_swizzle(int b, int nb) {
    const int x = b % kXcds, i = b / kXcds, q = nb / kXcds, r = nb % kXcds;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

}  // namespace adct
