// Workgroup order across the XCDs.  The hardware hands the workgroups of a
// launch to the eight XCDs in turn (workgroup b to XCD b mod 8), and each
// XCD has its own L2; renumbering them so that XCD x takes one contiguous
// range of logical blocks keeps neighbouring blocks, whose loads and gathers
// overlap, in one L2.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hbmc {

constexpr int kXcds = 8;

// logical block of hardware block b among nb (a bijection of [0, nb))
__device__ inline int64_t xcd_block(int64_t b, int64_t nb) {
    const int64_t x = b % kXcds, i = b / kXcds, q = nb / kXcds, r = nb % kXcds;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

}  // namespace hbmc
