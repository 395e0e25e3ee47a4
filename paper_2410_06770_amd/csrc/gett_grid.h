// gett_grid.h -- workgroup-to-tile mapping shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace gett {

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Renumber them so that each XCD receives a contiguous run of logical
// tiles: neighbouring tiles share A rows or B columns in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int total) {
    const int xcd = bid & 7, local = bid >> 3;
    const int base = total >> 3, rem = total & 7;
    return xcd * base + (xcd < rem ? xcd : rem) + local;
}

// Logical tile -> (tm, tn): groups of 8 tile-rows swept along N.
__device__ __forceinline__ void tile_coords(int tile, int tilesM, int tilesN, int &tm, int &tn) {
    constexpr int GM = 8;
    const int per = GM * tilesN;
    const int g = tile / per;
    const int first = g * GM;
    const int gsz = min(tilesM - first, GM);
    const int r = tile - g * per;
    tm = first + r % gsz;
    tn = r / gsz;
}

}  // namespace gett
