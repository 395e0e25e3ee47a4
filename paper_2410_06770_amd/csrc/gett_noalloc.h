// gett_noalloc.h -- internals of the allocation-free entry point: the
// per-device scratch array and the device-side writer of offset tables.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gett.h"

namespace gett {

constexpr int kMaxDevices = 64;
// A group of the canonical form has at most this many modes here.  Modes of
// extent 1 are dropped before, so a group with more modes would have at least
// 2^32 positions: far past the 2^31-entry table limit of the planner.
constexpr int kFillModes = 32;

struct FillMode {
    int64_t ext, i0, i1;
};

// The three groups (M, N, K) of a canonical form, passed by value to the
// table writer: table t of group G is slot t of its modes, padded with zeros
// to pad[G] entries; the six tables follow each other in the order
// M slot 0, M slot 1, N slot 0, N slot 1, K slot 0, K slot 1.
struct FillGroups {
    FillMode modes[3][kFillModes];
    int32_t nmodes[3];
    int32_t pad_;
    int64_t size[3];   // positions of each group (product of its extents)
    int64_t pad[3];    // padded table length of each group
};

// Device address of this device's scratch array (dev must be current on the
// calling thread); looked up once per device and kept.
int noalloc_scratch(int dev, void **ptr, int64_t *bytes);

// Write the six offset tables of `f` to out (device memory) on stream s.
int launch_table_fill(const FillGroups &f, int64_t *out, hipStream_t s);

}  // namespace gett
