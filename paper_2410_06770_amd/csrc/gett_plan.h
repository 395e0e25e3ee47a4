// gett_plan.h -- host planner: argument checks, M/N/K grouping, offset tables.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace gett {

// The 14 xGETT arguments (Section 5.7), pointers excluded, and the Hadamard
// pairs of the extended calls: mode hada[h] of A and mode hadb[h] of B are
// one index carried by A, B and C alike (neither summed nor free; Section 9
// lists such batch modes as future work).  Output modes: A's free modes,
// B's free modes, then the Hadamard pairs, placed by PERM.
struct Args {
    int64_t ranka;
    const int64_t *exta, *inca;
    int64_t rankb;
    const int64_t *extb, *incb;
    int64_t conts;
    const int64_t *conta, *contb, *perm, *incc;
    int64_t hads = 0;
    const int64_t *hada = nullptr, *hadb = nullptr;
};

// INFO codes of validate beyond the 14 of the paper's argument list.
constexpr int kInfoHads = -101, kInfoHada = -102, kInfoHadb = -103;

// LAPACK-style INFO (0 or -i, i in the 14-argument order; kInfoHad* for the
// Hadamard lists).  Pointers are only tested against NULL.
int validate(const Args &a, const void *A, const void *B, const void *C);

// Number of output modes: RANKA + RANKB - 2 CONTS - HADS.
inline int64_t out_rank(const Args &a) { return a.ranka + a.rankb - 2 * a.conts - a.hads; }

// Extents and increments of C by output position (valid arguments only).
void output_modes(const Args &a, std::vector<int64_t> &ext, std::vector<int64_t> &inc);

// One mode of a group: extent and the increments of the two tensors that
// carry the group (M: A and C; N: B and C; K: A and B).
struct GMode {
    int64_t ext;
    int64_t i0, i1;
};

// A Hadamard mode: extent and the increments in A, B and C.
struct HMode {
    int64_t ext, ia, ib, ic;
};

// The contraction as a GEMM over three mode groups, repeated over the
// positions of the Hadamard group.
struct Canon {
    bool empty = false;          // a zero extent: nothing to do
    bool swapped = false;        // A and B exchanged (so that C's fastest mode is in N)
    std::vector<GMode> m, n, k;  // ordered, first mode fastest
    std::vector<HMode> h;        // Hadamard modes (increments follow any swap)
    int64_t M = 1, N = 1, K = 1, H = 1;
    bool aFastK = false, bFastK = false;
    int boxX = 0;                // B loader box width (0: none)
};

// Canonicalise for mode-ordering option `order` (0..3) and tile width bn.
// Every order swaps A and B when C's fastest mode belongs to A, merges
// jointly contiguous modes, orders M by A's strides and K by the operand
// that reads along K; they differ in the N order:
//   0: N by B's strides (the B loads coalesce);
//   1: N by C's strides (the epilogue's stores coalesce);
//   2: N boxed, 4 positions of C's fastest N mode by bn/4 of B's;
//   3: N boxed, 16 positions of C's fastest N mode by bn/16 of B's.
// Boxes fall back to order 0 when the extents do not divide.
Canon canonicalise(const Args &a, int order, int bn);

// Offsets of a group for tensor slot s (0: i0, 1: i1), padded with zeros to
// `padded` entries; first mode fastest.
void group_offsets(const std::vector<GMode> &g, int slot, int64_t padded, int64_t *out);

// Offsets of the Hadamard group in A, B and C (H entries each, first mode
// fastest) into outA/outB/outC.
void hadamard_offsets(const std::vector<HMode> &h, int64_t *outA, int64_t *outB, int64_t *outC);

// Smallest and largest entry of a group's offset table for slot s (padding
// zeros included): every coordinate combination occurs, so each mode
// contributes min(0, inc (ext - 1)) and max(0, inc (ext - 1)).
void group_range(const std::vector<GMode> &g, int slot, int64_t &lo, int64_t &hi);

// Element range each operand of a canonical form can address (free table
// plus contracted table): lowest offset and span, for A (M, K slot 0) and
// B (N, K slot 1).
void operand_ranges(const Canon &c, int64_t &aLo, int64_t &aSpan, int64_t &bLo, int64_t &bSpan);

// Canonical (schedule-independent) orders used by the FP8 path: rows of A are
// A's free modes in ascending order, rows of B likewise, contracted positions
// follow the pairs in CONTA order; first fastest.  Extent-1 and zero extents
// are kept (they do not change the linear order).
void canonical_groups(const Args &a, std::vector<GMode> &rowsA, std::vector<GMode> &rowsB,
                      std::vector<GMode> &kAB);

// 64-entry feature vector of a signature for precision prec.
void features(const Args &a, int prec, float *out);

// Plan-cache key of a signature.
std::string signature_key(const Args &a, int prec, int64_t extra0, int64_t extra1);

}  // namespace gett
