// gett_config.h -- tile menus, split-K rule and launch descriptors shared by
// the host planner and the gfx950 kernels.
//
// A planned contraction is a GEMM over three linearised index spaces:
//   M = free modes of the (possibly swapped) A operand,
//   N = free modes of the B operand,
//   K = contracted pairs,
// and every element address comes from per-group offset tables:
//   C[offCM[m] + offCN[n]] += sum_k A[offAM[m] + offAK[k]] * B[offBK[k] + offBN[n]].
// Section 6 of the paper computes the same sums by walking the free and the
// contracted coordinates with odometers (Algorithms 1 and 2); the tables hold
// exactly the increment-times-coordinate sums those walks produce, once per
// group instead of once per term.
#pragma once

#include <stdint.h>

namespace gett {

// Real precisions 0-3; complex data (interleaved real and imaginary parts,
// Section 2.3's c and z prefixes): kZ64 = complex FP64 on FP64 MFMA, kC32 =
// complex FP32 on FP32 MFMA, four real products per complex term.
enum Prec : int { kF64 = 0, kF32 = 1, kBF3 = 2, kFP8 = 3, kZ64 = 4, kC32 = 5 };
constexpr int kNumPrec = 6;
constexpr bool prec_complex(int prec) { return prec == kZ64 || prec == kC32; }
// Bytes of one element of the precision's data.
constexpr int prec_bytes(int prec) {
    return prec == kF64 ? 8 : prec == kZ64 ? 16 : prec == kC32 ? 8 : 4;
}

constexpr int kThreads = 256;       // 4 waves of 64 per workgroup
constexpr int kLdsPerCu = 160 * 1024;   // LDS of one CU (gfx950)
constexpr int kNumTiles = 5;        // tile menu size per precision
constexpr int kNumOrders = 4;
constexpr int kNumSplits = 4;       // split-K options: 1, 2, 4 slices, or "fill"
constexpr int kSplitFactor[kNumSplits] = {1, 2, 4, 0};   // 0 = enough slices to fill the chip
constexpr int kFillTarget = 2048;   // workgroups the "fill" option aims at
constexpr int kMaxSplits = 4096;

// Number of K slices actually launched for split option `split`: every slice
// starts below K (so the kernel's look-ahead loads stay inside the padded
// contracted tables) and gets at least two K steps.
inline int split_count(int split, int64_t tiles, int64_t K, int bk, int64_t *kPer) {
    int64_t S = kSplitFactor[split];
    if (S == 0) {
        S = tiles >= kFillTarget ? 1 : (kFillTarget + tiles - 1) / tiles;
        const int64_t maxS = K / (2 * (int64_t)bk);
        if (S > maxS) S = maxS;
        if (S > kMaxSplits) S = kMaxSplits;
    }
    if (S < 1) S = 1;
    int64_t per = (K + S - 1) / S;
    per = (per + bk - 1) / bk * bk;
    S = (K + per - 1) / per;
    if (kPer) *kPer = per;
    return (int)S;
}
constexpr int kTablePad = 256;      // M/N tables padded to a multiple of this

// load_fence: the compiler keeps the next step's global loads ahead of the
// step's MFMA block (a scheduling barrier between them).  Without it the
// loads may move into the MFMA block; which is faster depends on the tile
// (measured on gfx950 per precision and tile).
// depth: how many K steps ahead of the MFMAs the global loads run (1 or 2).
// Depth 2 keeps two register sets of staged values, so a load has two steps
// of MFMA work to land in instead of one.
// addr32: when both operands' addressed spans fit 4 GB, the tile loads
// through a uniform 64-bit base plus 32-bit lane offsets (fewer VALU
// instructions per value; real precisions, measured per tile).
// packed (BF16x3, FP64): the entry is the packed form -- a pass writes each
// operand element once into dense rows (BF16x3: split into bfloat16 hi/lo),
// then a GEMM kernel runs on those rows (its own kernels; the other flags do
// not apply).
struct TileShape { int bm, bn, bk; bool load_fence; int depth; bool addr32; bool packed; };

// Tile menus.  FP64/FP32 run 16x16x4 MFMA steps (BK multiple of 4), the BF16x3
// path 16x16x32 BF16 MFMA steps (BK multiple of 32).  Each workgroup is a 2x2
// grid of waves, so BM and BN are multiples of 32.  BF16x3 entries 1 and 4
// and FP64 entry 4 are the packed forms (GEMM tiles on packed rows, 32
// (BF16x3) or 16 (FP64) positions a step).
constexpr TileShape kTiles[kNumPrec][kNumTiles] = {
    /* FP64   */ {{64, 64, 16, true, 1, true}, {64, 128, 16, true, 1, true},
                  {128, 64, 16, false, 1, false}, {128, 128, 16, true, 1, true},
                  {128, 128, 16, true, 1, false, true}},
    /* FP32   */ {{64, 64, 16, true, 2, true}, {64, 128, 16, true, 2, true},
                  {128, 64, 16, true, 2, true}, {128, 128, 16, true, 2, true},
                  {128, 128, 32, true, 2, true}},
    /* BF16x3 */ {{64, 64, 32, true, 1, true}, {192, 256, 32, true, 1, false, true},
                  {128, 64, 32, true, 1, true}, {128, 128, 32, true, 1, false},
                  {128, 128, 32, true, 1, false, true}},
    /* FP8    */ {{64, 64, 128, true, 1, false}, {64, 128, 128, true, 1, false},
                  {128, 64, 128, true, 1, false}, {128, 128, 128, true, 1, false},
                  {128, 128, 128, true, 1, false}},
    /* Z64    */ {{64, 64, 8, true, 1, false}, {64, 128, 8, true, 1, false},
                  {128, 64, 8, true, 1, false}, {128, 128, 8, true, 1, false},
                  {64, 64, 16, true, 1, false}},
    /* C32    */ {{64, 64, 16, true, 1, false}, {64, 128, 16, true, 1, false},
                  {128, 64, 16, true, 1, false}, {128, 128, 16, true, 1, false},
                  {128, 128, 8, true, 1, false}},
};

// The direct 128 x 128 tile (entry 3 of the BF16x3 and FP64 menus): it runs
// in a packed entry's place when the packed rows would not fit the
// workspace cap, and in the allocation-free entry.
constexpr int kPackedFallbackTile = 3;

// Flag of the menu entry with this shape (first match).
constexpr bool tile_load_fence(int prec, int bm, int bn, int bk) {
    for (int t = 0; t < kNumTiles; ++t)
        if (kTiles[prec][t].bm == bm && kTiles[prec][t].bn == bn && kTiles[prec][t].bk == bk)
            return kTiles[prec][t].load_fence;
    return true;
}

constexpr bool tile_addr32(int prec, int bm, int bn, int bk) {
    for (int t = 0; t < kNumTiles; ++t)
        if (kTiles[prec][t].bm == bm && kTiles[prec][t].bn == bn && kTiles[prec][t].bk == bk)
            return kTiles[prec][t].addr32;
    return false;
}

constexpr int tile_depth(int prec, int bm, int bn, int bk) {
    for (int t = 0; t < kNumTiles; ++t)
        if (kTiles[prec][t].bm == bm && kTiles[prec][t].bn == bn && kTiles[prec][t].bk == bk)
            return kTiles[prec][t].depth;
    return 1;
}

// Arguments of one tile kernel launch (passed by value in the kernarg segment).
struct TileParams {
    const void *A;
    const void *B;
    void *C;
    const int64_t *offAM, *offCM;   // M tables (padded)
    const int64_t *offBN, *offCN;   // N tables (padded)
    const int64_t *offAK, *offBK;   // K tables (padded to a multiple of BK)
    int64_t M, N, K;
    int64_t kPerSplit;              // contracted positions per split (multiple of BK)
    int32_t tilesM, tilesN, splits;
    int32_t bBoxX;                  // B loader sub-box width along its fast free mode
    double *ws;                     // split-K partials [h][split][M][N] (complex: re, im
                                    // pairs), n fastest; null = direct
    // Lowest element offset either operand addresses (free plus contracted
    // table minima, padding included), and whether each operand's whole
    // addressed span fits 32-bit byte offsets from there: then the FP64/FP32
    // tiles address it as a uniform 64-bit base plus a 32-bit lane offset.
    int64_t aLo, bLo;
    int32_t off32;
    // Hadamard modes (shared by A, B and C): H positions, each with its own
    // base offsets into A, B and C; the grid runs every tile once per
    // position.  H = 1 and null tables without Hadamard modes.
    int32_t H;
    const int64_t *offAH, *offBH, *offCH;
    // C <- alpha * sum + beta * C_in ((re, im) pairs; im is 0 for real
    // data); beta == 0 does not read C.  alpha = beta = 1 is the paper's
    // accumulate.
    double alpha[2], beta[2];
#ifdef GETT_ADDR_CHECK
    // Checked build only: the addressed element ranges [lo, lo + span] of A,
    // B and C (C from its own increments) that every access is tested against.
    int64_t aSpan, bSpan, cLo, cSpan;
#endif
};

// Tiles compiled into the persistent batch kernel (menu indices of each
// precision): every problem of a batch runs one of them, chosen per problem
// by the schedule policy, and a uniform switch in the kernel picks it.
constexpr int kBatchTiles = 2;
constexpr int kBatchTile[kNumPrec][kBatchTiles] = {{0, 2}, {0, 2}, {0, 2}, {0, 0}, {0, 0}, {0, 0}};

// One problem of a batched launch (device-resident descriptor).
struct BatchProblem {
    TileParams p;
    int32_t aFastK, bFastK;
    int32_t tileBase;               // first work item of this problem
    int32_t tsel;                   // which batch tile (index into kBatchTile) it runs
};

}  // namespace gett
