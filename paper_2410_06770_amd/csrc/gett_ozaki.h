// gett_ozaki.h -- launch descriptors of the DGETT emulated on INT8 matrix
// cores (Ozaki scheme): per-row exponents, 7-bit slices, and the slice-pair
// GEMM with the double combination.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gett {

constexpr int kOzMinSlices = 3, kOzMaxSlices = 8;
constexpr int64_t kOzMaxKSlice = 16384;   // positions per K slice: exact INT32 sums

// One operand's canonical rows (as the FP8 path walks them): rows R with
// offsets offR (GEMM order), or with rowsFast the rows in the operand's
// memory order (offR) and their GEMM rows (rowMap); contracted offsets offK.
struct OzOperand {
    const double *X;
    const int64_t *offR;
    const int32_t *rowMap;
    int64_t R;
    const int64_t *offK;
    int64_t K;
    bool rowsFast;
};

struct OzParams {
    const uint8_t *A, *B;      // slice 0 planes; slice s at + s * planeA / planeB bytes
    int64_t planeA, planeB;
    const int32_t *EA, *EB;    // row exponents (fill value for all-zero rows)
    int64_t Kq;                // packed row length (multiple of 64)
    int64_t kPer;              // positions per K slice (multiple of 64, <= kOzMaxKSlice)
    int32_t tilesM, tilesN, splits, pad_;
    double *C;
    const int64_t *offCM, *offCN;
    int64_t M, N;
    double *ws;                // FP64 partials [split][M][N] when splits > 1, else null
};

// E[0 .. Epad) filled, then the exponents of the operand's rows folded in.
int launch_oz_exponents(const OzOperand &o, int64_t Kq, int32_t *E, int64_t Epad, hipStream_t s);
// S slices (3 .. 8) of the operand's rows: plane s at P + s * plane bytes.
int launch_oz_slices(int S, const OzOperand &o, int64_t Kq, uint8_t *P, int64_t plane,
                     const int32_t *E, hipStream_t s);
// The slice-pair GEMM on 64 x 64 tiles (8 waves), grid tilesM * tilesN * splits.
int launch_oz_gemm(int S, const OzParams &g, hipStream_t s);

}  // namespace gett
