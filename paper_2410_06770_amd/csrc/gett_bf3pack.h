// gett_bf3pack.h -- launch descriptors of the packed forms (BF16x3 and FP64):
// the pack pass and the GEMMs on the packed rows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gett {

constexpr int kPackedBK = 32;                     // packed positions per step
constexpr int64_t kPackedMaxKq = (int64_t)1 << 24;   // row length limit (32-bit lane offsets)

// Arguments of one packed GEMM launch.  A and B hold the hi planes of the
// packed operands (rows padded to the tile, Kq positions each, in blocks of
// 16 rows by 32 positions), the lo planes follow at +planeA / +planeB
// elements.
struct Bf3Packed {
    const uint16_t *A, *B;
    int64_t planeA, planeB;
    int64_t Kq;          // packed row length (multiple of 32)
    int64_t kPer;        // packed positions per K slice (multiple of 32)
    int32_t tilesM, tilesN, splits, pad_;
    float *C;
    const int64_t *offCM, *offCN;
    int64_t M, N;
    double *ws;          // FP64 partials [split][M][N] when splits > 1, else null
    double alpha, beta;  // C <- alpha * sum + beta * C_in (beta == 0: C_in not read)
};

// Pack one operand: rows R (table offR in GEMM order, or with rowsFast the
// rows in the operand's memory order with rowMap giving each one's GEMM row).
// BF16x3 (f64 false): float values split into hi plane P and lo plane
// P + plane (bfloat16 elements); FP64: double values copied into plane P.
int launch_pack(bool f64, const void *X, const int64_t *offR, const int32_t *rowMap, int64_t R,
                const int64_t *offK, int64_t K, int64_t Kq, bool rowsFast, void *P, int64_t plane,
                hipStream_t s);

// The packed FP64 form: planes of doubles in 2 KB blocks of 16 rows by 16
// positions; GEMM tile 128 x 128 (4 waves, two workgroups per CU).
constexpr int kPacked64BK = 16;   // packed positions per step
struct F64Packed {
    const double *A, *B;
    int64_t Kq;          // packed row length (multiple of 16)
    int64_t kPer;        // packed positions per K slice (multiple of 16)
    int32_t tilesM, tilesN, splits, pad_;
    double *C;
    const int64_t *offCM, *offCN;
    int64_t M, N;
    double *ws;          // FP64 partials [split][M][N] when splits > 1, else null
    double alpha, beta;  // C <- beta * C_in + alpha * sum (beta == 0: C_in not read)
};
int launch_f64_packed_gemm(const F64Packed &g, hipStream_t s);

// GEMM tiles (bm x bn): 128 x 128 (4 waves, two workgroups per CU) and
// 192 x 256 (8 waves, one per CU); rows padded to the tile.
int launch_bf3_packed_gemm(int bm, int bn, const Bf3Packed &g, hipStream_t s);

}  // namespace gett
