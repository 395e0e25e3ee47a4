// gett_fp8.hip -- the FP8 (OCP E4M3) path of SGETT.
//
// quant:  one wave per (row, 128-block): the wave gathers the block's 128
//         values through the row and contracted offset tables, finds the
//         largest magnitude, picks the power-of-two scale 2^e (smallest e >=
//         -127 with amax / 2^e <= 448; exact integer logic on the binary
//         exponent), and writes the E4M3 codes (round to nearest even) into a
//         dense K-contiguous row, with e beside it.
// gemm:   both operands are then dense [rows][Kp] byte matrices, the shape the
//         16x16x128 FP8 MFMA reads directly: each lane takes 32 consecutive
//         codes of one row.  The block scales go in as the MFMA's E8M0 scale
//         operands (bias 127), so the matrix core applies 2^(eA + eB) to each
//         128-block product exactly and accumulates in FP32.  The epilogue
//         scatters through the C offset tables (PERM and INCC) and adds C_in.
#include "gett_internal.h"

namespace gett {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef int i8_t __attribute__((ext_vector_type(8)));

// Scale exponent from the block maximum (see file comment).
__device__ __forceinline__ int fp8_scale_exp(float amax) {
    if (!(amax > 0.f)) return 0;
    const unsigned u = __float_as_uint(amax);
    int x;              // amax = f * 2^x with f in [0.5, 1)
    float f;
    const int be = (int)((u >> 23) & 0xFF);
    if (be == 0) {      // subnormal
        f = frexpf(amax, &x);
    } else {
        x = be - 126;
        f = __uint_as_float((u & 0x807FFFFFu) | (126u << 23));
    }
    int e = f <= 0.875f ? x - 9 : x - 8;
    return e < -127 ? -127 : e;
}

// Encode v (|v| <= 448 by construction) to E4M3 with the hardware converter
// (round to nearest even); returns the code in the low byte.
__device__ __forceinline__ unsigned e4m3_code(float v) {
    const int packed = __builtin_amdgcn_cvt_pk_fp8_f32(v, 0.f, 0, false);
    return (unsigned)packed & 0xFFu;
}

__global__ __launch_bounds__(256) void fp8_quant_kernel(const float *__restrict__ X,
                                                        const int64_t *__restrict__ offR,
                                                        int64_t rows, int64_t rowsPad,
                                                        const int64_t *__restrict__ offK,
                                                        int64_t K, uint8_t *__restrict__ Q,
                                                        int32_t *__restrict__ E) {
    const int64_t nb = (K + 127) / 128;
    const int64_t Kp = nb * 128;
    const int lane = threadIdx.x & 63;
    const int64_t task = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);   // one wave per task
    if (task >= rowsPad * nb) return;
    const int64_t r = task / nb, blk = task - r * nb;
    uint8_t *q = Q + r * Kp + blk * 128;
    if (r >= rows) {     // padding rows of the operand: zero codes, zero exponent
        q[2 * lane] = 0;
        q[2 * lane + 1] = 0;
        if (lane == 0) E[r * nb + blk] = 0;
        return;
    }
    const int64_t base = offR[r];
    const int64_t k0 = blk * 128 + 2 * lane;
    const float v0 = k0 < K ? X[base + offK[k0]] : 0.f;
    const float v1 = k0 + 1 < K ? X[base + offK[k0 + 1]] : 0.f;
    float amax = fmaxf(fabsf(v0), fabsf(v1));
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) amax = fmaxf(amax, __shfl_xor(amax, s, 64));
    const int e = fp8_scale_exp(amax);
    const float inv = ldexpf(1.f, -e);    // exact power of two (e >= -127: 2^127 fits)
    const unsigned c0 = k0 < K ? e4m3_code(v0 * inv) : 0u;
    const unsigned c1 = k0 + 1 < K ? e4m3_code(v1 * inv) : 0u;
    *reinterpret_cast<uint16_t *>(q + 2 * lane) = (uint16_t)(c0 | (c1 << 8));
    if (lane == 0) E[r * nb + blk] = e;
}

// C tile BM x BN, 4 waves as 2 x 2, each wave (BM/2) x (BN/2) in 16x16 fragments.
template <int BM, int BN>
__global__ __launch_bounds__(256) void fp8_gemm_kernel(const uint8_t *__restrict__ QA,
                                                       const int32_t *__restrict__ EA,
                                                       const uint8_t *__restrict__ QB,
                                                       const int32_t *__restrict__ EB,
                                                       float *__restrict__ C,
                                                       const int64_t *__restrict__ offCM,
                                                       const int64_t *__restrict__ offCN,
                                                       int64_t M, int64_t N, int64_t K,
                                                       int tilesM, int tilesN) {
    constexpr int WTM = BM / 2, WTN = BN / 2, FM = WTM / 16, FN = WTN / 16;
    constexpr int LDK = 128 + 16;            // bytes per LDS row (16-byte pad)
    __shared__ __align__(16) uint8_t sA[BM * LDK];
    __shared__ __align__(16) uint8_t sB[BN * LDK];
    __shared__ int32_t sEA[BM], sEB[BN];

    const int64_t nb = (K + 127) / 128;
    const int64_t Kp = nb * 128;
    const int bid = blockIdx.x;
    const int tm = bid % tilesM, tn = bid / tilesM;
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;

    f4_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

    for (int64_t blk = 0; blk < nb; ++blk) {
        // stage the 128-wide block of both operands (rows are padded to 128)
        for (int c = t; c < BM * 8; c += 256) {
            const int r = c >> 3, part = c & 7;
            const uint4 v = *reinterpret_cast<const uint4 *>(QA + (m0 + r) * Kp + blk * 128 + part * 16);
            *reinterpret_cast<uint4 *>(sA + r * LDK + part * 16) = v;
        }
        for (int c = t; c < BN * 8; c += 256) {
            const int r = c >> 3, part = c & 7;
            const uint4 v = *reinterpret_cast<const uint4 *>(QB + (n0 + r) * Kp + blk * 128 + part * 16);
            *reinterpret_cast<uint4 *>(sB + r * LDK + part * 16) = v;
        }
        for (int r = t; r < BM; r += 256) sEA[r] = EA[(m0 + r) * nb + blk];
        for (int r = t; r < BN; r += 256) sEB[r] = EB[(n0 + r) * nb + blk];
        __syncthreads();
        i8_t a[FM], b[FN];
        int sa[FM], sb[FN];
        const int kc = 32 * (lane >> 4);
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            const int r = wm * WTM + i * 16 + (lane & 15);
            a[i] = *reinterpret_cast<const i8_t *>(sA + r * LDK + kc);
            sa[i] = sEA[r] + 127;
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int r = wn * WTN + j * 16 + (lane & 15);
            b[j] = *reinterpret_cast<const i8_t *>(sB + r * LDK + kc);
            sb[j] = sEB[r] + 127;
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                    a[i], b[j], acc[i][j], 0, 0, 0, sa[i], 0, sb[j]);
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int64_t n = n0 + wn * WTN + j * 16 + (lane & 15);
        if (n >= N) continue;
        const int64_t ocn = offCN[n];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t m = m0 + wm * WTM + i * 16 + 4 * (lane >> 4) + v;
                if (m >= M) continue;
                const int64_t off = offCM[m] + ocn;
                C[off] = C[off] + acc[i][j][v];
            }
    }
}

int launch_fp8_quant(const float *X, const int64_t *offR, int64_t rows, int64_t rowsPad,
                     const int64_t *offK, int64_t K, uint8_t *Q, int32_t *E, hipStream_t s) {
    const int64_t nb = (K + 127) / 128;
    const int64_t tasks = rowsPad * nb;
    const int64_t blocks = (tasks + 3) / 4;
    if (blocks > INT32_MAX) return GETT_ERR_INTERNAL;
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    hipLaunchKernelGGL(fp8_quant_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, offR, rows,
                       rowsPad, offK, K, Q, E);
    return launch_status();
}

int launch_fp8_gemm(int tile, const uint8_t *QA, const int32_t *EA, const uint8_t *QB,
                    const int32_t *EB, float *C, const int64_t *offCM, const int64_t *offCN,
                    int64_t M, int64_t N, int64_t K, hipStream_t s) {
    if (tile == 3) {
        const int tilesM = (int)((M + 127) / 128), tilesN = (int)((N + 127) / 128);
        (void)hipGetLastError();   // clear a stale error left by other HIP users
        hipLaunchKernelGGL((fp8_gemm_kernel<128, 128>), dim3(tilesM * tilesN), dim3(256), 0, s, QA,
                           EA, QB, EB, C, offCM, offCN, M, N, K, tilesM, tilesN);
    } else {
        // operands are padded to multiples of 128 rows, so 64-row tiles stay inside
        const int tilesM = (int)((M + 63) / 64), tilesN = (int)((N + 63) / 64);
        (void)hipGetLastError();   // clear a stale error left by other HIP users
        hipLaunchKernelGGL((fp8_gemm_kernel<64, 64>), dim3(tilesM * tilesN), dim3(256), 0, s, QA,
                           EA, QB, EB, C, offCM, offCN, M, N, K, tilesM, tilesN);
    }
    return launch_status();
}

}  // namespace gett
