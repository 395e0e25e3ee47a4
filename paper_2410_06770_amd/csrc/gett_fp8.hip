// gett_fp8.hip -- the FP8 (OCP E4M3) path of SGETT.
//
// quant:  each (row, 128-block) of an operand gets its largest magnitude
//         amax, the power-of-two scale 2^e (smallest e >= -127 with
//         amax / 2^e <= 448; exact integer logic on the binary exponent), and
//         E4M3 codes (round to nearest even) written into a dense
//         K-contiguous row, with e beside it.  Two loader shapes, as in the
//         tile kernels: when the contracted positions are the operand's
//         cheapest direction in memory, one wave takes a run of blocks of
//         one row with lanes along K; when the rows are, one wave takes 16 neighbouring
//         rows of one block with four lanes per row, so every load of the
//         wave reads 16 neighbours at four positions.
// gemm:   both operands are then dense [rows][Kp] byte matrices, the shape the
//         16x16x128 FP8 MFMA reads directly: each lane takes 32 consecutive
//         codes of one row.  The block scales go in as the MFMA's E8M0 scale
//         operands (bias 127), so the matrix core applies 2^(eA + eB) to each
//         128-block product exactly and accumulates in FP32.  The next
//         block's codes are loaded into registers while the current block
//         runs on the matrix cores (double-buffered LDS, one barrier per
//         block).  The epilogue scatters through the C offset tables (PERM
//         and INCC) and adds C_in.
#include "gett_grid.h"
#include "gett_internal.h"

namespace gett {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef int i8_t __attribute__((ext_vector_type(8)));
typedef unsigned u4_t __attribute__((ext_vector_type(4)));

// Element formats (kElem*, numbered as the scaled MFMA's format operands):
// OCP E4M3 (FP8), E2M3 (FP6) and E2M1 (FP4).

// Scale exponent from the block maximum: the smallest e >= -127 with
// amax / 2^e not above the format's largest magnitude vmax = F 2^X
// (F in [0.5, 1): 448 = 0.875 2^9, 7.5 = 0.9375 2^3, 6 = 0.75 2^3).  With
// amax = f 2^x, f in [0.5, 1), the condition f 2^x <= F 2^(X + e) holds from
// e = x - X when f <= F, else from x - X + 1 (exact integer logic).
template <int FMT>
__device__ __forceinline__ int fp8_scale_exp(float amax) {
    constexpr int X = FMT == kElemE4M3 ? 9 : 3;
    constexpr float F = FMT == kElemE4M3 ? 0.875f : FMT == kElemE2M3 ? 0.9375f : 0.75f;
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
    int e = f <= F ? x - X : x - X + 1;
    return e < -127 ? -127 : e;
}

// Encode v (|v| <= 448 by construction) to E4M3 with the hardware converter
// (round to nearest even); returns the code in the low byte.
__device__ __forceinline__ unsigned e4m3_code(float v) {
    const int packed = __builtin_amdgcn_cvt_pk_fp8_f32(v, 0.f, 0, false);
    return (unsigned)packed & 0xFFu;
}

// Four codes in one word, first value in the low byte.
__device__ __forceinline__ unsigned e4m3_word(float a, float b, float c, float d) {
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
    return (unsigned)w;
}

// E2M1 / E2M3 code of v (|v| <= 6 / 7.5 by construction), round to nearest
// even: sign, 2 exponent bits (bias 1), M mantissa bits.  With k = 0 below 1
// and k = floor(log2 |v|) from 1 up, the spacing is 2^(k - M) and
// n = rint(|v| 2^(M - k)) counts it; the code is k 2^M + n, which also
// covers the subnormals (k = 0), a carry into the next binade (n = 2^(M+1))
// and the largest value.  The sign bit is v's (signbit).
template <int FMT>
__device__ __forceinline__ unsigned mx_small_code(float v) {
    constexpr int M = FMT == kElemE2M1 ? 1 : 3;
    const float a = fabsf(v);
    int x;
    (void)frexpf(a, &x);                              // a = f 2^x, f in [0.5, 1)
    const int k = a < 1.f ? 0 : x - 1;
    const unsigned n = (unsigned)rintf(ldexpf(a, M - k));
    return ((unsigned)k << M) + n + (signbit(v) ? (1u << (M + 2)) : 0u);
}

template <int FMT>
__device__ __forceinline__ unsigned elem_code(float v) {
    if constexpr (FMT == kElemE4M3) return e4m3_code(v);
    else return mx_small_code<FMT>(v);
}

template <int FMT>
__device__ __forceinline__ unsigned elem_word(float a, float b, float c, float d) {
    if constexpr (FMT == kElemE4M3) return e4m3_word(a, b, c, d);
    else return mx_small_code<FMT>(a) | (mx_small_code<FMT>(b) << 8) |
                (mx_small_code<FMT>(c) << 16) | (mx_small_code<FMT>(d) << 24);
}

// Lanes along K: one wave per (row, run of up to kQuantRun consecutive
// 128-blocks); lane l takes positions l and l + 64 of each block, so each
// load instruction reads 64 neighbouring table entries and, where K runs
// contiguously, 64 neighbouring values.  All of a wave's loads are issued
// before its first block is reduced, so a run's blocks are in flight
// together (one block per wave left the loads latency-bound).  The waves of
// a workgroup take consecutive runs of one row (giving them neighbouring
// rows of one run instead measured slower, and so did renumbering the
// workgroups so that each XCD takes a contiguous range of rows).  Loads past the run's last block repeat
// that block, and positions past K read position K - 1 again (the
// contracted table holds exactly K offsets); both are discarded, so every
// load stays inside the table and the operand.
constexpr int kQuantRun = 8;

// BS: positions per scale, 128, or 32 (the MX-style blocks: lane l's two
// positions l and l + 64 fall in blocks l / 32 and 2 + l / 32 of the 128).
// FMT: element format (E4M3 with either block size; E2M3 and E2M1 with 32).
template <int BS, int FMT>
__global__ __launch_bounds__(256) void fp8_quant_kernel(const float *__restrict__ X,
                                                        const int64_t *__restrict__ offR,
                                                        int64_t rows, int64_t rowsPad,
                                                        const int64_t *__restrict__ offK,
                                                        int64_t K, uint8_t *__restrict__ Q,
                                                        int32_t *__restrict__ E) {
    constexpr int SUB = 128 / BS;                                        // scales per 128
    const int64_t nb = (K + 127) / 128;
    const int64_t Kp = nb * 128;
    const int64_t nbs = nb * SUB;
    const int64_t runs = (nb + kQuantRun - 1) / kQuantRun;
    const int lane = threadIdx.x & 63;
    const int64_t task = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);   // one wave per task
    if (task >= rowsPad * runs) return;
    const int64_t r = task / runs, run = task - r * runs, b0 = run * kQuantRun;
    const int nbl = (int)(nb - b0 < kQuantRun ? nb - b0 : kQuantRun);    // blocks in this run
    uint8_t *q = Q + r * Kp;
    if (r >= rows) {     // padding rows of the operand: zero codes, zero exponents
        for (int j = 0; j < nbl; ++j) {
            q[(b0 + j) * 128 + lane] = 0;
            q[(b0 + j) * 128 + 64 + lane] = 0;
            if (lane < SUB) E[r * nbs + (b0 + j) * SUB + lane] = 0;
        }
        return;
    }
    const int64_t base = offR[r];
    float v0[kQuantRun], v1[kQuantRun];
#pragma unroll
    for (int j = 0; j < kQuantRun; ++j) {
        const int64_t blk = j < nbl ? b0 + j : nb - 1;
        const int64_t k0 = blk * 128 + lane, k1 = k0 + 64;
        const float x0 = X[base + offK[k0 < K ? k0 : K - 1]];
        const float x1 = X[base + offK[k1 < K ? k1 : K - 1]];
        v0[j] = k0 < K ? x0 : 0.f;
        v1[j] = k1 < K ? x1 : 0.f;
    }
#pragma unroll
    for (int j = 0; j < kQuantRun; ++j) {
        if (j >= nbl) break;                            // uniform across the wave
        const int64_t k0 = (b0 + j) * 128 + lane, k1 = k0 + 64;
        if constexpr (BS == 128) {
            float amax = fmaxf(fabsf(v0[j]), fabsf(v1[j]));
#pragma unroll
            for (int s = 32; s > 0; s >>= 1) amax = fmaxf(amax, __shfl_xor(amax, s, 64));
            const int e = fp8_scale_exp<FMT>(amax);
            const float inv = ldexpf(1.f, -e);  // exact power of two (e >= -127: 2^127 fits)
            q[k0] = (uint8_t)(k0 < K ? elem_code<FMT>(v0[j] * inv) : 0u);
            q[k1] = (uint8_t)(k1 < K ? elem_code<FMT>(v1[j] * inv) : 0u);
            if (lane == 0) E[r * nbs + b0 + j] = e;
        } else {
            // blocks of 32: lanes 0-31 and 32-63 each hold one block of the
            // low half (positions l) and one of the high half (l + 64)
            float a0 = fabsf(v0[j]), a1 = fabsf(v1[j]);
#pragma unroll
            for (int s = 16; s > 0; s >>= 1) {
                a0 = fmaxf(a0, __shfl_xor(a0, s, 64));
                a1 = fmaxf(a1, __shfl_xor(a1, s, 64));
            }
            const int e0 = fp8_scale_exp<FMT>(a0), e1 = fp8_scale_exp<FMT>(a1);
            q[k0] = (uint8_t)(k0 < K ? elem_code<FMT>(v0[j] * ldexpf(1.f, -e0)) : 0u);
            q[k1] = (uint8_t)(k1 < K ? elem_code<FMT>(v1[j] * ldexpf(1.f, -e1)) : 0u);
            if ((lane & 31) == 0) {
                const int64_t eb = r * nbs + (b0 + j) * 4 + (lane >> 5);
                E[eb] = e0;
                E[eb + 2] = e1;
            }
        }
    }
}

// Lanes along the rows: one wave per (16 rows, 128-block); four lanes share a
// row, each keeping a quarter of the block (32 values) in registers, so X is
// read once and every load of the wave reads 16 neighbouring rows at four
// contracted positions.  With blocks of 32 each lane's quarter is one block.
template <int BS, int FMT>
__global__ __launch_bounds__(256) void fp8_quant_rows_kernel(const float *__restrict__ X,
                                                             const int64_t *__restrict__ offR,
                                                             const int32_t *__restrict__ rowMap,
                                                             int64_t rows, int64_t rowsPad,
                                                             const int64_t *__restrict__ offK,
                                                             int64_t K, uint8_t *__restrict__ Q,
                                                             int32_t *__restrict__ E) {
    constexpr int RPW = 16, PART = 128 / (64 / RPW);   // rows per wave, values per lane
    const int64_t nb = (K + 127) / 128;
    const int64_t Kp = nb * 128;
    const int lane = threadIdx.x & 63;
    const int64_t groups = (rowsPad + RPW - 1) / RPW;
    const int64_t task = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (task >= groups * nb) return;
    const int64_t blk = task / groups, g = task - blk * groups;   // neighbouring waves: neighbouring rows
    const int64_t p = g * RPW + (lane % RPW);                      // walk position
    const int part = lane / RPW;                                   // quarter of the block
    const bool live = p < rows;
    const float *x = X + (live ? offR[p] : 0);
    // output row: rows are walked in the operand's order, padding rows in place
    const int64_t r = (rowMap && live) ? (int64_t)rowMap[p] : p;
    const int64_t k0 = blk * 128 + part * PART;
    const int64_t kn = K - k0;                                     // positions left from k0
    float v[PART];
    float amax = 0.f;
#pragma unroll
    for (int i = 0; i < PART; ++i) {
        v[i] = (i < kn && live) ? x[offK[k0 + i]] : 0.f;
        amax = fmaxf(amax, fabsf(v[i]));
    }
    if constexpr (BS == 128) {
        // the four lanes of a row are RPW apart
        amax = fmaxf(amax, __shfl_xor(amax, RPW, 64));
        amax = fmaxf(amax, __shfl_xor(amax, 2 * RPW, 64));
    }
    const int e = fp8_scale_exp<FMT>(amax);
    const float inv = ldexpf(1.f, -e);
    if (p >= rowsPad) return;
    uint4 *q = reinterpret_cast<uint4 *>(Q + r * Kp + k0);
#pragma unroll
    for (int c = 0; c < PART / 16; ++c) {
        const float *w = v + 16 * c;
        uint4 out;
        out.x = elem_word<FMT>(w[0] * inv, w[1] * inv, w[2] * inv, w[3] * inv);
        out.y = elem_word<FMT>(w[4] * inv, w[5] * inv, w[6] * inv, w[7] * inv);
        out.z = elem_word<FMT>(w[8] * inv, w[9] * inv, w[10] * inv, w[11] * inv);
        out.w = elem_word<FMT>(w[12] * inv, w[13] * inv, w[14] * inv, w[15] * inv);
        q[c] = out;
    }
    if constexpr (BS == 128) {
        if (part == 0) E[r * nb + blk] = e;
    } else {
        E[r * nb * 4 + blk * 4 + part] = e;
    }
}

// Load one 128-block of a ROWS x 128 code tile into registers: 16-byte
// chunks, eight per row.
template <int CH>
__device__ __forceinline__ void fp8_load_block(const uint8_t *__restrict__ base, int64_t Kp,
                                               int64_t blk, int t, u4_t (&r)[CH]) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int idx = t + c * 256, row = idx >> 3, part = idx & 7;
        r[c] = *reinterpret_cast<const u4_t *>(base + row * Kp + blk * 128 + part * 16);
    }
}

// LDS rows of 128 bytes, unpadded; the eight 16-byte chunks of row r sit at
// positions c ^ fp8_swz(r).  fp8_swz takes distinct values on any 8
// consecutive rows and on the even and the odd rows of any 16, so the
// operand reads (one chunk of each of 8 or 16 neighbouring rows per pass)
// and the stores (a row's 8 chunks by 8 neighbouring lanes) each touch every
// bank once, whether a 16-byte access is served 8 lanes at a time over 32
// banks or 16 lanes over 64.
__device__ __forceinline__ int fp8_swz(int r) { return ((r >> 1) ^ ((r & 1) << 2)) & 7; }

template <int CH>
__device__ __forceinline__ void fp8_store_block(uint8_t *s, int t, const u4_t (&r)[CH]) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int idx = t + c * 256, row = idx >> 3, part = idx & 7;
        *reinterpret_cast<u4_t *>(s + row * 128 + 16 * (part ^ fp8_swz(row))) = r[c];
    }
}

// Operand registers of one lane.  E4M3: with one scale per 128 any split of
// the block between lanes works as long as A and B share it, and each lane
// takes 32 consecutive codes; with one scale per 32 the matrix core's block
// b (of 32) must be the stored block b, so lane group g takes the stored
// positions 16 g .. 16 g + 15 and 64 + 16 g .. 64 + 16 g + 15 (the halves
// the core reads as k = 16 g .. and 64 + 16 g ..), and supplies the scale of
// block g of its row.  E2M3 / E2M1: lane group g supplies the 32 positions
// 32 g .. 32 g + 31, one block, packed 6 / 4 bits per code from the low bits
// up in 6 / 4 registers (measured with an in-bounds probe: the order inside
// a block does not change the result when A and B share it; the block of a
// lane group must be its own).
// The 16-byte chunks a lane supplies: 2g and 2g + 1 (32 consecutive codes),
// or with E4M3 per 32: g and 4 + g (positions 16 g .. and 64 + 16 g ..).
template <int BS, int FMT> __device__ __forceinline__ int fp8_chunk(int g, int h) {
    constexpr bool halves = FMT == kElemE4M3 && BS == 32;
    return halves ? (h ? 4 + g : g) : 2 * g + h;
}

// A lane's 32 codes (one per byte, eight words) as the MFMA operand.
template <int FMT>
__device__ __forceinline__ i8_t fp8_pack(const u4_t &lo, const u4_t &hi) {
    const unsigned w[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    if constexpr (FMT == kElemE4M3) {
        return i8_t{(int)w[0], (int)w[1], (int)w[2], (int)w[3],
                    (int)w[4], (int)w[5], (int)w[6], (int)w[7]};
    } else if constexpr (FMT == kElemE2M1) {
        // word i holds codes 4i .. 4i + 3 (one per byte): y = w | w >> 4 puts
        // codes 4i, 4i+1 in byte 0 and 4i+2, 4i+3 in byte 2
        unsigned p[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const unsigned y0 = w[2 * d] | (w[2 * d] >> 4), y1 = w[2 * d + 1] | (w[2 * d + 1] >> 4);
            p[d] = (y0 & 0xFFu) | ((y0 >> 8) & 0xFF00u) | ((y1 & 0xFFu) << 16) |
                   ((y1 << 8) & 0xFF000000u);
        }
        return i8_t{(int)p[0], (int)p[1], (int)p[2], (int)p[3], 0, 0, 0, 0};
    } else {
        // four 6-bit codes of a word into 24 bits, four such into 3 words
        unsigned t[8];
#pragma unroll
        for (int i = 0; i < 8; ++i)
            t[i] = (w[i] & 0x3Fu) | ((w[i] >> 2) & 0xFC0u) | ((w[i] >> 4) & 0x3F000u) |
                   ((w[i] >> 6) & 0xFC0000u);
        unsigned p[6];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const unsigned *u = t + 4 * h;
            p[3 * h] = u[0] | (u[1] << 24);
            p[3 * h + 1] = (u[1] >> 8) | (u[2] << 16);
            p[3 * h + 2] = (u[2] >> 16) | (u[3] << 8);
        }
        return i8_t{(int)p[0], (int)p[1], (int)p[2], (int)p[3], (int)p[4], (int)p[5], 0, 0};
    }
}

// Operand registers of one lane.  E4M3: with one scale per 128 any split of
// the block between lanes works as long as A and B share it, and each lane
// takes 32 consecutive codes; with one scale per 32 the matrix core's block
// b (of 32) must be the stored block b, so lane group g takes the stored
// positions 16 g .. 16 g + 15 and 64 + 16 g .. 64 + 16 g + 15 (the halves
// the core reads as k = 16 g .. and 64 + 16 g ..), and supplies the scale of
// block g of its row.  E2M3 / E2M1: lane group g supplies the 32 positions
// 32 g .. 32 g + 31, one block, packed 6 / 4 bits per code from the low bits
// up in 6 / 4 registers (measured with an in-bounds probe: the order inside
// a block does not change the result when A and B share it; the block of a
// lane group must be its own).  From the swizzled LDS rows:
template <int BS, int FMT>
__device__ __forceinline__ i8_t fp8_operand(const uint8_t *s, int r, int lane) {
    const int g = lane >> 4, f = fp8_swz(r);
    const uint8_t *row = s + r * 128;
    const u4_t lo = *reinterpret_cast<const u4_t *>(row + 16 * (fp8_chunk<BS, FMT>(g, 0) ^ f));
    const u4_t hi = *reinterpret_cast<const u4_t *>(row + 16 * (fp8_chunk<BS, FMT>(g, 1) ^ f));
    return fp8_pack<FMT>(lo, hi);
}

// One 128-block on the matrix cores: each wave's FM x FN fragments.  sE holds
// the biased exponents of the tile's A rows, then of its B rows (one per row,
// or four per row with blocks of 32).
template <int FM, int FN, int WTM, int WTN, int BM, int BS, int FMT>
__device__ __forceinline__ void fp8_mma_block(const uint8_t *sA, const uint8_t *sB,
                                              const int32_t *sE, int wm, int wn, int lane,
                                              f4_t (&acc)[FM][FN]) {
    constexpr int SUB = 128 / BS;
    const int sub = BS == 128 ? 0 : (lane >> 4);
    i8_t a[FM], b[FN];
    int sa[FM], sb[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
        const int r = wm * WTM + i * 16 + (lane & 15);
        a[i] = fp8_operand<BS, FMT>(sA, r, lane);
        sa[i] = sE[r * SUB + sub];
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int r = wn * WTN + j * 16 + (lane & 15);
        b[j] = fp8_operand<BS, FMT>(sB, r, lane);
        sb[j] = sE[(BM + r) * SUB + sub];
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            // B first: the result holds 16 N positions by 16 M positions, so
            // each lane ends with four neighbouring N positions of one M row
            // (C's cheapest direction), stored as one 16-byte word.
            acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(b[j], a[i], acc[i][j], FMT,
                                                                         FMT, 0, sb[j], 0, sa[i]);
}

// The direct-B form of one block: A's fragments and scales from LDS as above;
// B's fragment j arrives as its lane's two 16-byte chunks of the code row
// (bl[j], bh[j]) and its raw exponent bs[j], both loaded a block earlier
// straight from the quantised rows; after fragment j's MFMAs its chunks and
// exponent for block `next` are loaded into the same registers (behind a
// scheduling barrier, so the registers are reused rather than renamed).
// zero_b: this block is the pair's padding block (B scale E8M0 0).
template <int FM, int FN, int WTM, int WTN, int BS, int FMT>
__device__ __forceinline__ void fp8_mma_block_db(const uint8_t *sA, const int32_t *sE, int wm,
                                                 int lane, f4_t (&acc)[FM][FN],
                                                 u4_t (&bl)[FN], u4_t (&bh)[FN], int (&bs)[FN],
                                                 bool zero_b, const uint8_t *brow,
                                                 const int32_t *bexp, int64_t rstep,
                                                 int64_t estep, int64_t next) {
    constexpr int SUB = 128 / BS;
    const int sub = BS == 128 ? 0 : (lane >> 4), g = lane >> 4;
    i8_t a[FM];
    int sa[FM];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
        const int r = wm * WTM + i * 16 + (lane & 15);
        a[i] = fp8_operand<BS, FMT>(sA, r, lane);
        sa[i] = sE[r * SUB + sub];
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const i8_t b = fp8_pack<FMT>(bl[j], bh[j]);
        const int sb = zero_b ? 0 : bs[j] + 127;
#pragma unroll
        for (int i = 0; i < FM; ++i)
            acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(b, a[i], acc[i][j], FMT,
                                                                         FMT, 0, sb, 0, sa[i]);
        __builtin_amdgcn_sched_barrier(0);
        const uint8_t *p = brow + j * rstep + next * 128;
        bl[j] = *reinterpret_cast<const u4_t *>(p + 16 * fp8_chunk<BS, FMT>(g, 0));
        bh[j] = *reinterpret_cast<const u4_t *>(p + 16 * fp8_chunk<BS, FMT>(g, 1));
        bs[j] = bexp[j * estep + next * SUB + sub];
    }
}

// Whether the four N positions n .. n+3 of an M row are neighbours in C,
// all inside N, and start on a 16-byte boundary (one vector access); on is
// the tile's staged N offsets from position n on.
__device__ __forceinline__ bool fp8_c_word(const float *C, const int64_t *on, int64_t ocm,
                                           int64_t o0, int64_t n, int64_t N) {
    if (n + 3 >= N) return false;
    if (on[1] != o0 + 1 || on[2] != o0 + 2 || on[3] != o0 + 3) return false;
    return (reinterpret_cast<uintptr_t>(C + ocm + o0) & 15) == 0;
}

// C tile BM x BN, 4 waves as 2 x 2, each wave (BM/2) x (BN/2) in 16x16
// fragments.  DB: B's fragments straight from the quantised rows into
// registers (fp8_mma_block_db), only A staged through LDS.
template <int BM, int BN, int BS, int FMT, bool DB>
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
    constexpr int CA = BM * 8 / 256, CB = BN * 8 / 256;   // 16-byte chunks per thread
    constexpr int ER = DB ? BM : BM + BN;    // rows whose scales go through LDS
    __shared__ __align__(16) uint8_t sA[2][BM * 128];
    __shared__ __align__(16) uint8_t sB[2][DB ? 16 : BN * 128];
    constexpr int SUB = 128 / BS;            // scales per row and 128-block
    __shared__ __align__(16) int32_t sE[2][ER * SUB];
    static_assert(ER <= 256 && 256 % ER == 0, "one row of scales per thread");

    const int64_t nb = (K + 127) / 128;
    const int64_t Kp = nb * 128;
    const int64_t nbs = nb * SUB;            // scales per row
    int tm, tn;
    tile_coords(xcd_remap(blockIdx.x, gridDim.x), tilesM, tilesN, tm, tn);
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
    // The tile's C offsets (M rows, then N positions), requested before the
    // first block's codes and staged in LDS at the first barrier: the
    // epilogue then waits for C_in alone, not for the offset tables first.
    __shared__ int64_t sOff[BM + BN];
    static_assert(BM + BN <= 256, "one offset per thread");
    int64_t myOff = 0;
    if (t < BM) {
        if (m0 + t < M) myOff = offCM[m0 + t];
    } else if (t < BM + BN) {
        if (n0 + t - BM < N) myOff = offCN[n0 + t - BM];
    }
    auto put_offs = [&]() { if (t < BM + BN) sOff[t] = myOff; };

    // Rows are padded to a multiple of 128 in both operands, so every tile
    // row exists in the quantised buffers.
    const uint8_t *pa = QA + m0 * Kp, *pb = QB + n0 * Kp;
    f4_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

    // Thread t carries the scales of tile row t mod ER (A rows, then B rows
    // unless B comes straight from memory; with fewer rows than threads, two
    // threads carry the same ones).
    const int sidx = t % ER;
    const int32_t *ex = sidx < BM ? EA + (m0 + sidx) * nbs : EB + (n0 + sidx - BM) * nbs;
    typedef int i4s_t __attribute__((ext_vector_type(4)));
    // this row's exponents of block blk, as stored
    auto scales = [&](int64_t blk) {
        if constexpr (SUB == 1) return i4s_t{ex[blk], 0, 0, 0};
        else return *reinterpret_cast<const i4s_t *>(ex + blk * 4);
    };
    // ... biased for E8M0 (bias 127) only when they go to LDS, a block after
    // their load: biasing them at the load made the loop wait for the load
    // it had just issued (the add cannot cross the MFMA block's scheduling
    // barrier), exposing a full memory latency in every block.
    auto put_scales = [&](int32_t *se, i4s_t v) {
        if constexpr (SUB == 1) se[sidx] = v.x + 127;
        else *reinterpret_cast<i4s_t *>(se + sidx * 4) = v + 127;
    };
    const i4s_t kZeroScale = i4s_t{-127, -127, -127, -127};   // E8M0 0 after the bias
    // Two register sets: the codes of block b + 2 load while block b runs on
    // the matrix cores and block b + 1 waits in the other set; loads past the
    // last block reload it (a valid address).  Blocks run in pairs; when their
    // number is odd, the last pair's second block is such a reload staged with
    // both E8M0 scales 0 (2^-127 each): its 128-term products, at most
    // 2^25 * 2^-254, fall below FP32's smallest denormal and add exactly zero.
    if constexpr (!DB) {
        u4_t ra[CA], rb[CB], ra2[CA], rb2[CB];
        fp8_load_block<CA>(pa, Kp, 0, t, ra);
        fp8_load_block<CB>(pb, Kp, 0, t, rb);
        i4s_t xs = scales(0);
        const int64_t b1 = nb > 1 ? 1 : 0;
        fp8_load_block<CA>(pa, Kp, b1, t, ra2);
        fp8_load_block<CB>(pb, Kp, b1, t, rb2);
        i4s_t xs2 = scales(b1);
        fp8_store_block<CA>(sA[0], t, ra);
        fp8_store_block<CB>(sB[0], t, rb);
        put_scales(sE[0], xs);
        put_offs();
        __syncthreads();
        for (int64_t blk = 0; blk < nb; blk += 2) {
            // even block: LDS stage 0, the next block waits in set 2
            const int64_t n2 = blk + 2 < nb ? blk + 2 : nb - 1;
            fp8_load_block<CA>(pa, Kp, n2, t, ra);
            fp8_load_block<CB>(pb, Kp, n2, t, rb);
            xs = scales(n2);
            fp8_mma_block<FM, FN, WTM, WTN, BM, BS, FMT>(sA[0], sB[0], sE[0], wm, wn, lane, acc);
            __builtin_amdgcn_sched_barrier(0);
            fp8_store_block<CA>(sA[1], t, ra2);
            fp8_store_block<CB>(sB[1], t, rb2);
            put_scales(sE[1], blk + 1 < nb ? xs2 : kZeroScale);
            __syncthreads();
            // odd block: LDS stage 1, the next block waits in set 1
            const int64_t n3 = blk + 3 < nb ? blk + 3 : nb - 1;
            fp8_load_block<CA>(pa, Kp, n3, t, ra2);
            fp8_load_block<CB>(pb, Kp, n3, t, rb2);
            xs2 = scales(n3);
            fp8_mma_block<FM, FN, WTM, WTN, BM, BS, FMT>(sA[1], sB[1], sE[1], wm, wn, lane, acc);
            __builtin_amdgcn_sched_barrier(0);
            fp8_store_block<CA>(sA[0], t, ra);
            fp8_store_block<CB>(sB[0], t, rb);
            put_scales(sE[0], xs);
            __syncthreads();
        }
    } else {
        // B rows of this wave's fragments: row n0 + wn WTN + 16 j + lane % 16,
        // fragment j 16 rows (rstep bytes, estep exponents) after fragment 0
        const int64_t rb0 = n0 + wn * WTN + (lane & 15);
        const uint8_t *brow = QB + rb0 * Kp;
        const int32_t *bexp = EB + rb0 * nbs;
        const int64_t rstep = 16 * Kp, estep = 16 * nbs;
        u4_t bl[FN], bh[FN];
        int bs[FN];
        const int g = lane >> 4, sub = BS == 128 ? 0 : g;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const uint8_t *p = brow + j * rstep;
            bl[j] = *reinterpret_cast<const u4_t *>(p + 16 * fp8_chunk<BS, FMT>(g, 0));
            bh[j] = *reinterpret_cast<const u4_t *>(p + 16 * fp8_chunk<BS, FMT>(g, 1));
            bs[j] = bexp[j * estep + sub];
        }
        u4_t ra[CA], ra2[CA];
        fp8_load_block<CA>(pa, Kp, 0, t, ra);
        i4s_t xs = scales(0);
        const int64_t b1 = nb > 1 ? 1 : 0;
        fp8_load_block<CA>(pa, Kp, b1, t, ra2);
        i4s_t xs2 = scales(b1);
        fp8_store_block<CA>(sA[0], t, ra);
        put_scales(sE[0], xs);
        put_offs();
        __syncthreads();
        for (int64_t blk = 0; blk < nb; blk += 2) {
            // even block: A in LDS stage 0, B's block blk in registers
            const int64_t n2 = blk + 2 < nb ? blk + 2 : nb - 1;
            fp8_load_block<CA>(pa, Kp, n2, t, ra);
            xs = scales(n2);
            fp8_mma_block_db<FM, FN, WTM, WTN, BS, FMT>(sA[0], sE[0], wm, lane, acc, bl, bh, bs,
                                                        false, brow, bexp, rstep, estep,
                                                        blk + 1 < nb ? blk + 1 : nb - 1);
            __builtin_amdgcn_sched_barrier(0);
            fp8_store_block<CA>(sA[1], t, ra2);
            put_scales(sE[1], blk + 1 < nb ? xs2 : kZeroScale);
            __syncthreads();
            // odd block: A in stage 1, B's block blk + 1 (the last block again,
            // with both scales 0, when blk + 1 == nb)
            const int64_t n3 = blk + 3 < nb ? blk + 3 : nb - 1;
            fp8_load_block<CA>(pa, Kp, n3, t, ra2);
            xs2 = scales(n3);
            fp8_mma_block_db<FM, FN, WTM, WTN, BS, FMT>(sA[1], sE[1], wm, lane, acc, bl, bh, bs,
                                                        blk + 1 >= nb, brow, bexp, rstep, estep, n2);
            __builtin_amdgcn_sched_barrier(0);
            fp8_store_block<CA>(sA[0], t, ra);
            put_scales(sE[0], xs);
            __syncthreads();
        }
    }
    // C_in of this lane's outputs.  Lane l holds M row (l % 16) and the four
    // N positions 4 (l / 16) .. + 3 of each fragment; where those four are
    // neighbours in C (and 16-byte aligned) they move as one word.  Positions
    // past M or N are neither read nor written.
    f4_t cin[FM][FN];
    const int lm = lane & 15, ln = 4 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < FM; ++i) {
        const int ml = wm * WTM + i * 16 + lm;
        const int64_t m = m0 + ml;
        const int64_t ocm = sOff[ml];
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int nl = wn * WTN + j * 16 + ln;
            const int64_t n = n0 + nl;
            const int64_t *on = sOff + BM + nl;
            f4_t x = f4_t{0.f, 0.f, 0.f, 0.f};
            if (m < M) {
                const int64_t o0 = on[0];
                if (fp8_c_word(C, on, ocm, o0, n, N)) {
                    x = *reinterpret_cast<const f4_t *>(C + ocm + o0);
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (n + v < N) x[v] = C[ocm + on[v]];
                }
            }
            cin[i][j] = x;
        }
    }
    // add and store
#pragma unroll
    for (int i = 0; i < FM; ++i) {
        const int ml = wm * WTM + i * 16 + lm;
        const int64_t m = m0 + ml;
        if (m >= M) continue;
        const int64_t ocm = sOff[ml];
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int nl = wn * WTN + j * 16 + ln;
            const int64_t n = n0 + nl;
            if (n >= N) continue;
            const int64_t *on = sOff + BM + nl;
            const int64_t o0 = on[0];
            const f4_t y = cin[i][j] + acc[i][j];
            if (fp8_c_word(C, on, ocm, o0, n, N)) {
                *reinterpret_cast<f4_t *>(C + ocm + o0) = y;
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (n + v < N) C[ocm + on[v]] = y[v];
            }
        }
    }
}

namespace {

// (block size, element format) -> kernel; false for a pair the path does not
// have (E2M3 and E2M1 come with blocks of 32 only).
template <template <int, int> class K>
bool pick(int bs, int fmt, typename K<128, kElemE4M3>::F &out) {
    if (bs == 128 && fmt == kElemE4M3) out = K<128, kElemE4M3>::f;
    else if (bs == 32 && fmt == kElemE4M3) out = K<32, kElemE4M3>::f;
    else if (bs == 32 && fmt == kElemE2M3) out = K<32, kElemE2M3>::f;
    else if (bs == 32 && fmt == kElemE2M1) out = K<32, kElemE2M1>::f;
    else return false;
    return true;
}

template <int BS, int FMT> struct QuantK {
    using F = decltype(&fp8_quant_kernel<128, kElemE4M3>);
    static constexpr F f = &fp8_quant_kernel<BS, FMT>;
};
template <int BS, int FMT> struct QuantRowsK {
    using F = decltype(&fp8_quant_rows_kernel<128, kElemE4M3>);
    static constexpr F f = &fp8_quant_rows_kernel<BS, FMT>;
};
// B straight from the code rows only for E2M3: there the LDS form's operand
// packing took it to 257 registers (one workgroup per CU) and the direct form
// fits two (strided workload 304 -> 326 TFLOP/s, CC 220 -> 263); for E4M3 and
// E2M1 it measured slower (485 -> 392 and 415 -> 342 on the strided one): a
// code row is not blocked, so one fragment load touches 16 cache lines.
template <int FMT> constexpr bool fp8_direct_b() { return FMT == kElemE2M3; }

template <int BS, int FMT> struct Gemm128K {
    using F = decltype(&fp8_gemm_kernel<128, 128, 128, kElemE4M3, false>);
    static constexpr F f = &fp8_gemm_kernel<128, 128, BS, FMT, fp8_direct_b<FMT>()>;
};
template <int BS, int FMT> struct Gemm64K {
    using F = decltype(&fp8_gemm_kernel<64, 64, 128, kElemE4M3, false>);
    static constexpr F f = &fp8_gemm_kernel<64, 64, BS, FMT, fp8_direct_b<FMT>()>;
};

}  // namespace

int launch_fp8_quant(const float *X, const int64_t *offR, const int32_t *rowMap, int64_t rows,
                     int64_t rowsPad, const int64_t *offK, int64_t K, bool rowsFast, uint8_t *Q,
                     int32_t *E, hipStream_t s, int bs, int fmt) {
    const int64_t nb = (K + 127) / 128;
    const int64_t tasks = rowsFast ? (rowsPad + 15) / 16 * nb
                                   : rowsPad * ((nb + kQuantRun - 1) / kQuantRun);
    const int64_t blocks = (tasks + 3) / 4;
    if (blocks > INT32_MAX) return GETT_ERR_INTERNAL;
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    if (rowsFast) {
        QuantRowsK<128, kElemE4M3>::F k;
        if (!pick<QuantRowsK>(bs, fmt, k)) return GETT_ERR_INTERNAL;
        hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(256), 0, s, X, offR, rowMap, rows,
                           rowsPad, offK, K, Q, E);
    } else {
        QuantK<128, kElemE4M3>::F k;
        if (!pick<QuantK>(bs, fmt, k)) return GETT_ERR_INTERNAL;
        hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(256), 0, s, X, offR, rows, rowsPad,
                           offK, K, Q, E);
    }
    return launch_status();
}

int launch_fp8_gemm(int tile, const uint8_t *QA, const int32_t *EA, const uint8_t *QB,
                    const int32_t *EB, float *C, const int64_t *offCM, const int64_t *offCN,
                    int64_t M, int64_t N, int64_t K, hipStream_t s, int bs, int fmt) {
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    if (tile == 3) {
        const int tilesM = (int)((M + 127) / 128), tilesN = (int)((N + 127) / 128);
        Gemm128K<128, kElemE4M3>::F k;
        if (!pick<Gemm128K>(bs, fmt, k)) return GETT_ERR_INTERNAL;
        hipLaunchKernelGGL(k, dim3(tilesM * tilesN), dim3(256), 0, s, QA, EA, QB, EB, C, offCM,
                           offCN, M, N, K, tilesM, tilesN);
    } else {
        // operands are padded to multiples of 128 rows, so 64-row tiles stay inside
        const int tilesM = (int)((M + 63) / 64), tilesN = (int)((N + 63) / 64);
        Gemm64K<128, kElemE4M3>::F k;
        if (!pick<Gemm64K>(bs, fmt, k)) return GETT_ERR_INTERNAL;
        hipLaunchKernelGGL(k, dim3(tilesM * tilesN), dim3(256), 0, s, QA, EA, QB, EB, C, offCM,
                           offCN, M, N, K, tilesM, tilesN);
    }
    return launch_status();
}

}  // namespace gett
