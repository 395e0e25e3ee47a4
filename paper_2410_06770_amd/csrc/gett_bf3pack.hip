// gett_bf3pack.hip -- the packed form of the BF16x3 path of SGETT.
//
// The direct BF16x3 tiles split every FP32 value into bfloat16 hi and lo
// each time a tile loads it, so an element of A is split once per tile
// column of C (and one of B once per tile row), and the split, with the
// gather's address arithmetic, leaves the vector ALU with several times the
// matrix-core instruction count.  The packed form splits each element once:
//
// pack:  every row of an operand (a free position, in the order of the
//        schedule's offset tables) becomes two dense bfloat16 rows, hi and
//        lo, of Kq = K rounded up to 32 positions (zeros past K), in two
//        planes.  A plane is stored in blocks of 16 rows by one step of 32
//        positions (1 KB, rows of 64 bytes inside), row groups outermost and
//        steps next, so that a step of a tile's rows is whole cache lines
//        (64-byte row pieces 2 KB or more apart would each fetch a 128-byte
//        line of which the next step needs the other half, after it has left
//        the L1).  The contracted positions are stored in a fixed
//        permutation shared by both operands (the sum is over the same
//        pairs): groups of 512 positions, group g holding S = min(512,
//        Kq - 512 g) / 8 chunks of 8, and chunk c of a group holds the
//        positions 512 g + c + S e, e = 0 .. 7.  So a wave whose lanes run
//        along K reads 64 neighbouring positions per load and still writes
//        one 16-byte chunk per lane and plane, and a wave whose lanes run
//        along the rows reads 16 neighbouring rows per load (its rows are
//        walked in the operand's memory order and written to their table
//        position).
// gemm:  a 128 x 128 tile (4 waves as 2 x 2) walks the packed rows in steps
//        of 32 positions with 16-byte loads only (no offset tables, no
//        conversion), stages them through LDS, and forms hi*hi + hi*lo +
//        lo*hi on the BF16 MFMA with one FP32 accumulator per output, as the
//        direct tiles do; the epilogue is theirs too (offset tables of C,
//        alpha and beta in FP64, one rounding; or FP64 partials of a K slice).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gett_bf3pack.h"
#include "gett_grid.h"
#include "gett_internal.h"

namespace gett {

namespace {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u4_t __attribute__((ext_vector_type(4)));

// hi = bf16(x) (round to nearest even), lo = bf16(x - hi) (the subtraction
// is exact) for two values, packed with the first in the low half.
__device__ __forceinline__ void split_pair(float x0, float x1, uint32_t &hi, uint32_t &lo) {
    typedef float f2_t __attribute__((ext_vector_type(2)));
    typedef __bf16 b2_t __attribute__((ext_vector_type(2)));
    hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2_t{x0, x1}, b2_t));
    const float h0 = __uint_as_float(hi << 16), h1 = __uint_as_float(hi & 0xffff0000u);
    lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2_t{x0 - h0, x1 - h1}, b2_t));
}

__device__ __forceinline__ void split8(const float (&v)[8], u4_t &hi, u4_t &lo) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) split_pair(v[2 * i], v[2 * i + 1], h[i], l[i]);
    hi = u4_t{h[0], h[1], h[2], h[3]};
    lo = u4_t{l[0], l[1], l[2], l[3]};
}

// Contracted position of element e of packed chunk c (see the file comment).
__device__ __forceinline__ int64_t chunk_pos(int64_t c, int e, int64_t Kq) {
    const int64_t g = c >> 6;
    const int64_t S = min<int64_t>(512, Kq - 512 * g) >> 3;
    return 512 * g + (c & 63) + S * e;
}

// Element offset of packed positions j .. j + 7 (j a multiple of 8) of row
// r in a plane of Kq positions per row (see the file comment).
__device__ __forceinline__ int64_t pk_off(int64_t r, int64_t j, int64_t Kq) {
    return ((r >> 4) * (Kq >> 5) + (j >> 5)) * 512 + (r & 15) * 32 + (j & 31);
}

// FP64 planes (the packed FP64 form): blocks of 16 rows by 16 positions
// (2 KB, rows of 128 bytes), row groups outermost; element offset of packed
// positions j .. j + 7 (j a multiple of 8) of row r.
__device__ __forceinline__ int64_t pk64_off(int64_t r, int64_t j, int64_t Kq) {
    return ((r >> 4) * (Kq >> 4) + (j >> 4)) * 256 + (r & 15) * 16 + (j & 15);
}

// Where a pass puts one chunk (8 packed positions of one row): BF16x3 splits
// the values into the hi and lo planes, FP64 copies them.
template <bool F64> struct PackOut;
template <> struct PackOut<false> {
    using T = float;
    static __device__ __forceinline__ void put(void *P, int64_t plane, int64_t r, int64_t c,
                                               int64_t Kq, const float (&v)[8]) {
        u4_t hi, lo;
        split8(v, hi, lo);
        uint16_t *dst = static_cast<uint16_t *>(P) + pk_off(r, 8 * c, Kq);
        *reinterpret_cast<u4_t *>(dst) = hi;
        *reinterpret_cast<u4_t *>(dst + plane) = lo;
    }
};
template <> struct PackOut<true> {
    using T = double;
    static __device__ __forceinline__ void put(void *P, int64_t, int64_t r, int64_t c, int64_t Kq,
                                               const double (&v)[8]) {
        typedef double d2v_t __attribute__((ext_vector_type(2)));
        d2v_t *dst = reinterpret_cast<d2v_t *>(static_cast<double *>(P) + pk64_off(r, 8 * c, Kq));
#pragma unroll
        for (int i = 0; i < 4; ++i) dst[i] = d2v_t{v[2 * i], v[2 * i + 1]};
    }
};

constexpr int kPackRowsK = 4;      // rows per wave, lanes along K
constexpr int kPackBlocksR = 4;    // 16-row blocks per wave, lanes along the rows

// Lanes along K: one wave per (kPackRowsK rows, group of 512 packed
// positions); lane l fills chunk l of the group in each row, its contracted
// offsets read once for all of them.
template <bool F64>
__global__ __launch_bounds__(256) void pack_k_kernel(const typename PackOut<F64>::T *__restrict__ X,
                                                     const int64_t *__restrict__ offR, int64_t R,
                                                     const int64_t *__restrict__ offK, int64_t K,
                                                     int64_t Kq, void *__restrict__ P,
                                                     int64_t plane) {
    using T = typename PackOut<F64>::T;
    const int64_t ng = (Kq + 511) / 512;
    const int64_t nrb = (R + kPackRowsK - 1) / kPackRowsK;
    const int64_t task = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (task >= nrb * ng) return;
    const int lane = threadIdx.x & 63;
    const int64_t rb = task / ng, g = task - rb * ng;
    const int64_t S = min<int64_t>(512, Kq - 512 * g) >> 3;
    if (lane >= S) return;
    const int64_t c = 64 * g + lane;
    int64_t ko[8];
    uint32_t valid = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t k = chunk_pos(c, e, Kq);
        ko[e] = k < K ? offK[k] : 0;
        valid |= (k < K ? 1u : 0u) << e;
    }
#pragma unroll
    for (int q = 0; q < kPackRowsK; ++q) {
        const int64_t r = rb * kPackRowsK + q;
        if (r >= R) break;
        const T *xr = X + offR[r];
        T v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (valid >> e) & 1 ? xr[ko[e]] : T(0);
        PackOut<F64>::put(P, plane, r, c, Kq, v);
    }
}

// Lanes along the rows: one wave per (kPackBlocksR blocks of 16 rows in the
// operand's memory order, 4 chunks); lane l takes row l % 16 of each block
// and chunk c0 + l / 16, so each load reads 16 neighbouring rows, each row's
// four chunks are stored together, and the contracted offsets are read once
// for all the blocks.
template <bool F64>
__global__ __launch_bounds__(256) void pack_rows_kernel(
    const typename PackOut<F64>::T *__restrict__ X, const int64_t *__restrict__ rowsOp,
    const int32_t *__restrict__ rowMap, int64_t R, const int64_t *__restrict__ offK, int64_t K,
    int64_t Kq, void *__restrict__ P, int64_t plane) {
    using T = typename PackOut<F64>::T;
    const int64_t nc = Kq / 8;
    const int64_t cq = (nc + 3) / 4;
    const int64_t task = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t sb = task / cq, q = task - sb * cq;
    const int64_t c = q * 4 + (lane >> 4);
    if (sb * 16 * kPackBlocksR >= R || c >= nc) return;
    int64_t ko[8];
    uint32_t valid = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t k = chunk_pos(c, e, Kq);
        ko[e] = k < K ? offK[k] : 0;
        valid |= (k < K ? 1u : 0u) << e;
    }
#pragma unroll
    for (int b = 0; b < kPackBlocksR; ++b) {
        const int64_t p = (sb * kPackBlocksR + b) * 16 + (lane & 15);
        if (p >= R) break;
        const T *xr = X + rowsOp[p];
        T v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (valid >> e) & 1 ? xr[ko[e]] : T(0);
        PackOut<F64>::put(P, plane, rowMap[p], c, Kq, v);
    }
}

// LDS rows hold the 32 positions of a step, 64 bytes, unpadded; the four
// 16-byte chunks of row r are stored in the order c ^ swz(r), which keeps
// both the stores (four lanes per row, rows in lane order) and the MFMA
// operand reads (16 rows per chunk) free of bank conflicts with 32 or 64
// four-byte banks.  swz depends on bits 1-3 of r only.
constexpr int kLd = 32;
__device__ __forceinline__ int swz(int r) { return ((((r >> 1) ^ (r >> 3)) & 1) << 1) | ((r >> 2) & 1); }

template <int BM, int BN> struct PkCfg {
    static constexpr int WTM = BM / 2, WTN = BN / 2, FM = WTM / 16, FN = WTN / 16;
    static constexpr int PA = BM * kLd, PB = BN * kLd;   // elements of one LDS plane
    static constexpr int SA = 2 * PA, SB = 2 * PB;       // one stage: hi and lo planes
    static constexpr int CA = BM * 8 / 256, CB = BN * 8 / 256;   // 16-byte chunks per thread
    static constexpr int kLdsBytes = 2 * (SA + SB) * 2;
};

// Chunk i of thread t in a ROWS-row operand tile: four neighbouring threads
// take the four 16-byte chunks of one row's 32 positions, so a wave's load
// reads one whole 1 KB block; chunk i covers row (64 i) % ROWS + t / 4 of
// plane 64 i / ROWS.  Offsets are from the tile's first block of the step.
template <int ROWS> struct PkLoad {
    static_assert(ROWS % 64 == 0, "64 rows per chunk index");
    static constexpr int C = ROWS * 8 / 256;
    uint32_t goff;      // element offset of the thread's 16 bytes inside a block
    uint32_t soff;      // element offset in an LDS stage, before the chunk's constant
    int rg0;            // row group of row t / 4
    int64_t gstride;    // elements from one row group to the next (Kq * 16)
    __device__ __forceinline__ void init(int t, int64_t Kq) {
        const int c = t & 3, r = t >> 2;
        gstride = Kq * 16;
        goff = (uint32_t)((r & 15) * 32 + 8 * c);
        soff = (uint32_t)(r * kLd + 8 * (c ^ swz(r)));
        rg0 = r >> 4;
    }
    __device__ __forceinline__ void load(const uint16_t *hi, const uint16_t *lo,
                                         u4_t (&v)[C]) const {
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const uint16_t *base = (64 * i / ROWS ? lo : hi) +
                                   (int64_t)(((64 * i) % ROWS) / 16 + rg0) * gstride;
            v[i] = *reinterpret_cast<const u4_t *>(base + goff);
        }
    }
    __device__ __forceinline__ void store(uint16_t *s, const u4_t (&v)[C]) const {
#pragma unroll
        for (int i = 0; i < C; ++i)
            *reinterpret_cast<u4_t *>(s + (64 * i / ROWS) * ROWS * kLd + ((64 * i) % ROWS) * kLd +
                                      soff) = v[i];
    }
};

template <int BM, int BN>
__device__ __forceinline__ void pk_mma(const uint16_t *sA, const uint16_t *sB, int lane, int wm,
                                       int wn, f4_t (&acc)[BM / 32][BN / 32]) {
    using Cfg = PkCfg<BM, BN>;
    constexpr int FM = Cfg::FM, FN = Cfg::FN;
    const __bf16 *ahi = reinterpret_cast<const __bf16 *>(sA);
    const __bf16 *alo = ahi + Cfg::PA;
    const __bf16 *bhi = reinterpret_cast<const __bf16 *>(sB);
    const __bf16 *blo = bhi + Cfg::PB;
    const int kc = 8 * ((lane >> 4) ^ swz(lane & 15));   // rows start at multiples of 16
    bf8_t ah[FM], al[FM];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
        const int r = wm * Cfg::WTM + i * 16 + (lane & 15);
        ah[i] = *reinterpret_cast<const bf8_t *>(ahi + r * kLd + kc);
        al[i] = *reinterpret_cast<const bf8_t *>(alo + r * kLd + kc);
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int r = wn * Cfg::WTN + j * 16 + (lane & 15);
        const bf8_t bh = *reinterpret_cast<const bf8_t *>(bhi + r * kLd + kc);
        const bf8_t bl = *reinterpret_cast<const bf8_t *>(blo + r * kLd + kc);
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc[i][j], 0, 0, 0);
        }
    }
}

// A wave's outputs: fragment (i, j), register v of lane l holds M row
// mw + 16 i + 4 (l / 16) + v and N column nw + 16 j + l % 16.  FP64 partials
// of a K slice, or C <- alpha * sum + beta * C_in in FP64 rounded once; one
// column of fragments at a time, its C_in read before any of it is written
// (a store to C could alias a later load of C, so loads interleaved with
// stores would wait out one another).
// The tile's C offsets (its M rows, then its N positions), one per thread,
// requested at kernel start and staged in LDS at the first barrier: the
// epilogue then waits for C_in alone instead of for the offset tables first.
// Split-K partials address the workspace directly and skip them.
template <int BM, int BN>
struct PkCOffs {
    int64_t v = 0;
    __device__ __forceinline__ void load(const Bf3Packed &g, int64_t m0, int64_t n0, int t) {
        if (g.ws) return;
        if (t < BM) {
            if (m0 + t < g.M) v = g.offCM[m0 + t];
        } else if (t < BM + BN) {
            if (n0 + t - BM < g.N) v = g.offCN[n0 + t - BM];
        }
    }
    __device__ __forceinline__ void put(int64_t *s, int t) const {
        if (t < BM + BN) s[t] = v;
    }
};

template <int FM, int FN>
__device__ __forceinline__ void pk_epilogue(const Bf3Packed &g, const f4_t (&acc)[FM][FN],
                                            int64_t m0, int64_t n0, int mwl, int nwl, int lane,
                                            int split, const int64_t *sOffM,
                                            const int64_t *sOffN) {
    float *__restrict__ C = g.C;
    const int64_t mw = m0 + mwl, nw = n0 + nwl;
    if (g.ws) {
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int64_t n = nw + j * 16 + (lane & 15);
            if (n >= g.N) continue;
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t m = mw + i * 16 + 4 * (lane >> 4) + v;
                    if (m < g.M) g.ws[((int64_t)split * g.M + m) * g.N + n] = (double)acc[i][j][v];
                }
        }
        return;
    }
    const bool rdC = g.beta != 0.0;
    // C_in of a group of JG fragment columns first (one round trip per
    // group), then the group's results; the offsets are read from LDS again
    // for the stores.  The 128 x 128 tile takes all its columns in one group
    // (measured +4.5 % on the CC workload, +7.5 % on the strided one); the
    // 192 x 256 tile one column at a time (two-column groups fit its
    // registers but measured 1.5 % slower on the strided workload).
    constexpr int JG = FM * FN * 4 <= 64 ? FN : 1;
    static_assert(FN % JG == 0, "whole groups");
#pragma unroll
    for (int j0 = 0; j0 < FN; j0 += JG) {
        float cin[JG][FM][4];
#pragma unroll
        for (int jj = 0; jj < JG; ++jj) {
            const int nl = nwl + (j0 + jj) * 16 + (lane & 15);
            const bool nok = n0 + nl < g.N;
            const int64_t ocn = sOffN[nl];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int ml = mwl + i * 16 + 4 * (lane >> 4) + v;
                    const bool ok = nok && m0 + ml < g.M;
                    cin[jj][i][v] = (rdC && ok) ? C[sOffM[ml] + ocn] : 0.0f;
                }
        }
#pragma unroll
        for (int jj = 0; jj < JG; ++jj) {
            const int j = j0 + jj;
            const int nl = nwl + j * 16 + (lane & 15);
            const bool nok = n0 + nl < g.N;
            const int64_t ocn = sOffN[nl];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int ml = mwl + i * 16 + 4 * (lane >> 4) + v;
                    if (!(nok && m0 + ml < g.M)) continue;
                    const double sum = (double)acc[i][j][v];
                    C[sOffM[ml] + ocn] = (float)(rdC ? g.alpha * sum + g.beta * (double)cin[jj][i][v]
                                                     : g.alpha * sum);
                }
        }
    }
}

// One BM x BN output tile over the packed range of its K slice, two LDS
// stages and one barrier per step.  128 x 128 tiles (two workgroups per CU)
// keep two register sets: step s + 2 loads while step s runs on the matrix
// cores and step s + 1 waits in the other set (loads past the last step
// repeat it).  Larger tiles (one workgroup per CU, the accumulators in the
// accumulation registers) keep one set: step s + 1 loads while step s runs,
// behind a step's worth of MFMA work.
template <int BM, int BN>
__global__ __launch_bounds__(256) void bf3_packed_gemm_kernel(Bf3Packed g) {
    using Cfg = PkCfg<BM, BN>;
    constexpr int FM = Cfg::FM, FN = Cfg::FN;
    constexpr bool kTwoSets = BM * BN <= 128 * 128;
    extern __shared__ __align__(16) uint16_t lds[];
    uint16_t *sA = lds, *sB = lds + 2 * Cfg::SA;   // [stage][plane][row][kLd]

    const int tiles = g.tilesM * g.tilesN;
    const int logical = xcd_remap(blockIdx.x, tiles * g.splits);
    const int split = logical / tiles;
    int tm, tn;
    tile_coords(logical - split * tiles, g.tilesM, g.tilesN, tm, tn);
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int64_t kbeg = (int64_t)split * g.kPer;
    const int64_t kend = min(kbeg + g.kPer, g.Kq);
    const int64_t nsteps = (kend - kbeg) / 32;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
    __shared__ int64_t sOff[BM + BN];
    static_assert(BM + BN <= 256, "one C offset per thread");
    PkCOffs<BM, BN> co;
    co.load(g, m0, n0, t);
    PkLoad<BM> la;
    PkLoad<BN> lb;
    la.init(t, g.Kq);
    lb.init(t, g.Kq);
    // first block of the tile's rows at the slice's first step; a step is 512 elements on
    const uint16_t *aH = g.A + m0 * g.Kq + kbeg * 16, *aL = aH + g.planeA;
    const uint16_t *bH = g.B + n0 * g.Kq + kbeg * 16, *bL = bH + g.planeB;

    f4_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

    auto step = [&](int64_t s) { return 512 * (s < nsteps ? s : nsteps - 1); };
    if constexpr (kTwoSets) {
        u4_t ra0[Cfg::CA], rb0[Cfg::CB], ra1[Cfg::CA], rb1[Cfg::CB];
        la.load(aH, aL, ra0);
        lb.load(bH, bL, rb0);
        la.load(aH + step(1), aL + step(1), ra1);
        lb.load(bH + step(1), bL + step(1), rb1);
        la.store(sA, ra0);
        lb.store(sB, rb0);
        co.put(sOff, t);
        __syncthreads();
        for (int64_t s = 0; s < nsteps; s += 2) {
            // even step: LDS stage 0, set 1 waits for stage 1
            const int64_t k2 = step(s + 2);
            la.load(aH + k2, aL + k2, ra0);
            lb.load(bH + k2, bL + k2, rb0);
            __builtin_amdgcn_s_setprio(1);
            pk_mma<BM, BN>(sA, sB, lane, wm, wn, acc);
            __builtin_amdgcn_s_setprio(0);
            __builtin_amdgcn_sched_barrier(0);
            la.store(sA + Cfg::SA, ra1);
            lb.store(sB + Cfg::SB, rb1);
            __syncthreads();
            // odd step: LDS stage 1, set 0 waits for stage 0 (with an odd step
            // count the last one holds a repeat of the last step: not computed)
            const int64_t k3 = step(s + 3);
            la.load(aH + k3, aL + k3, ra1);
            lb.load(bH + k3, bL + k3, rb1);
            __builtin_amdgcn_s_setprio(1);
            if (s + 1 < nsteps) pk_mma<BM, BN>(sA + Cfg::SA, sB + Cfg::SB, lane, wm, wn, acc);
            __builtin_amdgcn_s_setprio(0);
            __builtin_amdgcn_sched_barrier(0);
            la.store(sA, ra0);
            lb.store(sB, rb0);
            __syncthreads();
        }
    } else {
        u4_t ra[Cfg::CA], rb[Cfg::CB];
        la.load(aH, aL, ra);
        lb.load(bH, bL, rb);
        la.store(sA, ra);
        lb.store(sB, rb);
        co.put(sOff, t);
        __syncthreads();
        for (int64_t s = 0; s < nsteps; ++s) {
            const int cur = (int)(s & 1);
            const int64_t k1 = step(s + 1);
            la.load(aH + k1, aL + k1, ra);
            lb.load(bH + k1, bL + k1, rb);
            __builtin_amdgcn_s_setprio(1);
            pk_mma<BM, BN>(sA + cur * Cfg::SA, sB + cur * Cfg::SB, lane, wm, wn, acc);
            __builtin_amdgcn_s_setprio(0);
            __builtin_amdgcn_sched_barrier(0);
            la.store(sA + (cur ^ 1) * Cfg::SA, ra);
            lb.store(sB + (cur ^ 1) * Cfg::SB, rb);
            __syncthreads();
        }
    }

    pk_epilogue<FM, FN>(g, acc, m0, n0, wm * Cfg::WTM, wn * Cfg::WTN, lane, split, sOff,
                        sOff + BM);
}

// The large tiles: 8 waves (512 threads) as 2 x 4, each wave (BM / 2) x
// (BN / 4), one workgroup per CU.  Thread t stages chunk i of row slot
// u = t / 4 + 128 i of the tile's A (B) rows, hi plane then lo plane (slot
// u is plane u / ROWS, row u % ROWS), four threads per row as above.
template <int ROWS> struct PkLoad8 {
    static_assert(ROWS % 64 == 0, "whole 16-row runs per wave");
    static constexpr int C = ROWS / 64;   // chunks per thread (2 ROWS x 4 over 512 threads)
    uint32_t goff;                         // element offset of the thread's 16 bytes in a block
    int32_t rsl;                           // t / 4
    int c;                                 // t % 4
    int64_t gstride;                       // elements from one row group to the next
    __device__ __forceinline__ void init(int t, int64_t Kq) {
        gstride = Kq * 16;
        c = t & 3;
        rsl = t >> 2;
        goff = (uint32_t)((rsl & 15) * 32 + 8 * c);
    }
    __device__ __forceinline__ void load(const uint16_t *hi, const uint16_t *lo,
                                         u4_t (&v)[C]) const {
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int u = rsl + 128 * i;
            const int pl = u >= ROWS, rr = pl ? u - ROWS : u;
            v[i] = *reinterpret_cast<const u4_t *>((pl ? lo : hi) + (int64_t)(rr >> 4) * gstride +
                                                   goff);
        }
    }
    __device__ __forceinline__ void store(uint16_t *s, const u4_t (&v)[C]) const {
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int u = rsl + 128 * i;
            const int pl = u >= ROWS, rr = pl ? u - ROWS : u;
            *reinterpret_cast<u4_t *>(s + pl * ROWS * kLd + rr * kLd + 8 * (c ^ swz(rr))) = v[i];
        }
    }
};

// DB: B's fragments straight from the packed planes into registers (a
// fragment's operand for one step is one 1 KB block, so a wave reads it in
// one coalesced load), one step ahead in a second register set; only A goes
// through LDS.  B fragments are shared by two waves, A fragments by four, so
// this moves the operand reads that LDS spares least onto the L1 path.
template <int BM, int BN, bool DB = false> struct Pk8Cfg {
    static constexpr int WTM = BM / 2, WTN = BN / 4, FM = WTM / 16, FN = WTN / 16;
    static constexpr int PA = BM * kLd, PB = BN * kLd;
    static constexpr int SA = 2 * PA, SB = DB ? 0 : 2 * PB;
    static constexpr int kLdsBytes = 2 * (SA + SB) * 2;
};

template <int BM, int BN, bool DB>
__global__ __launch_bounds__(512) void bf3_packed_gemm8_kernel(Bf3Packed g) {
    using Cfg = Pk8Cfg<BM, BN, DB>;
    constexpr int FM = Cfg::FM, FN = Cfg::FN;
    extern __shared__ __align__(16) uint16_t lds[];
    uint16_t *sA = lds, *sB = lds + 2 * Cfg::SA;   // [stage][plane][row][kLd]

    const int tiles = g.tilesM * g.tilesN;
    const int logical = xcd_remap(blockIdx.x, tiles * g.splits);
    const int split = logical / tiles;
    int tm, tn;
    tile_coords(logical - split * tiles, g.tilesM, g.tilesN, tm, tn);
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int64_t kbeg = (int64_t)split * g.kPer;
    const int64_t kend = min(kbeg + g.kPer, g.Kq);
    const int64_t nsteps = (kend - kbeg) / 32;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 2, wn = w & 3;
    __shared__ int64_t sOff[BM + BN];
    static_assert(BM + BN <= 512, "one C offset per thread");
    PkCOffs<BM, BN> co;
    co.load(g, m0, n0, t);
    PkLoad8<BM> la;
    PkLoad8<BN> lb;
    la.init(t, g.Kq);
    lb.init(t, g.Kq);
    // first block of the tile's rows at the slice's first step; a step is 512 elements on
    const uint16_t *aH = g.A + m0 * g.Kq + kbeg * 16, *aL = aH + g.planeA;
    const uint16_t *bH = g.B + n0 * g.Kq + kbeg * 16, *bL = bH + g.planeB;

    f4_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

    const int kc = 8 * ((lane >> 4) ^ swz(lane & 15));   // rows start at multiples of 16
    auto mma = [&](const uint16_t *stA, const uint16_t *stB) {
        const __bf16 *ahi = reinterpret_cast<const __bf16 *>(stA), *alo = ahi + Cfg::PA;
        const __bf16 *bhi = reinterpret_cast<const __bf16 *>(stB), *blo = bhi + Cfg::PB;
        bf8_t ah[FM], al[FM];
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            const int r = wm * Cfg::WTM + i * 16 + (lane & 15);
            ah[i] = *reinterpret_cast<const bf8_t *>(ahi + r * kLd + kc);
            al[i] = *reinterpret_cast<const bf8_t *>(alo + r * kLd + kc);
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int r = wn * Cfg::WTN + j * 16 + (lane & 15);
            const bf8_t bh = *reinterpret_cast<const bf8_t *>(bhi + r * kLd + kc);
            const bf8_t bl = *reinterpret_cast<const bf8_t *>(blo + r * kLd + kc);
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc[i][j], 0, 0, 0);
            }
        }
    };

    auto step = [&](int64_t s) { return 512 * (s < nsteps ? s : nsteps - 1); };
    if constexpr (!DB) {
        u4_t ra[PkLoad8<BM>::C], rb[PkLoad8<BN>::C];
        la.load(aH, aL, ra);
        lb.load(bH, bL, rb);
        la.store(sA, ra);
        lb.store(sB, rb);
        co.put(sOff, t);
        __syncthreads();
        for (int64_t s = 0; s < nsteps; ++s) {
            const int cur = (int)(s & 1);
            const int64_t k1 = step(s + 1);
            la.load(aH + k1, aL + k1, ra);
            lb.load(bH + k1, bL + k1, rb);
            // raised priority while issuing MFMAs: a wave that holds its operands
            // runs ahead of the waves still reading LDS (measured 6 % faster)
            __builtin_amdgcn_s_setprio(1);
            mma(sA + cur * Cfg::SA, sB + cur * Cfg::SB);
            __builtin_amdgcn_s_setprio(0);
            __builtin_amdgcn_sched_barrier(0);
            la.store(sA + (cur ^ 1) * Cfg::SA, ra);
            lb.store(sB + (cur ^ 1) * Cfg::SB, rb);
            __syncthreads();
        }
    } else {
        // lane l's 16 bytes of a fragment block: row l % 16, chunk l / 16
        // (the chunk it reads from LDS in the other form)
        const int64_t bl0 = (int64_t)(wn * Cfg::WTN / 16) * lb.gstride + (lane & 15) * 32 +
                            8 * (lane >> 4);
        auto bload = [&](int64_t k, bf8_t (&bh)[FN], bf8_t (&blo)[FN]) {
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int64_t o = bl0 + (int64_t)j * lb.gstride + k;
                bh[j] = *reinterpret_cast<const bf8_t *>(bH + o);
                blo[j] = *reinterpret_cast<const bf8_t *>(bL + o);
            }
        };
        // One B register set: fragment j's MFMAs for this step come first, then
        // (behind a scheduling barrier, so the registers are reused rather
        // than renamed) its load for the next step, which has the rest of this
        // step and the barrier to arrive.
        auto mma_b = [&](const uint16_t *stA, bf8_t (&bh)[FN], bf8_t (&blo)[FN], int64_t knext) {
            const __bf16 *ahi = reinterpret_cast<const __bf16 *>(stA), *alo = ahi + Cfg::PA;
            bf8_t ah[FM], al[FM];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const int r = wm * Cfg::WTM + i * 16 + (lane & 15);
                ah[i] = *reinterpret_cast<const bf8_t *>(ahi + r * kLd + kc);
                al[i] = *reinterpret_cast<const bf8_t *>(alo + r * kLd + kc);
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], blo[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                }
                __builtin_amdgcn_sched_barrier(0);
                const int64_t o = bl0 + (int64_t)j * lb.gstride + knext;
                bh[j] = *reinterpret_cast<const bf8_t *>(bH + o);
                blo[j] = *reinterpret_cast<const bf8_t *>(bL + o);
            }
        };
        u4_t ra[PkLoad8<BM>::C];
        bf8_t bh[FN], blo[FN];
        la.load(aH, aL, ra);
        bload(0, bh, blo);
        la.store(sA, ra);
        co.put(sOff, t);
        __syncthreads();
        for (int64_t s = 0; s < nsteps; ++s) {
            const int cur = (int)(s & 1);
            const int64_t k1 = step(s + 1);
            la.load(aH + k1, aL + k1, ra);
            __builtin_amdgcn_s_setprio(1);
            mma_b(sA + cur * Cfg::SA, bh, blo, k1);
            __builtin_amdgcn_s_setprio(0);
            __builtin_amdgcn_sched_barrier(0);
            la.store(sA + (cur ^ 1) * Cfg::SA, ra);
            __syncthreads();
        }
    }

    pk_epilogue<FM, FN>(g, acc, m0, n0, wm * Cfg::WTM, wn * Cfg::WTN, lane, split, sOff,
                        sOff + BM);
}

// ---------------------------------------------------------------------------
// The packed FP64 form: the same pass (values copied, not split) into 2 KB
// blocks of 16 rows by 16 positions, and a GEMM on the 16x16x4 FP64 MFMA.
// ---------------------------------------------------------------------------
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double d2v_t __attribute__((ext_vector_type(2)));

// LDS rows hold one step's 16 positions (128 bytes, unpadded); position k of
// row r sits at k ^ (r % 16), so the MFMA operand reads (16 rows, one
// position) and the 16-byte stores (eight threads per row) are free of bank
// conflicts.  A 16-byte chunk (positions 2c, 2c + 1) lands on the aligned
// pair c ^ ((r % 16) / 2), its two values swapped when r is odd.
template <int ROWS> struct Pk64Load {
    static_assert(ROWS % 32 == 0, "32 rows per chunk index");
    static constexpr int C = ROWS / 32;   // 16-byte chunks per thread (ROWS x 8 over 256)
    uint32_t goff;      // element offset of the thread's chunk inside a block
    int rg0, row0, c;
    int64_t gstride;    // elements from one row group to the next (Kq * 16)
    __device__ __forceinline__ void init(int t, int64_t Kq) {
        c = t & 7;
        row0 = t >> 3;   // 0 .. 31
        rg0 = row0 >> 4;
        gstride = Kq * 16;
        goff = (uint32_t)((row0 & 15) * 16 + 2 * c);
    }
    __device__ __forceinline__ void load(const double *base, d2v_t (&v)[C]) const {
#pragma unroll
        for (int i = 0; i < C; ++i)
            v[i] = *reinterpret_cast<const d2v_t *>(base + (int64_t)(2 * i + rg0) * gstride + goff);
    }
    __device__ __forceinline__ void store(double *sm, const d2v_t (&v)[C]) const {
        const int m = row0 & 15;   // the same for every chunk (rows 32 i apart)
        const int q = c ^ (m >> 1);
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int row = 32 * i + row0;
            const d2v_t x = (m & 1) ? d2v_t{v[i].y, v[i].x} : v[i];
            *reinterpret_cast<d2v_t *>(sm + row * 16 + 2 * q) = x;
        }
    }
};

template <int BM, int BN>
__global__ __launch_bounds__(256) void f64_packed_gemm_kernel(F64Packed g) {
    constexpr int WTM = BM / 2, WTN = BN / 2, FM = WTM / 16, FN = WTN / 16;
    constexpr int SA = BM * 16, SB = BN * 16;   // doubles of one LDS stage per operand
    extern __shared__ __align__(16) double lds64[];
    double *sA = lds64, *sB = lds64 + 2 * SA;

    const int tiles = g.tilesM * g.tilesN;
    const int logical = xcd_remap(blockIdx.x, tiles * g.splits);
    const int split = logical / tiles;
    int tm, tn;
    tile_coords(logical - split * tiles, g.tilesM, g.tilesN, tm, tn);
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int64_t kbeg = (int64_t)split * g.kPer;
    const int64_t kend = min(kbeg + g.kPer, g.Kq);
    const int64_t nsteps = (kend - kbeg) / 16;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
    Pk64Load<BM> la;
    Pk64Load<BN> lb;
    la.init(t, g.Kq);
    lb.init(t, g.Kq);
    const double *aB = g.A + m0 * g.Kq + kbeg * 16, *bB = g.B + n0 * g.Kq + kbeg * 16;

    d4_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

    const int lr = lane & 15, lk = lane >> 4;
    auto mma = [&](const double *stA, const double *stB) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int ph = (4 * kk + lk) ^ lr;   // rows start at multiples of 16
            double a[FM], b[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) a[i] = stA[(wm * WTM + i * 16 + lr) * 16 + ph];
#pragma unroll
            for (int j = 0; j < FN; ++j) b[j] = stB[(wn * WTN + j * 16 + lr) * 16 + ph];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    };

    auto step = [&](int64_t s) { return 256 * (s < nsteps ? s : nsteps - 1); };
    d2v_t ra[Pk64Load<BM>::C], rb[Pk64Load<BN>::C];
    la.load(aB, ra);
    lb.load(bB, rb);
    la.store(sA, ra);
    lb.store(sB, rb);
    __syncthreads();
    for (int64_t s = 0; s < nsteps; ++s) {
        const int cur = (int)(s & 1);
        const int64_t k1 = step(s + 1);
        la.load(aB + k1, ra);
        lb.load(bB + k1, rb);
        mma(sA + cur * SA, sB + cur * SB);
        __builtin_amdgcn_sched_barrier(0);
        la.store(sA + (cur ^ 1) * SA, ra);
        lb.store(sB + (cur ^ 1) * SB, rb);
        __syncthreads();
    }

    // Epilogue: fragment (i, j), register v of lane l holds M row
    // l / 16 + 4 v and N column l % 16 of the fragment; FP64 partials of a K
    // slice, or C <- beta C_in + alpha sum, one fragment's C_in read before
    // any of it is written.
    double *__restrict__ C = g.C;
    const bool rdC = g.beta != 0.0;
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int64_t n = n0 + wn * WTN + j * 16 + lr;
        const bool nok = n < g.N;
        const int64_t ocn = nok ? g.offCN[n] : 0;
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            int64_t off[4];
            bool ok[4];
            double cin[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t m = m0 + wm * WTM + i * 16 + lk + 4 * v;
                ok[v] = nok && m < g.M;
                if (g.ws) {
                    if (ok[v]) g.ws[((int64_t)split * g.M + m) * g.N + n] = acc[i][j][v];
                    ok[v] = false;
                    continue;
                }
                off[v] = ok[v] ? g.offCM[m] + ocn : 0;
                cin[v] = (rdC && ok[v]) ? C[off[v]] : 0.0;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (!ok[v]) continue;
                const double r = acc[i][j][v];
                C[off[v]] = rdC ? g.beta * cin[v] + g.alpha * r : g.alpha * r;
            }
        }
    }
}

}  // namespace

int launch_pack(bool f64, const void *X, const int64_t *offR, const int32_t *rowMap, int64_t R,
                const int64_t *offK, int64_t K, int64_t Kq, bool rowsFast, void *P, int64_t plane,
                hipStream_t s) {
    if (R == 0) return 0;
    const int64_t tasks = rowsFast ? (R + 16 * kPackBlocksR - 1) / (16 * kPackBlocksR) * ((Kq / 8 + 3) / 4)
                                   : (R + kPackRowsK - 1) / kPackRowsK * ((Kq + 511) / 512);
    const int64_t blocks = (tasks + 3) / 4;
    if (blocks > INT32_MAX) return GETT_ERR_INTERNAL;
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    if (f64) {
        const double *Xd = static_cast<const double *>(X);
        if (rowsFast)
            hipLaunchKernelGGL(pack_rows_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, Xd,
                               offR, rowMap, R, offK, K, Kq, P, plane);
        else
            hipLaunchKernelGGL(pack_k_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, Xd,
                               offR, R, offK, K, Kq, P, plane);
    } else {
        const float *Xf = static_cast<const float *>(X);
        if (rowsFast)
            hipLaunchKernelGGL(pack_rows_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s,
                               Xf, offR, rowMap, R, offK, K, Kq, P, plane);
        else
            hipLaunchKernelGGL(pack_k_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, Xf,
                               offR, R, offK, K, Kq, P, plane);
    }
    return launch_status();
}

template <int BM, int BN> static int launch_gemm(const Bf3Packed &g, hipStream_t s) {
    using Cfg = PkCfg<BM, BN>;
    static bool attr_set = false;   // set once per process (every device takes the same value)
    if (!attr_set) {
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(bf3_packed_gemm_kernel<BM, BN>),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                Cfg::kLdsBytes) != hipSuccess)
            return GETT_ERR_HIP;
        attr_set = true;
    }
    const int64_t total = (int64_t)g.tilesM * g.tilesN * g.splits;
    if (total > INT32_MAX) return GETT_ERR_INTERNAL;
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    auto kern = bf3_packed_gemm_kernel<BM, BN>;
    hipLaunchKernelGGL(kern, dim3((unsigned)total), dim3(256), Cfg::kLdsBytes, s, g);
    return launch_status();
}

constexpr bool kGemm8DirectB = true;

template <int BM, int BN> static int launch_gemm8(const Bf3Packed &g, hipStream_t s) {
    using Cfg = Pk8Cfg<BM, BN, kGemm8DirectB>;
    static bool attr_set = false;   // set once per process (every device takes the same value)
    if (!attr_set) {
        if (hipFuncSetAttribute(
                reinterpret_cast<const void *>(bf3_packed_gemm8_kernel<BM, BN, kGemm8DirectB>),
                hipFuncAttributeMaxDynamicSharedMemorySize, Cfg::kLdsBytes) != hipSuccess)
            return GETT_ERR_HIP;
        attr_set = true;
    }
    const int64_t total = (int64_t)g.tilesM * g.tilesN * g.splits;
    if (total > INT32_MAX) return GETT_ERR_INTERNAL;
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    auto kern = bf3_packed_gemm8_kernel<BM, BN, kGemm8DirectB>;
    hipLaunchKernelGGL(kern, dim3((unsigned)total), dim3(512), Cfg::kLdsBytes, s, g);
    return launch_status();
}

int launch_f64_packed_gemm(const F64Packed &g, hipStream_t s) {
    constexpr int BM = 128, BN = 128;
    constexpr int kLds = 2 * (BM + BN) * 16 * (int)sizeof(double);
    static bool attr_set = false;   // set once per process (every device takes the same value)
    if (!attr_set) {
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(f64_packed_gemm_kernel<BM, BN>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kLds) != hipSuccess)
            return GETT_ERR_HIP;
        attr_set = true;
    }
    const int64_t total = (int64_t)g.tilesM * g.tilesN * g.splits;
    if (total > INT32_MAX) return GETT_ERR_INTERNAL;
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    auto kern = f64_packed_gemm_kernel<BM, BN>;
    hipLaunchKernelGGL(kern, dim3((unsigned)total), dim3(256), kLds, s, g);
    return launch_status();
}

int launch_bf3_packed_gemm(int bm, int bn, const Bf3Packed &g, hipStream_t s) {
    if (bm == 128 && bn == 128) return launch_gemm<128, 128>(g, s);
    if (bm == 192 && bn == 256) return launch_gemm8<192, 256>(g, s);
    return GETT_ERR_INTERNAL;
}

}  // namespace gett
