// gett_tile.h -- table-driven contraction tiles for gfx950 (MI355X).
//
// One workgroup (4 waves, 2x2) owns a BM x BN tile of the planned GEMM
//   C[offCM[m] + offCN[n]] += sum_k A[offAM[m] + offAK[k]] * B[offBK[k] + offBN[n]]
// and walks K in steps of BK:
//   gather:  each thread reads its share of the A and B sub-tiles straight
//            from the strided tensors (no packed copy is ever written).  For
//            each operand the planner says whether its cheapest direction in
//            memory is the free axis or the contracted axis; consecutive
//            threads run along that axis so that a wave's loads share cache
//            lines.  The free offsets a thread needs are fixed for the whole
//            tile and held in registers; the contracted offsets of a step
//            come from one vector load (broadcast with readlane where they
//            are wave-uniform).
//   stage:   values go to LDS (double-buffered; the next step's global loads
//            are in flight while the current step runs on the matrix cores).
//            The BF16x3 path splits each FP32 value into hi/lo bfloat16 planes
//            on the way into LDS.
//   MFMA:    FP64 and FP32 use the 16x16x4 MFMA, BF16x3 the 16x16x32 BF16 MFMA
//            (hi*hi into one FP32 accumulator, hi*lo + lo*hi into another).
//   epilogue: the planner puts C's fastest mode on the N axis, which is the
//            lane axis of the MFMA result, so 16 lanes update 16 neighbouring
//            outputs; PERM and INCC live entirely in the offC tables.  With
//            split-K the partial sums go to a workspace instead and a second
//            kernel adds them to C_in in a fixed order, in FP64.
// The sum is Algorithm 1's inner loop (Section 6) for every output of the
// tile at once; only the summation order differs.
#pragma once

#include "gett_grid.h"
#include "gett_internal.h"

namespace gett {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef double d2_t __attribute__((ext_vector_type(2)));
typedef float f2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// T: an element of the data; R: its real type (the MFMA operand type);
// complex elements are (re, im) pairs.
template <int PREC> struct PrecT;
template <> struct PrecT<kF64> { using T = double; using R = double; using Acc = d4_t; };
template <> struct PrecT<kF32> { using T = float; using R = float; using Acc = f4_t; };
template <> struct PrecT<kBF3> { using T = float; using R = float; using Acc = f4_t; };
template <> struct PrecT<kZ64> { using T = d2_t; using R = double; using Acc = d4_t; };
template <> struct PrecT<kC32> { using T = f2_t; using R = float; using Acc = f4_t; };

// Shared-memory layout of one operand tile (ROWS free positions x BK).
//   FP64/FP32: [BK][ROWS + 1]  (k-major; a 16x4 MFMA operand is 16 neighbours
//              in one k row; the +1 keeps column writes off one bank)
//   complex:   real and imaginary planes, each [BK][ROWS + 1]
//   BF16x3:    hi and lo planes, each [ROWS][BK + 8] bfloat16 (k contiguous;
//              one 16-byte read gives a lane its 8 k values)
template <int PREC, int ROWS, int BK> struct OpLds {
    static constexpr bool kSplit = PREC == kBF3;
    static constexpr bool kCplx = prec_complex(PREC);
    static constexpr int kLd = kSplit ? BK + 8 : ROWS + 1;
    static constexpr int kPlane = BK * kLd;            // elements of one plane (plain values)
    static constexpr int kElems = kSplit ? 2 * ROWS * kLd : (kCplx ? 2 : 1) * kPlane;
    static constexpr int kBytes =
        kSplit ? kElems * 2 : kElems * ((PREC == kF64 || PREC == kZ64) ? 8 : 4);
};

// Zeros read in place of masked-off elements (contracted positions of a
// range's first step that lie below the range): a load from here needs no
// select afterwards, so the loaded value can go straight to LDS.
static __device__ __align__(16) double g_gett_zero[8] = {0, 0, 0, 0, 0, 0, 0, 0};

#ifdef GETT_ADDR_CHECK
// Checked build: every gathered element and every C element is tested
// against its tensor's addressed range [lo, lo + span] (element offsets from
// the tensor's pointer); an access outside is counted here and redirected to
// the zero buffer (loads) or dropped (stores), so it cannot fault.
static __device__ unsigned long long g_gett_viol = 0;

template <class T>
__device__ __forceinline__ const T *gett_checked(const T *X, const T *ptr, int64_t lo, int64_t span) {
    const T *zero = reinterpret_cast<const T *>(g_gett_zero);
    if (ptr == zero) return ptr;   // masked positions read the zero buffer on purpose
    const int64_t d = ptr - X;
    if (d < lo || d > lo + span) {
        atomicAdd(&g_gett_viol, 1ull);
        return zero;
    }
    return ptr;
}

__device__ __forceinline__ bool gett_check_c(int64_t off, int64_t lo, int64_t span) {
    if (off < lo || off > lo + span) {
        atomicAdd(&g_gett_viol, 1ull);
        return false;
    }
    return true;
}
#define GETT_CHECK_C(off, p) if (!gett_check_c((off), (p).cLo, (p).cSpan)) continue
#else
#define GETT_CHECK_C(off, p) (void)0
#endif

// Split two FP32 values into packed bfloat16 pairs: hi = bf16(x) (round to
// nearest even), lo = bf16(x - hi) (the subtraction is exact).  Element 0
// goes to the low half of each word.
__device__ __forceinline__ void bf16x3_split_pair(float x0, float x1, uint32_t &hi, uint32_t &lo) {
    typedef float f2_t __attribute__((ext_vector_type(2)));
    typedef __bf16 b2_t __attribute__((ext_vector_type(2)));
    hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2_t{x0, x1}, b2_t));
    const float h0 = __uint_as_float(hi << 16), h1 = __uint_as_float(hi & 0xffff0000u);
    lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2_t{x0 - h0, x1 - h1}, b2_t));
}

// Gather of one operand's ROWS x BK sub-tile into registers.
//
// Within a step, the LDS column c of both operands holds contracted position
// kpos(c) of the step; any permutation works as long as A and B share it.
// FP64/FP32 use the identity.  BF16x3 uses c = 2q + e <-> q + e * BK/2, so
// that a thread that runs along K with lanes q = 0 .. BK/2 - 1 (neighbouring
// lanes read neighbouring positions) holds two values that are neighbours in
// LDS and writes each plane as one 4-byte word, and a thread that runs along
// the free axis holds a contiguous run of columns and writes 16-byte chunks.
template <int PREC, int ROWS, int BK, bool FASTK, bool O32 = false> struct Gather {
    using T = typename PrecT<PREC>::T;
    using R = typename PrecT<PREC>::R;
    static constexpr bool kSplit = PREC == kBF3;
    static constexpr bool kCplx = prec_complex(PREC);
    static constexpr int PER = ROWS * BK / kThreads;   // values per thread
    static constexpr int KP = (kSplit && FASTK) ? 2 : 1;   // positions per row (FASTK)
    static constexpr int KL = BK / KP;                 // lanes along K per row (FASTK)
    static constexpr int NF = FASTK ? PER / KP : 1;     // rows per thread
    static_assert(ROWS * BK % kThreads == 0, "tile too small for the workgroup");
    static_assert(FASTK ? (kThreads % KL == 0) : (kThreads % ROWS == 0), "loader shape");
    static_assert(BK <= 64, "one wave holds a step's contracted offsets");
    static_assert(!kSplit || FASTK || PER % 8 == 0, "16-byte LDS chunks");

    // !FASTK: every value a thread loads sits in a wave-uniform LDS column,
    // so its contracted offset is the same for the whole wave and is read
    // with a scalar load (one per value, no lane shuffles).
    static constexpr bool kScalarK = !FASTK;
    static constexpr int NK = kScalarK ? PER : KP;     // offsets held per step
    // O32 (real values, operand span below 4 GB): the whole-step loads take
    // a wave-uniform 64-bit base and a 32-bit byte offset per lane, so a
    // value costs one 32-bit add (lanes along K) or none (lanes along the
    // free axis, whose contracted offset joins the uniform base).
    static_assert(!O32 || !kCplx, "32-bit addressing is for real values");

    const T *base[NF];  // X + free offset of each row this thread reads
    int row[NF];        // tile row of each free offset
    int j0;             // !FASTK: wave-uniform column group; FASTK: lane position q
    int64_t koff[NK];   // contracted offsets for the current step
    const T *lo;        // O32: X + the lowest element offset the operand addresses
    uint32_t vrow[NF];  // O32: byte offset of each row's free offset from lo
#ifdef GETT_ADDR_CHECK
    const T *cX;        // the operand's pointer and addressed range
    int64_t cLo, cSpan;
    __device__ __forceinline__ const T *chk(const T *ptr) const {
        return gett_checked(cX, ptr, cLo, cSpan);
    }
#else
    __device__ __forceinline__ const T *chk(const T *ptr) const { return ptr; }
#endif

    static __device__ __forceinline__ constexpr int kpos(int c) {
        return kSplit ? (c >> 1) + (c & 1) * (BK / 2) : c;
    }
    // !FASTK: LDS column of the thread's i-th value.
    __device__ __forceinline__ int col(int i) const {
        return kSplit ? j0 * PER + i : j0 + i * (kThreads / ROWS);
    }

    __device__ void init(const T *X, int t, int64_t r0, int64_t nrows,
                         const int64_t *__restrict__ offFree, int boxX, int64_t xlo = 0,
                         int64_t xspan = 0) {
        if constexpr (O32) lo = X + xlo;
#ifdef GETT_ADDR_CHECK
        cX = X;
        cLo = xlo;
        cSpan = xspan;
#else
        (void)xspan;
#endif
        if constexpr (!FASTK) {
            const int il = t % ROWS;                 // consecutive threads: consecutive il
            const int x = il % boxX, y = il / boxX;  // loader walks the box's x side
            const int r = y + (ROWS / boxX) * x;     // tile row (C-fast side first)
            const int64_t g = r0 + r;
            row[0] = r;
            base[0] = X + offFree[g];
            if constexpr (O32) vrow[0] = (uint32_t)(offFree[g] - xlo) * (uint32_t)sizeof(T);
            j0 = __builtin_amdgcn_readfirstlane(t / ROWS);
        } else {
            j0 = t % KL;
#pragma unroll
            for (int i = 0; i < NF; ++i) {
                const int r = t / KL + i * (kThreads / KL);
                const int64_t g = r0 + r;
                row[i] = r;
                base[i] = X + offFree[g];
                if constexpr (O32) vrow[i] = (uint32_t)(offFree[g] - xlo) * (uint32_t)sizeof(T);
            }
        }
    }

    // Contracted offsets of the step starting at k0: offK[k0 + kpos(c)] for
    // each (wave-uniform) column c a thread along the free axis loads, or
    // offK[k0 + q + e * KL] when threads run along K.
    __device__ __forceinline__ void load_koffs(const int64_t *__restrict__ offK, int64_t k0) {
        if constexpr (kScalarK) {
#pragma unroll
            for (int i = 0; i < PER; ++i) koff[i] = offK[k0 + kpos(col(i))];
        } else if constexpr (O32) {
            // only the low word takes part in 32-bit addressing: load just it
            const uint32_t *lo32 = reinterpret_cast<const uint32_t *>(offK);
#pragma unroll
            for (int e = 0; e < KP; ++e) koff[e] = lo32[2 * (k0 + j0 + e * KL)];
        } else {
#pragma unroll
            for (int e = 0; e < KP; ++e) koff[e] = offK[k0 + j0 + e * KL];
        }
    }

    // The same for a step that may start below klo (the first step of a
    // range): positions below klo take klo's offset (their values are masked).
    __device__ __forceinline__ void load_koffs_from(const int64_t *__restrict__ offK, int64_t k0,
                                                    int64_t klo) {
        if constexpr (kScalarK) {
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int64_t k = k0 + kpos(col(i));
                koff[i] = offK[k < klo ? klo : k];
            }
        } else {
#pragma unroll
            for (int e = 0; e < KP; ++e) {
                const int64_t k = k0 + j0 + e * KL;
                koff[e] = offK[k < klo ? klo : k];
            }
        }
    }

    // Values of the step starting at k0.  Rows past the operand's extent read
    // the element of row 0 (their padded offset is 0) and are never stored,
    // so only contracted positions need masking, and only in the first step
    // of a range (MASKED), which may start below klo: those positions read
    // the zero buffer instead.
    template <bool MASKED>
    __device__ __forceinline__ void load(int64_t k0, int64_t klo, T (&v)[PER]) const {
        load_with<MASKED>(koff, k0, klo, v);
    }

    // The same with contracted offsets held elsewhere (a copy taken before
    // the next step's offsets were requested into koff).
    template <bool MASKED>
    __device__ __forceinline__ void load_with(const int64_t (&ko_)[NK], int64_t k0, int64_t klo,
                                              T (&v)[PER]) const {
        const T *zero = reinterpret_cast<const T *>(g_gett_zero);
        if constexpr (O32 && !MASKED) {
            // lo + vrow + (contracted offset) * size, all within 4 GB of lo:
            // the 32-bit sum wraps to the exact byte offset.
            const char *b = reinterpret_cast<const char *>(lo);
            if constexpr (kScalarK) {
                // The empty asm statements keep the uniform base in SGPRs and
                // the lane offset a 32-bit value inside the loop, so the load
                // is selected as base + zero-extended offset (no 64-bit add).
                uint32_t vr = vrow[0];
#ifndef GETT_ADDR_CHECK
                asm("" : "+v"(vr));
#endif
#pragma unroll
                for (int i = 0; i < PER; ++i) {
                    uint64_t bk = reinterpret_cast<uint64_t>(lo + ko_[i]);
#ifndef GETT_ADDR_CHECK
                    asm("" : "+s"(bk));
#endif
                    using GT = const __attribute__((address_space(1))) char;
#ifdef GETT_ADDR_CHECK
                    v[i] = *chk(reinterpret_cast<const T *>(reinterpret_cast<const char *>(bk) + vr));
#else
                    v[i] = *reinterpret_cast<const __attribute__((address_space(1))) T *>(
                        reinterpret_cast<GT *>(bk) + vr);
#endif
                }
            } else {
#pragma unroll
                for (int e = 0; e < KP; ++e) {
                    const uint32_t kb = (uint32_t)ko_[e] * (uint32_t)sizeof(T);
#pragma unroll
                    for (int i = 0; i < NF; ++i)
                        v[i * KP + e] = *chk(reinterpret_cast<const T *>(b + (uint32_t)(vrow[i] + kb)));
                }
            }
        } else if constexpr (kScalarK) {
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const T *ptr = base[0] + ko_[i];
                if constexpr (MASKED) ptr = (k0 + kpos(col(i)) >= klo) ? ptr : zero;
                v[i] = *chk(ptr);
            }
        } else {
#pragma unroll
            for (int e = 0; e < KP; ++e) {
                const bool kk = k0 + j0 + e * KL >= klo;
#pragma unroll
                for (int i = 0; i < NF; ++i) {
                    const T *ptr = base[i] + ko_[e];
                    if constexpr (MASKED) ptr = kk ? ptr : zero;
                    v[i * KP + e] = *chk(ptr);
                }
            }
        }
    }

    // Write the registers into the LDS tile.
    __device__ __forceinline__ void store(void *lds, const T (&v)[PER]) const {
        using L = OpLds<PREC, ROWS, BK>;
        if constexpr (kSplit) {
            uint32_t *hi = reinterpret_cast<uint32_t *>(lds);       // bfloat16 pairs
            uint32_t *lo = hi + ROWS * L::kLd / 2;
            if constexpr (FASTK) {
#pragma unroll
                for (int i = 0; i < NF; ++i) {
                    uint32_t h, l;
                    bf16x3_split_pair(v[2 * i], v[2 * i + 1], h, l);
                    const int w = (row[i] * L::kLd + 2 * j0) / 2;
                    hi[w] = h;
                    lo[w] = l;
                }
            } else {
                const int w0 = (row[0] * L::kLd + j0 * PER) / 2;
#pragma unroll
                for (int c = 0; c < PER / 8; ++c) {
                    uint4 h, l;
                    bf16x3_split_pair(v[8 * c + 0], v[8 * c + 1], h.x, l.x);
                    bf16x3_split_pair(v[8 * c + 2], v[8 * c + 3], h.y, l.y);
                    bf16x3_split_pair(v[8 * c + 4], v[8 * c + 5], h.z, l.z);
                    bf16x3_split_pair(v[8 * c + 6], v[8 * c + 7], h.w, l.w);
                    *reinterpret_cast<uint4 *>(hi + w0 + 4 * c) = h;
                    *reinterpret_cast<uint4 *>(lo + w0 + 4 * c) = l;
                }
            }
        } else if constexpr (kCplx) {
            R *s = reinterpret_cast<R *>(lds);
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int r = FASTK ? row[i] : row[0];
                const int j = FASTK ? j0 : col(i);
                s[j * L::kLd + r] = v[i].x;
                s[L::kPlane + j * L::kLd + r] = v[i].y;
            }
        } else {
            T *s = reinterpret_cast<T *>(lds);
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int r = FASTK ? row[i] : row[0];
                const int j = FASTK ? j0 : col(i);
                s[j * L::kLd + r] = v[i];
            }
        }
    }
};

template <int PREC, int BM, int BN, int BK> struct TileCfg {
    static constexpr int WTM = BM / 2, WTN = BN / 2;   // per-wave sub-tile
    static constexpr int FM = WTM / 16, FN = WTN / 16; // 16x16 fragments per wave
    using LA = OpLds<PREC, BM, BK>;
    using LB = OpLds<PREC, BN, BK>;
    static constexpr int kStageBytes = LA::kBytes + LB::kBytes;
    static constexpr int kLdsBytes = 2 * kStageBytes;
    static_assert(BK % (PREC == kBF3 ? 32 : 4) == 0, "BK");
    // The tile's C offsets (BM + BN of them) can sit in LDS after the two
    // stages; the tile kernel stages them there when that leaves the number
    // of workgroups a CU's 160 KB of LDS holds unchanged.
    static constexpr int kCOffBytes = (BM + BN) * 8;
    static_assert(kLdsBytes % 8 == 0 && BM + BN <= kThreads, "C offset staging");
    static constexpr bool kCOffFree =
        kLdsPerCu / (kLdsBytes + kCOffBytes) == kLdsPerCu / kLdsBytes;
    static constexpr int kLaunchLds = kLdsBytes + (kCOffFree ? kCOffBytes : 0);
    // BF16x3 tiles for which that room would cost a workgroup keep the
    // offsets in the last 16 bytes of each row of stage 0's A hi plane
    // (columns BK .. BK + 7, which neither the stores nor the MFMA reads
    // touch): two a row, room for 2 BM of them.
    static constexpr bool kCOffPad = !kCOffFree && PREC == kBF3 && BN <= BM;
    // where the tile kernel stages its C offsets (kCOffNone / kCOffAfter / kCOffInPad)
    static constexpr int kCOffMode = kCOffFree ? 1 : (kCOffPad ? 2 : 0);
};

// LDS of the batch kernel: the larger of its two tiles' stages, plus room
// for the C offsets when that costs no workgroup per CU.
template <int PREC> struct BatchLds {
    using C0 = TileCfg<PREC, kTiles[PREC][kBatchTile[PREC][0]].bm, kTiles[PREC][kBatchTile[PREC][0]].bn,
                       kTiles[PREC][kBatchTile[PREC][0]].bk>;
    using C1 = TileCfg<PREC, kTiles[PREC][kBatchTile[PREC][1]].bm, kTiles[PREC][kBatchTile[PREC][1]].bn,
                       kTiles[PREC][kBatchTile[PREC][1]].bk>;
    static constexpr int kBase = C0::kLdsBytes > C1::kLdsBytes ? C0::kLdsBytes : C1::kLdsBytes;
    static constexpr int kWith0 = C0::kLdsBytes + C0::kCOffBytes;
    static constexpr int kWith1 = C1::kLdsBytes + C1::kCOffBytes;
    static constexpr int kWith = kWith0 > kWith1 ? kWith0 : kWith1;
    static constexpr bool kCOff = kLdsPerCu / kWith == kLdsPerCu / kBase;
    static constexpr int kBytes = kCOff ? kWith : kBase;
};

// MFMA work of one staged K step for the FP64/FP32 tiles that load two
// steps ahead: the wave's FM x FN fragments over the stage's BK contracted
// positions.
template <int PREC, int BM, int BN, int BK>
__device__ __forceinline__ void mma_stage(typename PrecT<PREC>::Acc (&acc)[BM / 32][BN / 32],
                                          const unsigned char *stA, const unsigned char *stB,
                                          int lane, int wm, int wn) {
    static_assert(PREC == kF64 || PREC == kF32, "plain MFMA tiles only");
    using Cfg = TileCfg<PREC, BM, BN, BK>;
    using T = typename PrecT<PREC>::T;
    constexpr int FM = Cfg::FM, FN = Cfg::FN;
    const T *sa = reinterpret_cast<const T *>(stA);
    const T *sb = reinterpret_cast<const T *>(stB);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
        const int kr = ks * 4 + (lane >> 4);
        T a[FM], b[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
            a[i] = sa[kr * Cfg::LA::kLd + wm * Cfg::WTM + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < FN; ++j)
            b[j] = sb[kr * Cfg::LB::kLd + wn * Cfg::WTN + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                if constexpr (PREC == kF64)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
                else
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
            }
    }
}

// MFMA work of one staged K step of the BF16x3 tiles that load two steps
// ahead: hi*hi, hi*lo and lo*hi, all into acc.
template <int BM, int BN, int BK>
__device__ __forceinline__ void mma_stage_split(f4_t (&acc)[BM / 32][BN / 32],
                                                const unsigned char *stA, const unsigned char *stB,
                                                int lane, int wm, int wn) {
    using Cfg = TileCfg<kBF3, BM, BN, BK>;
    constexpr int FM = Cfg::FM, FN = Cfg::FN;
    const __bf16 *ahi = reinterpret_cast<const __bf16 *>(stA);
    const __bf16 *alo = ahi + BM * Cfg::LA::kLd;
    const __bf16 *bhi = reinterpret_cast<const __bf16 *>(stB);
    const __bf16 *blo = bhi + BN * Cfg::LB::kLd;
#pragma unroll
    for (int ks = 0; ks < BK / 32; ++ks) {
        const int kc = ks * 32 + 8 * (lane >> 4);
        bf8_t ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            const int r = wm * Cfg::WTM + i * 16 + (lane & 15);
            ah[i] = *reinterpret_cast<const bf8_t *>(ahi + r * Cfg::LA::kLd + kc);
            al[i] = *reinterpret_cast<const bf8_t *>(alo + r * Cfg::LA::kLd + kc);
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int r = wn * Cfg::WTN + j * 16 + (lane & 15);
            bh[j] = *reinterpret_cast<const bf8_t *>(bhi + r * Cfg::LB::kLd + kc);
            bl[j] = *reinterpret_cast<const bf8_t *>(blo + r * Cfg::LB::kLd + kc);
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
            }
    }
}

// One BM x BN tile over contracted range [kbeg, kend), reading A and B from
// pA and pB and updating C at pC (the call's pointers, moved to a Hadamard
// position when there is one); `slice` numbers the tile's FP64 partial-sum
// slab when K is split.
template <int PREC, int BM, int BN, int BK, bool AFK, bool BFK, bool O32 = false, int COM = 0>
__device__ __forceinline__ void gett_tile(const TileParams &p, const void *pA, const void *pB,
                                          void *pC, int64_t m0, int64_t n0, int64_t kbeg,
                                          int64_t kend, int split, unsigned char *smem) {
    using Cfg = TileCfg<PREC, BM, BN, BK>;
    using T = typename PrecT<PREC>::T;
    using R = typename PrecT<PREC>::R;
    using Acc = typename PrecT<PREC>::Acc;
    constexpr int FM = Cfg::FM, FN = Cfg::FN;
    constexpr bool kSplit = PREC == kBF3;
    constexpr bool kCplx = prec_complex(PREC);
    // Complex tiles keep the real and imaginary sums apart (acc | acx).  The
    // BF16x3 tiles add all three products into one FP32 set: the cross
    // terms are 2^-8 of hi*hi, so a second set would save little rounding
    // and costs occupancy.
    constexpr bool kTwoAcc = kCplx;

    const int t = threadIdx.x;
    const int lane = lane_id();
    const int w = wave_id();
    const int wm = w >> 1, wn = w & 1;

    // COM 1 or 2: the tile's C offsets (its M rows, then its N positions)
    // are requested here and staged in LDS at the first barrier, after the
    // operand stages (1) or in the BF16x3 rows' unused tail bytes (2), so the
    // epilogue waits for C_in alone instead of for the offset tables first.
    // K-split partials address the workspace and skip them.
    constexpr bool CO = COM != 0;
    static_assert(COM != 2 || (PREC == kBF3 && BN <= BM), "row tails hold 2 BM offsets");
    auto coff = [&](int i) -> int64_t & {
        if constexpr (COM == 2)
            return reinterpret_cast<int64_t *>(smem + (i >> 1) * (Cfg::LA::kLd * 2) + BK * 2)[i & 1];
        else
            return reinterpret_cast<int64_t *>(smem + Cfg::kLdsBytes)[i];
    };
    int64_t myCOff = 0;
    if constexpr (CO) {
        if (!p.ws) {
            if (t < BM) {
                if (m0 + t < p.M) myCOff = p.offCM[m0 + t];
            } else if (t < BM + BN) {
                if (n0 + t - BM < p.N) myCOff = p.offCN[n0 + t - BM];
            }
        }
    }
    auto put_coffs = [&]() {
        if constexpr (CO) {
            if (t < BM + BN) coff(t) = myCOff;
        }
    };

    Gather<PREC, BM, BK, AFK, O32> ga;
    Gather<PREC, BN, BK, BFK, O32> gb;
    const T *__restrict__ A = static_cast<const T *>(pA);
    const T *__restrict__ B = static_cast<const T *>(pB);
#ifdef GETT_ADDR_CHECK
    ga.init(A, t, m0, p.M, p.offAM, BM, p.aLo, p.aSpan);
    gb.init(B, t, n0, p.N, p.offBN, p.bBoxX, p.bLo, p.bSpan);
#else
    ga.init(A, t, m0, p.M, p.offAM, BM, p.aLo);
    gb.init(B, t, n0, p.N, p.offBN, p.bBoxX, p.bLo);
#endif

    Acc acc[FM][FN];
    Acc acx[kTwoAcc ? FM : 1][kTwoAcc ? FN : 1];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            acc[i][j] = Acc{};
            if constexpr (kTwoAcc) acx[i][j] = Acc{};
        }

    T va[Gather<PREC, BM, BK, AFK, O32>::PER];
    T vb[Gather<PREC, BN, BK, BFK, O32>::PER];

    auto stageA = [&](int buf) { return smem + buf * Cfg::kStageBytes; };
    auto stageB = [&](int buf) { return smem + buf * Cfg::kStageBytes + Cfg::LA::kBytes; };

    // The K loop is branch-free.  Steps are aligned to end at kend, so only
    // the leading steps can be partial (their positions below kbeg read
    // zeros) and every step inside the loop is whole.  Each step loads the
    // values DEPTH steps ahead and the offsets of the step after those; the
    // last steps' loads read past kend, which is in bounds: the contracted
    // tables carry zero padding past K (offset 0, i.e. a valid element) and
    // a split slice that ends below K reads real positions of the next
    // slice.  The values are never used.  A loop without branches lets the
    // accumulators live in the MFMA registers throughout.
    constexpr int DEPTH = tile_depth(PREC, BM, BN, BK);
    static_assert(DEPTH == 1 || (DEPTH == 2 && !kCplx), "load depth (complex tiles use 1)");
    int64_t nsteps = (kend - kbeg + BK - 1) / BK;
    if constexpr (DEPTH == 2) nsteps += nsteps & 1;   // pairs of steps (one may be all zeros)
    const int64_t kfirst = kend - nsteps * BK;       // may lie below kbeg (and below 0)

    if constexpr (DEPTH == 1) {
        ga.load_koffs_from(p.offAK, kfirst, kbeg);
        gb.load_koffs_from(p.offBK, kfirst, kbeg);
        ga.template load<true>(kfirst, kbeg, va);
        gb.template load<true>(kfirst, kbeg, vb);
        ga.load_koffs(p.offAK, kfirst + BK);          // kfirst + BK > kbeg
        gb.load_koffs(p.offBK, kfirst + BK);
        ga.store(stageA(0), va);
        gb.store(stageB(0), vb);
        put_coffs();
        __syncthreads();

        // One K step: issue the next step's loads first (they land while the
        // MFMAs run), compute on the current LDS stage, then stage the loaded
        // values and synchronise.
        for (int64_t s = 0; s < nsteps; ++s) {
            const int cur = static_cast<int>(s & 1);
            const int64_t k1 = kfirst + (s + 1) * BK;
            ga.template load<false>(k1, kbeg, va);
            gb.template load<false>(k1, kbeg, vb);
            ga.load_koffs(p.offAK, k1 + BK);
            gb.load_koffs(p.offBK, k1 + BK);
            if constexpr (O32 || tile_load_fence(PREC, BM, BN, BK)) __builtin_amdgcn_sched_barrier(0);
            if constexpr (kCplx) {
                // (ar + i ai)(br + i bi): re += ar br - ai bi, im += ar bi + ai br,
                // four real MFMAs per fragment and k step.
                const R *sa = reinterpret_cast<const R *>(stageA(cur));
                const R *sb = reinterpret_cast<const R *>(stageB(cur));
#pragma unroll
                for (int ks = 0; ks < BK / 4; ++ks) {
                    const int kr = ks * 4 + (lane >> 4);
                    R ar[FM], ai[FM], br[FN], bi[FN];
#pragma unroll
                    for (int i = 0; i < FM; ++i) {
                        const int o = kr * Cfg::LA::kLd + wm * Cfg::WTM + i * 16 + (lane & 15);
                        ar[i] = sa[o];
                        ai[i] = sa[Cfg::LA::kPlane + o];
                    }
#pragma unroll
                    for (int j = 0; j < FN; ++j) {
                        const int o = kr * Cfg::LB::kLd + wn * Cfg::WTN + j * 16 + (lane & 15);
                        br[j] = sb[o];
                        bi[j] = sb[Cfg::LB::kPlane + o];
                    }
#pragma unroll
                    for (int i = 0; i < FM; ++i) {
                        const R nai = -ai[i];
#pragma unroll
                        for (int j = 0; j < FN; ++j) {
                            if constexpr (PREC == kZ64) {
                                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], acc[i][j], 0, 0, 0);
                                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai, bi[j], acc[i][j], 0, 0, 0);
                                acx[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], acx[i][j], 0, 0, 0);
                                acx[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], acx[i][j], 0, 0, 0);
                            } else {
                                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], br[j], acc[i][j], 0, 0, 0);
                                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(nai, bi[j], acc[i][j], 0, 0, 0);
                                acx[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], bi[j], acx[i][j], 0, 0, 0);
                                acx[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[i], br[j], acx[i][j], 0, 0, 0);
                            }
                        }
                    }
                }
            } else if constexpr (!kSplit) {
                const T *sa = reinterpret_cast<const T *>(stageA(cur));
                const T *sb = reinterpret_cast<const T *>(stageB(cur));
#pragma unroll
                for (int ks = 0; ks < BK / 4; ++ks) {
                    const int kr = ks * 4 + (lane >> 4);
                    T a[FM], b[FN];
#pragma unroll
                    for (int i = 0; i < FM; ++i)
                        a[i] = sa[kr * Cfg::LA::kLd + wm * Cfg::WTM + i * 16 + (lane & 15)];
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        b[j] = sb[kr * Cfg::LB::kLd + wn * Cfg::WTN + j * 16 + (lane & 15)];
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j) {
                            if constexpr (PREC == kF64)
                                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
                            else
                                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
                        }
                }
            } else {
                const __bf16 *ahi = reinterpret_cast<const __bf16 *>(stageA(cur));
                const __bf16 *alo = ahi + BM * Cfg::LA::kLd;
                const __bf16 *bhi = reinterpret_cast<const __bf16 *>(stageB(cur));
                const __bf16 *blo = bhi + BN * Cfg::LB::kLd;
#pragma unroll
                for (int ks = 0; ks < BK / 32; ++ks) {
                    const int kc = ks * 32 + 8 * (lane >> 4);
                    bf8_t ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
                    for (int i = 0; i < FM; ++i) {
                        const int r = wm * Cfg::WTM + i * 16 + (lane & 15);
                        ah[i] = *reinterpret_cast<const bf8_t *>(ahi + r * Cfg::LA::kLd + kc);
                        al[i] = *reinterpret_cast<const bf8_t *>(alo + r * Cfg::LA::kLd + kc);
                    }
#pragma unroll
                    for (int j = 0; j < FN; ++j) {
                        const int r = wn * Cfg::WTN + j * 16 + (lane & 15);
                        bh[j] = *reinterpret_cast<const bf8_t *>(bhi + r * Cfg::LB::kLd + kc);
                        bl[j] = *reinterpret_cast<const bf8_t *>(blo + r * Cfg::LB::kLd + kc);
                    }
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j) {
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                        }
                }
            }
            ga.store(stageA(cur ^ 1), va);
            gb.store(stageB(cur ^ 1), vb);
            __syncthreads();
        }
    } else {
        // Two register sets: set h holds the values of the steps s with
        // s % 2 == h.  Step s loads step s + 2 into set s % 2 (staged into
        // LDS one step earlier), computes on its LDS stage, then stages set
        // (s + 1) % 2, loaded a whole step before, into the other LDS stage.
        // Loads complete in issue order, so each step requests the offsets
        // of step s + 3 before the values of step s + 2 (those use a copy of
        // the offsets already held): the next step then waits for its
        // offsets without waiting for values it needs only a step later.
        using GA = Gather<PREC, BM, BK, AFK, O32>;
        using GB = Gather<PREC, BN, BK, BFK, O32>;
        T va2[GA::PER];
        T vb2[GB::PER];
        int64_t koa[GA::NK], kob[GB::NK];
        ga.load_koffs_from(p.offAK, kfirst, kbeg);
        gb.load_koffs_from(p.offBK, kfirst, kbeg);
        ga.template load<true>(kfirst, kbeg, va);
        gb.template load<true>(kfirst, kbeg, vb);
        ga.load_koffs_from(p.offAK, kfirst + BK, kbeg);
        gb.load_koffs_from(p.offBK, kfirst + BK, kbeg);
#pragma unroll
        for (int e = 0; e < GA::NK; ++e) koa[e] = ga.koff[e];
#pragma unroll
        for (int e = 0; e < GB::NK; ++e) kob[e] = gb.koff[e];
        ga.load_koffs(p.offAK, kfirst + 2 * BK);      // kfirst + 2 BK > kbeg
        gb.load_koffs(p.offBK, kfirst + 2 * BK);
        ga.template load_with<true>(koa, kfirst + BK, kbeg, va2);
        gb.template load_with<true>(kob, kfirst + BK, kbeg, vb2);
        ga.store(stageA(0), va);
        gb.store(stageB(0), vb);
        put_coffs();
        __syncthreads();

        for (int64_t s = 0; s < nsteps; s += 2) {
            // even step: LDS stage 0 computed, set 1 staged into stage 1
            const int64_t k2 = kfirst + (s + 2) * BK;
#pragma unroll
            for (int e = 0; e < GA::NK; ++e) koa[e] = ga.koff[e];
#pragma unroll
            for (int e = 0; e < GB::NK; ++e) kob[e] = gb.koff[e];
            ga.load_koffs(p.offAK, k2 + BK);
            gb.load_koffs(p.offBK, k2 + BK);
            __builtin_amdgcn_sched_barrier(0);
            ga.template load_with<false>(koa, k2, kbeg, va);
            gb.template load_with<false>(kob, k2, kbeg, vb);
            if constexpr (O32 || tile_load_fence(PREC, BM, BN, BK)) __builtin_amdgcn_sched_barrier(0);
            if constexpr (kSplit) mma_stage_split<BM, BN, BK>(acc, stageA(0), stageB(0), lane, wm, wn);
            else mma_stage<PREC, BM, BN, BK>(acc, stageA(0), stageB(0), lane, wm, wn);
            ga.store(stageA(1), va2);
            gb.store(stageB(1), vb2);
            __syncthreads();
            // odd step: LDS stage 1 computed, set 0 staged into stage 0
            const int64_t k3 = k2 + BK;
#pragma unroll
            for (int e = 0; e < GA::NK; ++e) koa[e] = ga.koff[e];
#pragma unroll
            for (int e = 0; e < GB::NK; ++e) kob[e] = gb.koff[e];
            ga.load_koffs(p.offAK, k3 + BK);
            gb.load_koffs(p.offBK, k3 + BK);
            __builtin_amdgcn_sched_barrier(0);
            ga.template load_with<false>(koa, k3, kbeg, va2);
            gb.template load_with<false>(kob, k3, kbeg, vb2);
            if constexpr (O32 || tile_load_fence(PREC, BM, BN, BK)) __builtin_amdgcn_sched_barrier(0);
            if constexpr (kSplit) mma_stage_split<BM, BN, BK>(acc, stageA(1), stageB(1), lane, wm, wn);
            else mma_stage<PREC, BM, BN, BK>(acc, stageA(1), stageB(1), lane, wm, wn);
            ga.store(stageA(0), va);
            gb.store(stageB(0), vb);
            __syncthreads();
        }
    }

    // Epilogue.  Fragment (i, j), register v of lane l holds D[row][l%16]
    // (row = M position, column = N position) with row = 4*(l/16) + v for
    // the FP32 and BF16 MFMA but row = l/16 + 4*v for the FP64 MFMA.
    // C <- alpha * sum + beta * C_in; C_in is not read when beta is zero.
    T *__restrict__ Cp = static_cast<T *>(pC);
    const bool rdC = p.beta[0] != 0.0 || p.beta[1] != 0.0;
    constexpr bool kF64Layout = PREC == kF64 || PREC == kZ64;
    if (p.ws) {
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int64_t n = n0 + wn * Cfg::WTN + j * 16 + (lane & 15);
            const bool nok = n < p.N;
#pragma unroll
            for (int i = 0; i < FM; ++i) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rr = kF64Layout ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
                    const int64_t m = m0 + wm * Cfg::WTM + i * 16 + rr;
                    if (!(nok && m < p.M)) continue;
                    const int64_t w = ((int64_t)split * p.M + m) * p.N + n;
                    if constexpr (kCplx) {
                        p.ws[2 * w] = (double)acc[i][j][v];
                        p.ws[2 * w + 1] = (double)acx[i][j][v];
                    } else {
                        p.ws[w] = (double)acc[i][j][v];
                    }
                }
            }
        }
        return;
    }
    // A group of EG fragments of one column at a time, its C_in read before
    // any of it is written: the loads are in flight together (a store to C
    // could alias a later load of C, so loads interleaved with stores wait
    // out one another).  Groups are small enough to leave the tiles'
    // register counts (and so their occupancy) as they are.
    constexpr int EG = 1;
    static_assert(FM % EG == 0, "whole groups");
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int nl = wn * Cfg::WTN + j * 16 + (lane & 15);
        const int64_t n = n0 + nl;
        const bool nok = n < p.N;
        const int64_t ocn = CO ? coff(BM + nl) : p.offCN[n];
#pragma unroll
        for (int i0 = 0; i0 < FM; i0 += EG) {
            int64_t off[EG][4];
            bool ok[EG][4];
            T cin[EG][4];
#pragma unroll
            for (int e = 0; e < EG; ++e) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rr = kF64Layout ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
                    const int ml = wm * Cfg::WTM + (i0 + e) * 16 + rr;
                    const int64_t m = m0 + ml;
                    ok[e][v] = nok && m < p.M;
                    off[e][v] = ok[e][v] ? (CO ? coff(ml) : p.offCM[m]) + ocn : 0;
#ifdef GETT_ADDR_CHECK
                    if (ok[e][v]) ok[e][v] = gett_check_c(off[e][v], p.cLo, p.cSpan);
#endif
                    cin[e][v] = (rdC && ok[e][v]) ? Cp[off[e][v]] : T{};
                }
            }
#pragma unroll
            for (int e = 0; e < EG; ++e) {
                const int i = i0 + e;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if (!ok[e][v]) continue;
                    const int64_t o = off[e][v];
                    if constexpr (PREC == kF64) {
                        const double r = acc[i][j][v];
                        Cp[o] = rdC ? p.beta[0] * cin[e][v] + p.alpha[0] * r : p.alpha[0] * r;
                    } else if constexpr (PREC == kF32) {
                        const float r = acc[i][j][v];
                        const float al = (float)p.alpha[0], be = (float)p.beta[0];
                        Cp[o] = rdC ? be * cin[e][v] + al * r : al * r;
                    } else if constexpr (PREC == kBF3) {
                        const double sum = (double)acc[i][j][v];
                        Cp[o] = (float)(rdC ? p.alpha[0] * sum + p.beta[0] * (double)cin[e][v]
                                            : p.alpha[0] * sum);
                    } else {
                        const R xr = acc[i][j][v], xi = acx[i][j][v];
                        const R ar = (R)p.alpha[0], ai = (R)p.alpha[1];
                        R outr = ar * xr - ai * xi, outi = ar * xi + ai * xr;
                        if (rdC) {
                            const T c = cin[e][v];
                            const R br = (R)p.beta[0], bi = (R)p.beta[1];
                            outr += br * c.x - bi * c.y;
                            outi += br * c.y + bi * c.x;
                        }
                        Cp[o] = T{outr, outi};
                    }
                }
            }
        }
    }
}

template <int PREC, int BM, int BN, int BK, bool AFK, bool BFK, bool O32>
__global__ __launch_bounds__(kThreads) void gett_tile_kernel(TileParams p) {
    extern __shared__ __align__(16) unsigned char smem[];
    using T = typename PrecT<PREC>::T;
    const int tiles = p.tilesM * p.tilesN;
    const int perH = tiles * p.splits;
    const int total = perH * p.H;
    const int logical = xcd_remap(blockIdx.x, total);
    // Hadamard position h (every tile and K slice runs once per position):
    // A, B and C move to that position's base offsets.
    const int h = logical / perH;
    const int rest = logical - h * perH;
    const int split = rest / tiles;
    int tm, tn;
    tile_coords(rest - split * tiles, p.tilesM, p.tilesN, tm, tn);
    const int64_t kbeg = (int64_t)split * p.kPerSplit;
    int64_t kend = kbeg + p.kPerSplit;
    if (kend > p.K) kend = p.K;
    const T *A = static_cast<const T *>(p.A);
    const T *B = static_cast<const T *>(p.B);
    T *C = static_cast<T *>(p.C);
    if (p.H > 1) {
        A += p.offAH[h];
        B += p.offBH[h];
        C += p.offCH[h];
    }
    gett_tile<PREC, BM, BN, BK, AFK, BFK, O32, TileCfg<PREC, BM, BN, BK>::kCOffMode>(
        p, A, B, C, (int64_t)tm * BM, (int64_t)tn * BN,
                                               kbeg, kend, h * p.splits + split, smem);
}

// C[off(m,n)] from the FP64 partials ws[h][s][m][n] of the K slices s, in
// slice order: C_in + p_0 + p_1 + ... (the paper's accumulate) when alpha =
// beta = 1, otherwise alpha * (p_0 + p_1 + ...) + beta * C_in (C_in not read
// when beta = 0); complex partials are (re, im) pairs.
template <int PREC>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(TileParams p) {
    using T = typename PrecT<PREC>::T;
    using R = typename PrecT<PREC>::R;
    const int64_t MN = p.M * p.N;
    const int64_t total = MN * p.H;
    T *Cp = static_cast<T *>(p.C);
    const bool plain = p.alpha[0] == 1.0 && p.alpha[1] == 0.0 && p.beta[0] == 1.0 &&
                       p.beta[1] == 0.0;
    const bool rdC = p.beta[0] != 0.0 || p.beta[1] != 0.0;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t h = idx / MN, r = idx - h * MN;
        const int64_t m = r / p.N, n = r - m * p.N;
        const int64_t off = p.offCM[m] + p.offCN[n];
        GETT_CHECK_C(off, p);
        const int64_t hoff = p.H > 1 ? p.offCH[h] : 0;
        const double *ws = p.ws + (prec_complex(PREC) ? 2 : 1) * (h * p.splits * MN + r);
        if constexpr (prec_complex(PREC)) {
            double sr = 0.0, si = 0.0;
            if (plain) {
                sr = (double)Cp[hoff + off].x;
                si = (double)Cp[hoff + off].y;
            }
            for (int z = 0; z < p.splits; ++z) {
                sr += ws[2 * (int64_t)z * MN];
                si += ws[2 * (int64_t)z * MN + 1];
            }
            if (!plain) {
                double outr = p.alpha[0] * sr - p.alpha[1] * si;
                double outi = p.alpha[0] * si + p.alpha[1] * sr;
                if (rdC) {
                    const double cr = (double)Cp[hoff + off].x, ci = (double)Cp[hoff + off].y;
                    outr += p.beta[0] * cr - p.beta[1] * ci;
                    outi += p.beta[0] * ci + p.beta[1] * cr;
                }
                sr = outr;
                si = outi;
            }
            Cp[hoff + off] = T{(R)sr, (R)si};
        } else {
            double s = plain ? (double)Cp[hoff + off] : 0.0;
            for (int z = 0; z < p.splits; ++z) s += ws[(int64_t)z * MN];
            if (!plain) s = rdC ? p.alpha[0] * s + p.beta[0] * (double)Cp[hoff + off] : p.alpha[0] * s;
            Cp[hoff + off] = (T)s;
        }
    }
}

// ---------------------------------------------------------------------------
// Batched launch: one persistent grid walks a work list of (problem, tile,
// K slice) items, longest first, each workgroup taking the next unclaimed
// item from a counter (so one that drew long items takes fewer); every item
// runs the same tile code as a single call.  Each problem's descriptor says
// which of the batch tiles it runs (its own schedule) and which operands
// read along K, and a uniform switch picks the matching compiled variant.
// ---------------------------------------------------------------------------
template <int PREC, int TS>
__device__ __forceinline__ void batch_item(const TileParams &p, int aFastK, int bFastK, int tile,
                                           unsigned char *smem) {
    constexpr TileShape ts = kTiles[PREC][kBatchTile[PREC][TS]];
    // A problem cut along K numbers its items slice-major: slice z covers
    // [z kPerSplit, min(K, (z+1) kPerSplit)) and writes FP64 partials.
    const int32_t tilesMN = p.tilesM * p.tilesN;
    const int32_t split = tile / tilesMN;
    int tm, tn;
    tile_coords(tile - split * tilesMN, p.tilesM, p.tilesN, tm, tn);
    const int64_t m0 = (int64_t)tm * ts.bm, n0 = (int64_t)tn * ts.bn;
    const int64_t kbeg = (int64_t)split * p.kPerSplit;
    const int64_t kend = min(p.K, kbeg + p.kPerSplit);
    const int variant = aFastK * 2 + bFastK;
    if (variant == 0)
        gett_tile<PREC, ts.bm, ts.bn, ts.bk, false, false, false, BatchLds<PREC>::kCOff ? 1 : 0>(
            p, p.A, p.B, p.C, m0, n0, kbeg, kend, split, smem);
    else if (variant == 1)
        gett_tile<PREC, ts.bm, ts.bn, ts.bk, false, true, false, BatchLds<PREC>::kCOff ? 1 : 0>(
            p, p.A, p.B, p.C, m0, n0, kbeg, kend, split, smem);
    else if (variant == 2)
        gett_tile<PREC, ts.bm, ts.bn, ts.bk, true, false, false, BatchLds<PREC>::kCOff ? 1 : 0>(
            p, p.A, p.B, p.C, m0, n0, kbeg, kend, split, smem);
    else
        gett_tile<PREC, ts.bm, ts.bn, ts.bk, true, true, false, BatchLds<PREC>::kCOff ? 1 : 0>(
            p, p.A, p.B, p.C, m0, n0, kbeg, kend, split, smem);
}

template <int PREC>
__global__ __launch_bounds__(kThreads) void gett_batch_kernel(const BatchProblem *__restrict__ probs,
                                                              const int32_t *__restrict__ items,
                                                              int32_t nitems, int32_t *next) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t s_item;
    // *next starts at 0 (the launch's descriptor copy clears it); every
    // workgroup leaves once the count has passed the last item.
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(next, 1);
        __syncthreads();
        const int32_t it = s_item;
        if (it >= nitems) break;
        const int32_t pi = items[2 * it];
        const int32_t tile = items[2 * it + 1];
        const BatchProblem &bp = probs[pi];
        const TileParams p = bp.p;
        if (bp.tsel == 0)
            batch_item<PREC, 0>(p, bp.aFastK, bp.bFastK, tile, smem);
        else
            batch_item<PREC, 1>(p, bp.aFastK, bp.bFastK, tile, smem);
        __syncthreads();   // the next item reuses the LDS stages and s_item
    }
}

// The batch's problems cut along K: C = C_in + sum of the slices' partials in
// slice order, in FP64 (the descriptors are read on the device, so a graph
// replay with new pointers reduces into the new C).
template <int PREC>
__global__ __launch_bounds__(256) void batch_reduce_kernel(const BatchProblem *__restrict__ probs,
                                                           const int32_t *__restrict__ list,
                                                           int32_t n) {
    using T = typename PrecT<PREC>::T;
    for (int32_t li = blockIdx.y; li < n; li += gridDim.y) {
        const TileParams &p = probs[list[li]].p;
        const int64_t MN = p.M * p.N;
        T *Cp = static_cast<T *>(p.C);
        for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < MN;
             idx += (int64_t)gridDim.x * blockDim.x) {
            const int64_t m = idx / p.N, nn = idx - m * p.N;
            const int64_t off = p.offCM[m] + p.offCN[nn];
            GETT_CHECK_C(off, p);
            double s = (double)Cp[off];
            for (int z = 0; z < p.splits; ++z) s += p.ws[(int64_t)z * MN + idx];
            Cp[off] = (T)s;
        }
    }
}

// Host-side launch helpers (instantiated per precision in its own file).
template <int PREC, int BM, int BN, int BK, bool AFK, bool BFK, bool O32>
static int launch_one(const TileParams &p, hipStream_t s) {
    using Cfg = TileCfg<PREC, BM, BN, BK>;
    auto kern = gett_tile_kernel<PREC, BM, BN, BK, AFK, BFK, O32>;
    static bool attr_set = false;   // per instantiation; LDS above 64 KB needs opting in
    if (!attr_set) {
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                Cfg::kLaunchLds) != hipSuccess)
            return GETT_ERR_HIP;
        attr_set = true;
    }
    const int total = p.tilesM * p.tilesN * p.splits * p.H;
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    hipLaunchKernelGGL(kern, dim3(total), dim3(kThreads), Cfg::kLaunchLds, s, p);
    return launch_status();
}

template <int PREC, int BM, int BN, int BK, bool O32>
static int launch_fast_o(bool afk, bool bfk, const TileParams &p, hipStream_t s) {
    if (afk) {
        if (bfk) return launch_one<PREC, BM, BN, BK, true, true, O32>(p, s);
        return launch_one<PREC, BM, BN, BK, true, false, O32>(p, s);
    }
    if (bfk) return launch_one<PREC, BM, BN, BK, false, true, O32>(p, s);
    return launch_one<PREC, BM, BN, BK, false, false, O32>(p, s);
}

// Tiles marked addr32 in the menu take the 32-bit addressing variant when
// both operands' spans allow it (real precisions).
template <int PREC, int BM, int BN, int BK>
static int launch_fast(bool afk, bool bfk, const TileParams &p, hipStream_t s) {
    if constexpr (tile_addr32(PREC, BM, BN, BK)) {
        if (p.off32) return launch_fast_o<PREC, BM, BN, BK, true>(afk, bfk, p, s);
    }
    return launch_fast_o<PREC, BM, BN, BK, false>(afk, bfk, p, s);
}

template <int PREC>
static int launch_prec(int tile, bool afk, bool bfk, const TileParams &p, hipStream_t s) {
    constexpr TileShape t0 = kTiles[PREC][0], t1 = kTiles[PREC][1], t2 = kTiles[PREC][2],
                        t3 = kTiles[PREC][3], t4 = kTiles[PREC][4];
    // packed entries run their own kernels (never through here)
    switch (tile) {
    case 0: if constexpr (!t0.packed) return launch_fast<PREC, t0.bm, t0.bn, t0.bk>(afk, bfk, p, s); break;
    case 1: if constexpr (!t1.packed) return launch_fast<PREC, t1.bm, t1.bn, t1.bk>(afk, bfk, p, s); break;
    case 2: if constexpr (!t2.packed) return launch_fast<PREC, t2.bm, t2.bn, t2.bk>(afk, bfk, p, s); break;
    case 3: if constexpr (!t3.packed) return launch_fast<PREC, t3.bm, t3.bn, t3.bk>(afk, bfk, p, s); break;
    case 4: if constexpr (!t4.packed) return launch_fast<PREC, t4.bm, t4.bn, t4.bk>(afk, bfk, p, s); break;
    default: break;
    }
    return GETT_ERR_INTERNAL;
}

template <int PREC> static int batch_lds() { return BatchLds<PREC>::kBytes; }

template <int PREC> static int launch_splitk_reduce_prec(const TileParams &p, hipStream_t s) {
    const int64_t MN = p.M * p.N * p.H;
    int64_t blocks = (MN + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    hipLaunchKernelGGL(splitk_reduce_kernel<PREC>, dim3(blocks), dim3(256), 0, s, p);
    return launch_status();
}

template <int PREC> static int batch_grid_size_prec() {
    int dev = 0, cus = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, gett_batch_kernel<PREC>, kThreads,
                                                     batch_lds<PREC>()) != hipSuccess || occ < 1)
        occ = 1;
    return cus * occ;
}

template <int PREC>
static int launch_batch_prec(const BatchProblem *d_probs, const int32_t *d_items, int32_t nitems,
                             int32_t *d_next, int32_t grid, hipStream_t s) {
    if (grid < 1 || nitems < 1) return 0;
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    hipLaunchKernelGGL(gett_batch_kernel<PREC>, dim3(grid), dim3(kThreads), batch_lds<PREC>(), s,
                       d_probs, d_items, nitems, d_next);
    return launch_status();
}

template <int PREC>
static int launch_batch_reduce_prec(const BatchProblem *d_probs, const int32_t *d_list, int32_t n,
                                    hipStream_t s) {
    if (n < 1) return 0;
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    hipLaunchKernelGGL(batch_reduce_kernel<PREC>, dim3(64, (unsigned)min(n, 65535)), dim3(256), 0,
                       s, d_probs, d_list, n);
    return launch_status();
}

// Out-of-range accesses counted by this file's kernels on the current device
// (checked build; -1 otherwise).
static int64_t addr_violations_here(bool reset) {
#ifdef GETT_ADDR_CHECK
    unsigned long long v = 0;
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_gett_viol), sizeof v) != hipSuccess)
        return -1;
    if (reset) {
        const unsigned long long z = 0;
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_gett_viol), &z, sizeof z) != hipSuccess) return -1;
    }
    return (int64_t)v;
#else
    (void)reset;
    return -1;
#endif
}

// Defines the per-precision entry points used by the host dispatcher.
#define GETT_DEFINE_PRECISION(PREC, SUFFIX)                                                        \
    int launch_tile_##SUFFIX(int tile, bool afk, bool bfk, const TileParams &p, hipStream_t s) {   \
        return launch_prec<PREC>(tile, afk, bfk, p, s);                                            \
    }                                                                                              \
    int launch_splitk_reduce_##SUFFIX(const TileParams &p, hipStream_t s) {                       \
        return launch_splitk_reduce_prec<PREC>(p, s);                                              \
    }                                                                                              \
    int batch_grid_size_##SUFFIX() { return batch_grid_size_prec<PREC>(); }                        \
    int launch_batch_##SUFFIX(const BatchProblem *d, const int32_t *it, int32_t n, int32_t *nx,    \
                              int32_t g, hipStream_t s) {                                          \
        return launch_batch_prec<PREC>(d, it, n, nx, g, s);                                        \
    }                                                                                              \
    int launch_batch_reduce_##SUFFIX(const BatchProblem *d, const int32_t *l, int32_t n,           \
                                     hipStream_t s) {                                              \
        return launch_batch_reduce_prec<PREC>(d, l, n, s);                                         \
    }                                                                                              \
    int64_t addr_violations_##SUFFIX(bool reset) { return addr_violations_here(reset); }

// The same for precisions without a batched entry point (complex data).
#define GETT_DEFINE_TILE_PRECISION(PREC, SUFFIX)                                                   \
    int launch_tile_##SUFFIX(int tile, bool afk, bool bfk, const TileParams &p, hipStream_t s) {   \
        return launch_prec<PREC>(tile, afk, bfk, p, s);                                            \
    }                                                                                              \
    int launch_splitk_reduce_##SUFFIX(const TileParams &p, hipStream_t s) {                       \
        return launch_splitk_reduce_prec<PREC>(p, s);                                              \
    }                                                                                              \
    int64_t addr_violations_##SUFFIX(bool reset) { return addr_violations_here(reset); }

}  // namespace gett
