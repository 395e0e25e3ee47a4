// gett_ozaki.hip -- DGETT emulated on the INT8 matrix cores (the Ozaki
// scheme: Ozaki, Ogita, Oishi and Rump 2012; its INT8 form, Ootomo, Ozaki
// and Yokota 2024).
//
// exponent: every row of A and of B (canonical rows, contracted positions
//        by the offset tables) gets the binary exponent e of its largest
//        magnitude (frexp convention: max = f 2^e, f in [0.5, 1)), by an
//        integer atomic maximum over partial maxima; all-zero rows keep the
//        fill value (their products are zero whatever their exponent).
// slice: each value x of a row becomes S 7-bit slices by truncation:
//        x <- x 2^-e; for s = 1 .. S: x <- 128 x, q_s = trunc(x), x <- x - q_s
//        (exact in double, |q_s| <= 127).  Slice s of an operand is a plane
//        of int8 in 1 KB blocks of 16 rows by 64 positions (rows of 64 bytes:
//        the 16-byte piece lane l of the 16x16x64 INT8 MFMA reads is row
//        l % 16, positions 16 (l / 16) .. + 15), positions stored in the same
//        fixed permutation for both operands as the other packed forms.
// gemm:  a 64 x 64 tile, 8 waves as 2 x 4, each 32 x 16.  For every d = s + t
//        (2 .. S + 1) one INT32 accumulator set sums the slice pairs (s, t)
//        over the tile's positions -- exact: at most S pairs of at most 16384
//        positions of 127^2, under 2^31 -- with the S A-slices of a step
//        staged through LDS and each wave's B-slice fragments loaded straight
//        into registers.  The epilogue combines in double, from
//        the smallest scale up: v = sum over d = S+1 .. 2 of
//        ldexp(P_d, eA + eB - 7 d), then C <- C_in + v (one K slice) or the
//        FP64 partial v (several K slices, reduced afterwards).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gett_grid.h"
#include "gett_internal.h"
#include "gett_ozaki.h"

namespace gett {

namespace {

typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef uint32_t u2_t __attribute__((ext_vector_type(2)));

constexpr int kNoExp = -2147483647 - 1;   // fill value: no nonzero value seen

// Position of element e of chunk c (8 packed positions) in the groups of 512
// (the permutation the other packed forms use).
__device__ __forceinline__ int64_t oz_pos(int64_t c, int e, int64_t Kq) {
    const int64_t g = c >> 6;
    const int64_t S = min<int64_t>(512, Kq - 512 * g) >> 3;
    return 512 * g + (c & 63) + S * e;
}

// Byte offset of packed positions j .. j + 7 (j a multiple of 8) of row r.
__device__ __forceinline__ int64_t oz_off(int64_t r, int64_t j, int64_t Kq) {
    return ((r >> 4) * (Kq >> 6) + (j >> 6)) * 1024 + (r & 15) * 64 + (j & 63);
}

__device__ __forceinline__ int oz_exp(double v) {
    int e = 0;
    (void)frexp(v, &e);
    return v != 0.0 ? e : kNoExp;
}

__global__ void oz_fill_kernel(int32_t *__restrict__ E, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) E[i] = kNoExp;
}

// The two loader shapes of the other packed forms: lanes along K (one wave
// per (4 rows, group of 512 positions), lane l holding chunk l of the group)
// or along the rows (one wave per (4 x 16 rows in the operand's memory
// order, 4 chunks), lane l holding row l % 16 and chunk c0 + l / 16).  A
// lane's 8 values of one row are loaded, then handed to OP.
template <class OP>
__device__ __forceinline__ void oz_rows_k(const double *__restrict__ X,
                                          const int64_t *__restrict__ offR, int64_t R,
                                          const int64_t *__restrict__ offK, int64_t K, int64_t Kq,
                                          OP op) {
    const int64_t ng = (Kq + 511) / 512;
    const int64_t nrb = (R + 3) / 4;
    const int64_t task = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (task >= nrb * ng) return;   // whole waves leave together
    const int lane = threadIdx.x & 63;
    const int64_t rb = task / ng, g = task - rb * ng;
    const int64_t S = min<int64_t>(512, Kq - 512 * g) >> 3;
    const bool on = lane < S;
    const int64_t c = 64 * g + lane;
    int64_t ko[8];
    uint32_t valid = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t k = on ? oz_pos(c, e, Kq) : K;
        ko[e] = k < K ? offK[k] : 0;
        valid |= (k < K ? 1u : 0u) << e;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t r = rb * 4 + q;
        if (r >= R) break;   // uniform
        const double *xr = X + offR[r];
        double v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (valid >> e) & 1 ? xr[ko[e]] : 0.0;
        op(r, c, on, v, true);
    }
}

template <class OP>
__device__ __forceinline__ void oz_rows_r(const double *__restrict__ X,
                                          const int64_t *__restrict__ rowsOp,
                                          const int32_t *__restrict__ rowMap, int64_t R,
                                          const int64_t *__restrict__ offK, int64_t K, int64_t Kq,
                                          OP op) {
    const int64_t nc = Kq / 8;
    const int64_t cq = (nc + 3) / 4;
    const int64_t task = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t sb = task / cq, q = task - sb * cq;
    if (sb * 64 >= R) return;       // whole waves leave together
    const int64_t c = q * 4 + (lane >> 4);
    const bool con = c < nc;
    int64_t ko[8];
    uint32_t valid = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t k = con ? oz_pos(c, e, Kq) : K;
        ko[e] = k < K ? offK[k] : 0;
        valid |= (k < K ? 1u : 0u) << e;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t p = (sb * 4 + b) * 16 + (lane & 15);
        const bool on = con && p < R;
        const double *xr = X + (on ? rowsOp[p] : 0);
        double v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (on && ((valid >> e) & 1)) ? xr[ko[e]] : 0.0;
        op(on ? (int64_t)rowMap[p] : -1, c, on, v, false);
    }
}

// Largest exponent of a lane's 8 values, folded into E[r] (one atomic per
// row and wave; the loader along K gives all lanes of a wave the same row).
struct OzExp {
    int32_t *E;
    __device__ __forceinline__ void operator()(int64_t r, int64_t, bool on, const double (&v)[8],
                                               bool along_k) const {
        int e = kNoExp;
#pragma unroll
        for (int i = 0; i < 8; ++i) e = max(e, oz_exp(v[i]));
        (void)along_k;
        if (!on) e = kNoExp;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) e = max(e, __shfl_xor(e, o));
        if ((threadIdx.x & 63) == 0 && e != kNoExp) atomicMax(E + r, e);
    }
};

template <int S> struct OzSlice {
    const int32_t *E;
    uint8_t *P;           // plane 0; plane s at + s * plane bytes
    int64_t plane, Kq;
    __device__ __forceinline__ void operator()(int64_t r, int64_t c, bool on, const double (&v)[8],
                                               bool) const {
        if (!on) return;
        const int e0 = E[r];
        const int e = e0 == kNoExp ? 0 : e0;
        uint32_t w[S][2];
#pragma unroll
        for (int s = 0; s < S; ++s) w[s][0] = w[s][1] = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            double x = ldexp(v[i], -e);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                x *= 128.0;
                const double q = trunc(x);
                x -= q;
                w[s][i >> 2] |= ((uint32_t)(uint8_t)(int8_t)(int)q) << (8 * (i & 3));
            }
        }
        uint8_t *dst = P + oz_off(r, 8 * c, Kq);
#pragma unroll
        for (int s = 0; s < S; ++s)
            *reinterpret_cast<u2_t *>(dst + s * plane) = u2_t{w[s][0], w[s][1]};
    }
};

__global__ __launch_bounds__(256) void oz_exp_k_kernel(const double *X, const int64_t *offR,
                                                       int64_t R, const int64_t *offK, int64_t K,
                                                       int64_t Kq, int32_t *E) {
    oz_rows_k(X, offR, R, offK, K, Kq, OzExp{E});
}
// Exponents with lanes along the rows: a workgroup takes 4 x 16 rows and 4
// consecutive quads of chunks, one quad per wave (lane l: row l % 16, chunk
// l / 16 of the quad).  The four lanes of a row combine their maxima by
// shuffles, the four waves theirs through LDS, and one atomic per row and
// workgroup remains (one per row and chunk queued hundreds of atomics on
// each row's word; a loop over a run of quads per wave instead serialised
// its loads and ran slower still).
__global__ __launch_bounds__(256) void oz_exp_r_kernel(const double *__restrict__ X,
                                                       const int64_t *__restrict__ rowsOp,
                                                       const int32_t *__restrict__ rowMap,
                                                       int64_t R,
                                                       const int64_t *__restrict__ offK,
                                                       int64_t K, int64_t Kq,
                                                       int32_t *__restrict__ E) {
    __shared__ int red[4][64];
    const int64_t nc = Kq / 8;
    const int64_t cq = (nc + 3) / 4;
    const int64_t qb = (cq + 3) / 4;                 // quad blocks per 64 rows
    const int64_t blk = blockIdx.x;
    const int64_t sb = blk / qb;
    if (sb * 64 >= R) return;                       // whole workgroups leave together
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t q = (blk - sb * qb) * 4 + w;
    const int64_t c = q * 4 + (lane >> 4);
    const bool con = q < cq && c < nc;
    int64_t ko[8];
    uint32_t valid = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t k = con ? oz_pos(c, e, Kq) : K;
        ko[e] = k < K ? offK[k] : 0;
        valid |= (k < K ? 1u : 0u) << e;
    }
    int em[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t p = (sb * 4 + b) * 16 + (lane & 15);
        const bool on = con && p < R;
        const double *xr = X + (on ? rowsOp[p] : 0);
        int e = kNoExp;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (on && ((valid >> i) & 1)) e = max(e, oz_exp(xr[ko[i]]));
        e = max(e, __shfl_xor(e, 16));
        e = max(e, __shfl_xor(e, 32));
        em[b] = e;
    }
    if (lane < 16) {
#pragma unroll
        for (int b = 0; b < 4; ++b) red[w][b * 16 + lane] = em[b];
    }
    __syncthreads();
    if (w == 0) {
        const int e = max(max(red[0][lane], red[1][lane]), max(red[2][lane], red[3][lane]));
        const int64_t p = (sb * 4 + (lane >> 4)) * 16 + (lane & 15);
        if (p < R && e != kNoExp) atomicMax(E + rowMap[p], e);
    }
}

template <int S>
__global__ __launch_bounds__(256) void oz_slice_k_kernel(const double *X, const int64_t *offR,
                                                         int64_t R, const int64_t *offK, int64_t K,
                                                         int64_t Kq, const int32_t *E, uint8_t *P,
                                                         int64_t plane) {
    oz_rows_k(X, offR, R, offK, K, Kq, OzSlice<S>{E, P, plane, Kq});
}
template <int S>
__global__ __launch_bounds__(256) void oz_slice_r_kernel(const double *X, const int64_t *rowsOp,
                                                         const int32_t *rowMap, int64_t R,
                                                         const int64_t *offK, int64_t K,
                                                         int64_t Kq, const int32_t *E, uint8_t *P,
                                                         int64_t plane) {
    oz_rows_r(X, rowsOp, rowMap, R, offK, K, Kq, OzSlice<S>{E, P, plane, Kq});
}

// LDS rows of 64 bytes (one step of one row of one slice); the four 16-byte
// chunks of row r in the order c ^ swz(r) (bank-conflict free for the
// stores, four threads per row, and for the MFMA reads, 16 rows per chunk).
__device__ __forceinline__ int oz_swz(int r) {
    return ((((r >> 1) ^ (r >> 3)) & 1) << 1) | ((r >> 2) & 1);
}

constexpr int kOzBM = 64, kOzBN = 64, kOzBK = 64;

template <int S>
__global__ __launch_bounds__(512) void oz_gemm_kernel(OzParams g) {
    constexpr int kStage = S * 64 * 64;             // bytes per stage: the S A slices
    constexpr int NP = (S + 1) / 2;                 // staging passes (two planes a pass)
    extern __shared__ __align__(16) uint8_t ozl[];

    const int tiles = g.tilesM * g.tilesN;
    const int logical = xcd_remap(blockIdx.x, tiles * g.splits);
    const int split = logical / tiles;
    int tm, tn;
    tile_coords(logical - split * tiles, g.tilesM, g.tilesN, tm, tn);
    const int64_t m0 = (int64_t)tm * kOzBM, n0 = (int64_t)tn * kOzBN;
    const int64_t kbeg = (int64_t)split * g.kPer;
    const int64_t kend = min(kbeg + g.kPer, g.Kq);
    const int64_t nsteps = (kend - kbeg) / kOzBK;

    const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 2, wn = w & 3;
    // The tile's C offsets and scale exponents (its M rows, then its N
    // positions), requested at kernel start and staged in LDS at the first
    // barrier: the epilogue then waits for C_in alone.  Split-K partials
    // address the workspace directly and take no C offsets.
    __shared__ int64_t sOff[kOzBM + kOzBN];
    __shared__ int sExp[kOzBM + kOzBN];
    int64_t myOff = 0;
    int myExp = 0;
    if (t < kOzBM) {
        const int64_t m = m0 + t;
        if (m < g.M) {
            myExp = max(g.EA[m], -4000);             // all-zero rows: any exponent
            if (!g.ws) myOff = g.offCM[m];
        }
    } else if (t < kOzBM + kOzBN) {
        const int64_t n = n0 + t - kOzBM;
        if (n < g.N) {
            myExp = max(g.EB[n], -4000);
            if (!g.ws) myOff = g.offCN[n];
        }
    }
    // staging of A: thread t moves chunk (t & 3) of row (t >> 2) & 63 of
    // slice plane 2 i + (t >> 8), i < NP (past S in the last pass of odd S:
    // nothing)
    const int srow = (t >> 2) & 63, sc = t & 3, spl = t >> 8;
    const int64_t rgs = g.Kq * 16;                  // bytes from one row group to the next
    const uint32_t goff = (uint32_t)((srow >> 4) * rgs + (srow & 15) * 64 + 16 * sc);
    const uint32_t soff = (uint32_t)(srow * 64 + 16 * (sc ^ oz_swz(srow)));
    // the tile's first row group at the slice's first step; step j at + 1024 j
    const uint8_t *Ab = g.A + m0 * g.Kq + kbeg * 16;
    // B straight from the slice planes: a plane's block of 16 rows x 64
    // positions is one MFMA operand fragment for one step, and lane l's 16
    // bytes are row l % 16, positions 16 (l / 16) .. (the chunk the LDS
    // layout of A hands the same lane)
    const uint8_t *Bw = g.B + (n0 + wn * 16) * g.Kq + kbeg * 16 + (lane & 15) * 64 + 16 * (lane >> 4);

    v4i_t acc[S][2];
#pragma unroll
    for (int d = 0; d < S; ++d)
#pragma unroll
        for (int i = 0; i < 2; ++i) acc[d][i] = v4i_t{0, 0, 0, 0};

    auto stepoff = [&](int64_t s) { return 1024 * (s < nsteps ? s : nsteps - 1); };
    // every thread loads (plane S - 1 again past the last plane, so the loads
    // stay unconditional and countable); only the LDS store is skipped
    auto gload = [&](int64_t s, v4i_t (&v)[NP]) {
        const int64_t st = stepoff(s);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int pl = min(2 * i + spl, S - 1);
            v[i] = *reinterpret_cast<const v4i_t *>(Ab + (int64_t)pl * g.planeA + goff + st);
        }
    };
    auto lstore = [&](uint8_t *stage, const v4i_t (&v)[NP]) {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int pl = 2 * i + spl;
            if (pl < S) *reinterpret_cast<v4i_t *>(stage + pl * 4096 + soff) = v[i];
        }
    };
    auto bload = [&](int tt, int64_t st) {
        return *reinterpret_cast<const v4i_t *>(Bw + (int64_t)tt * g.planeB + st);
    };
    const int kc = 16 * ((lane >> 4) ^ oz_swz(lane & 15));   // rows start at multiples of 16
    // B slices outermost: slice tt's pairs run together, then (behind a
    // scheduling barrier, so its registers are reused) its load for the next
    // step, which uses B slice 0 first and so gives every load about a step
    // to arrive; the A fragments of all slices stay in registers for the step
    auto mma = [&](const uint8_t *stage, v4i_t (&b)[S], int64_t stnext) {
        v4i_t a[S][2];
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[s][i] = *reinterpret_cast<const v4i_t *>(stage + s * 4096 +
                                                           (wm * 32 + i * 16 + (lane & 15)) * 64 + kc);
#pragma unroll
        for (int tt = 0; tt < S; ++tt) {
#pragma unroll
            for (int s = 0; s + tt < S; ++s)       // slices s + 1, tt + 1: d - 2 = s + tt
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    acc[s + tt][i] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[s][i], b[tt], acc[s + tt][i], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
            b[tt] = bload(tt, stnext);
        }
    };

    v4i_t r[NP];
    v4i_t b[S];
    gload(0, r);
#pragma unroll
    for (int tt = 0; tt < S; ++tt) b[tt] = bload(tt, 0);
    lstore(ozl, r);
    if (t < kOzBM + kOzBN) {
        sOff[t] = myOff;
        sExp[t] = myExp;
    }
    __syncthreads();
    for (int64_t s = 0; s < nsteps; ++s) {
        const int cur = (int)(s & 1);
        gload(s + 1, r);
        __builtin_amdgcn_s_setprio(1);
        mma(ozl + cur * kStage, b, stepoff(s + 1));
        __builtin_amdgcn_s_setprio(0);
        __builtin_amdgcn_sched_barrier(0);
        lstore(ozl + (cur ^ 1) * kStage, r);
        __syncthreads();
    }

    // Epilogue: fragment i, register v of lane l holds M row 4 (l / 16) + v
    // and N column l % 16.  Combination in double from the smallest scale up.
    double *__restrict__ C = g.C;
    const int nl = wn * 16 + (lane & 15);
    const int64_t n = n0 + nl;
    const bool nok = n < g.N;
    const int eb = sExp[kOzBM + nl];
    const int64_t ocn = sOff[kOzBM + nl];
    // Every value and C_in of the lane first (one round trip for C_in), then
    // the stores.
    double val[2][4], cin[2][4];
    int64_t off[2][4];
    bool ok[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int ml = wm * 32 + i * 16 + 4 * (lane >> 4) + v;
            const int64_t m = m0 + ml;
            ok[i][v] = nok && m < g.M;
            const int ea = ok[i][v] ? sExp[ml] : 0;
            double x = 0.0;
#pragma unroll
            for (int d = S - 1; d >= 0; --d) x += ldexp((double)acc[d][i][v], ea + eb - 7 * (d + 2));
            val[i][v] = x;
            if (g.ws) {
                if (ok[i][v]) g.ws[((int64_t)split * g.M + m) * g.N + n] = x;
                ok[i][v] = false;
                continue;
            }
            off[i][v] = ok[i][v] ? sOff[ml] + ocn : 0;
            cin[i][v] = ok[i][v] ? C[off[i][v]] : 0.0;
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            if (ok[i][v]) C[off[i][v]] = cin[i][v] + val[i][v];
}

template <int S> int launch_slices(const OzOperand &o, int64_t Kq, uint8_t *P, int64_t plane,
                                   const int32_t *E, hipStream_t s) {
    const int64_t tasks = o.rowsFast ? (o.R + 63) / 64 * ((Kq / 8 + 3) / 4)
                                     : (o.R + 3) / 4 * ((Kq + 511) / 512);
    const int64_t blocks = (tasks + 3) / 4;
    if (blocks > INT32_MAX) return GETT_ERR_INTERNAL;
    if (o.rowsFast)
        hipLaunchKernelGGL(oz_slice_r_kernel<S>, dim3((unsigned)blocks), dim3(256), 0, s, o.X,
                           o.offR, o.rowMap, o.R, o.offK, o.K, Kq, E, P, plane);
    else
        hipLaunchKernelGGL(oz_slice_k_kernel<S>, dim3((unsigned)blocks), dim3(256), 0, s, o.X,
                           o.offR, o.R, o.offK, o.K, Kq, E, P, plane);
    return launch_status();
}

template <int S> int launch_gemm(const OzParams &g, hipStream_t s) {
    constexpr int kLds = 2 * (S * 64 * 64);
    static bool attr_set = false;   // set once per process (every device takes the same value)
    if (!attr_set) {
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(oz_gemm_kernel<S>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kLds) != hipSuccess)
            return GETT_ERR_HIP;
        attr_set = true;
    }
    const int64_t total = (int64_t)g.tilesM * g.tilesN * g.splits;
    if (total > INT32_MAX) return GETT_ERR_INTERNAL;
    auto kern = oz_gemm_kernel<S>;
    hipLaunchKernelGGL(kern, dim3((unsigned)total), dim3(512), kLds, s, g);
    return launch_status();
}

}  // namespace

int launch_oz_exponents(const OzOperand &o, int64_t Kq, int32_t *E, int64_t Epad, hipStream_t s) {
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    hipLaunchKernelGGL(oz_fill_kernel, dim3((unsigned)((Epad + 255) / 256)), dim3(256), 0, s, E,
                       Epad);
    int rc = launch_status();
    if (rc || o.R == 0) return rc;
    // rows: one workgroup per (64 rows, 4 quads of chunks); along K: one wave
    // per (4 rows, group of 512 positions), four waves per workgroup
    const int64_t blocks = o.rowsFast ? (o.R + 63) / 64 * (((Kq / 8 + 3) / 4 + 3) / 4)
                                      : ((o.R + 3) / 4 * ((Kq + 511) / 512) + 3) / 4;
    if (blocks > INT32_MAX) return GETT_ERR_INTERNAL;
    if (o.rowsFast)
        hipLaunchKernelGGL(oz_exp_r_kernel, dim3((unsigned)blocks), dim3(256), 0, s, o.X, o.offR,
                           o.rowMap, o.R, o.offK, o.K, Kq, E);
    else
        hipLaunchKernelGGL(oz_exp_k_kernel, dim3((unsigned)blocks), dim3(256), 0, s, o.X, o.offR,
                           o.R, o.offK, o.K, Kq, E);
    return launch_status();
}

int launch_oz_slices(int S, const OzOperand &o, int64_t Kq, uint8_t *P, int64_t plane,
                     const int32_t *E, hipStream_t s) {
    if (o.R == 0) return 0;
    (void)hipGetLastError();
    switch (S) {
    case 3: return launch_slices<3>(o, Kq, P, plane, E, s);
    case 4: return launch_slices<4>(o, Kq, P, plane, E, s);
    case 5: return launch_slices<5>(o, Kq, P, plane, E, s);
    case 6: return launch_slices<6>(o, Kq, P, plane, E, s);
    case 7: return launch_slices<7>(o, Kq, P, plane, E, s);
    case 8: return launch_slices<8>(o, Kq, P, plane, E, s);
    default: return GETT_ERR_INTERNAL;
    }
}

int launch_oz_gemm(int S, const OzParams &g, hipStream_t s) {
    (void)hipGetLastError();
    switch (S) {
    case 3: return launch_gemm<3>(g, s);
    case 4: return launch_gemm<4>(g, s);
    case 5: return launch_gemm<5>(g, s);
    case 6: return launch_gemm<6>(g, s);
    case 7: return launch_gemm<7>(g, s);
    case 8: return launch_gemm<8>(g, s);
    default: return GETT_ERR_INTERNAL;
    }
}

}  // namespace gett
