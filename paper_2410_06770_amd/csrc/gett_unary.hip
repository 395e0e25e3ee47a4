// gett_unary.hip -- kernels of the unary operations (transpose, reduction,
// trace; Section 9's future work) for gfx950.
//
// Both kernels read each element of A once; sums are formed in FP64 (real
// and imaginary parts separately for complex data) in a fixed order, so the
// result does not depend on the launch.
//   unary_tiled_kernel:   a workgroup owns 64 positions of O1 x 64 of O2 at
//     one O3 position; its lanes run along O1 (A's cheapest output mode), so
//     each of a thread's 16 rows is one coalesced load per summed position;
//     the summed offsets are wave-uniform (scalar loads).  The results go
//     through LDS and are stored with the lanes along O2 (C's cheapest
//     mode), or straight from registers when O1 is C's cheapest mode too.
//     When C has a single output mode (a reduction to a vector), the
//     workgroup's 64 row slots take 64 interleaved summed positions instead,
//     and their sums are added through LDS in slot order.
//   unary_lanes_r_kernel: when A's cheapest mode is a summed one, g lanes
//     share an output and walk the summed positions together (coalesced),
//     each keeping four partial sums (four loads in flight), then add their
//     sums with cross-lane shuffles.
// With S > 1 slices of the summed positions each slice writes an FP64
// partial and unary_finish_kernel adds them in slice order.
#include "gett_internal.h"
#include "gett_unary.h"

namespace gett {

typedef double ud2_t __attribute__((ext_vector_type(2)));
typedef float uf2_t __attribute__((ext_vector_type(2)));

template <int PREC> struct UT;
// T: an element; R: its real type.
template <> struct UT<0> { using T = double; using R = double; static constexpr bool kCplx = false; };
template <> struct UT<1> { using T = float; using R = float; static constexpr bool kCplx = false; };
template <> struct UT<4> { using T = ud2_t; using R = double; static constexpr bool kCplx = true; };
template <> struct UT<5> { using T = uf2_t; using R = float; static constexpr bool kCplx = true; };

// An FP64 (re, im) accumulator; the imaginary part stays 0 for real data.
struct Acc2 {
    double re, im;
};
template <class T> __device__ __forceinline__ void acc_add(Acc2 &a, T v);
template <> __device__ __forceinline__ void acc_add<double>(Acc2 &a, double v) { a.re += v; }
template <> __device__ __forceinline__ void acc_add<float>(Acc2 &a, float v) { a.re += (double)v; }
template <> __device__ __forceinline__ void acc_add<ud2_t>(Acc2 &a, ud2_t v) {
    a.re += v.x;
    a.im += v.y;
}
template <> __device__ __forceinline__ void acc_add<uf2_t>(Acc2 &a, uf2_t v) {
    a.re += (double)v.x;
    a.im += (double)v.y;
}

// C <- alpha * s + beta * C_in (C_in not read when beta = 0).
template <int PREC>
__device__ __forceinline__ void store_out(typename UT<PREC>::T *C, int64_t off, Acc2 s,
                                          const UnaryParams &p, bool rdC) {
    using T = typename UT<PREC>::T;
    using R = typename UT<PREC>::R;
    constexpr bool CPLX = UT<PREC>::kCplx;
    if constexpr (CPLX) {
        double xr = p.alpha[0] * s.re - p.alpha[1] * s.im;
        double xi = p.alpha[0] * s.im + p.alpha[1] * s.re;
        if (rdC) {
            const T c = C[off];
            const double cr = (double)c.x, ci = (double)c.y;
            xr += p.beta[0] * cr - p.beta[1] * ci;
            xi += p.beta[0] * ci + p.beta[1] * cr;
        }
        T o;
        o.x = (R)xr;
        o.y = (R)xi;
        C[off] = o;
    } else {
        double x = p.alpha[0] * s.re;
        if (rdC) x += p.beta[0] * (double)C[off];
        C[off] = (R)x;
    }
}

template <bool CPLX> __device__ __forceinline__ void store_part(double *ws, int64_t i, Acc2 s) {
    if constexpr (CPLX) {
        ws[2 * i] = s.re;
        ws[2 * i + 1] = s.im;
    } else {
        ws[i] = s.re;
    }
}

constexpr int kUT = 64;    // tile extent along O1 and O2
constexpr int kURows = 16; // rows of O2 per thread (4 waves x 16 = 64)

// LDS element of the transpose: one FP64 sum (real data) or a (re, im) pair.
template <bool CPLX> struct LdsT { using T = double; };
template <> struct LdsT<true> { using T = Acc2; };

// Offset in A of summed position r.
__device__ __forceinline__ int64_t r_off(const UnaryParams &p, int64_t r) {
    return p.rAffine ? r * p.rInc : p.offR[r];
}

template <int PREC, bool TRANS, bool RSLOTS>
__global__ __launch_bounds__(256) void unary_tiled_kernel(UnaryParams p) {
    using T = typename UT<PREC>::T;
    constexpr bool kCplx = UT<PREC>::kCplx;
    __shared__ typename LdsT<kCplx>::T lds[(TRANS || RSLOTS) ? kUT * (kUT + 1) : 1];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    // block -> (tile along O1, tile along O2, O3 position, slice)
    int64_t b = blockIdx.x;
    const int64_t t1 = b % p.tiles1;
    b /= p.tiles1;
    const int64_t t2 = b % p.tiles2;
    b /= p.tiles2;
    const int64_t i3 = b % p.n3;
    const int s = (int)(b / p.n3);
    const T *A = static_cast<const T *>(p.A) + p.offA3[i3];
    const int64_t o1 = t1 * kUT + lane;
    const int64_t o2b = t2 * kUT + w;
    const bool ok1 = o1 < p.e1;
    Acc2 acc[kURows];
#pragma unroll
    for (int i = 0; i < kURows; ++i) acc[i] = Acc2{0.0, 0.0};
    const int64_t rbeg = (int64_t)s * p.rPer;
    const int64_t rend = min(p.nR, rbeg + p.rPer);
    const T *rowA = A + o1 * p.ia1 + o2b * p.ia2;
    const int64_t step2 = 4 * p.ia2;
    if constexpr (RSLOTS) {
        // one output row (e2 = 1): slot w + 4 i takes positions rbeg + slot,
        // rbeg + slot + 64, ...; the slots' sums are added in slot order
        const T *q = A + o1 * p.ia1;
        if (ok1)
            for (int64_t r0 = rbeg; r0 < rend; r0 += 64) {
#pragma unroll
                for (int i = 0; i < kURows; ++i) {
                    const int64_t r = r0 + w + 4 * i;   // wave-uniform
                    if (r < rend) acc_add(acc[i], q[r_off(p, r)]);
                }
            }
#pragma unroll
        for (int i = 0; i < kURows; ++i) {
            if constexpr (kCplx) lds[(w + 4 * i) * (kUT + 1) + lane] = acc[i];
            else lds[(w + 4 * i) * (kUT + 1) + lane] = acc[i].re;
        }
        __syncthreads();
        if (w != 0) return;
        Acc2 tot{0.0, 0.0};
        for (int sl = 0; sl < kUT; ++sl) {
            if constexpr (kCplx) {
                tot.re += lds[sl * (kUT + 1) + lane].re;
                tot.im += lds[sl * (kUT + 1) + lane].im;
            } else {
                tot.re += lds[sl * (kUT + 1) + lane];
            }
        }
        if (!ok1) return;
        if (p.S > 1) {
            store_part<kCplx>(p.ws + (int64_t)s * p.nO * (kCplx ? 2 : 1), o1 + p.e1 * i3, tot);
        } else {
            const bool rdC = p.beta[0] != 0.0 || p.beta[1] != 0.0;
            store_out<PREC>(static_cast<T *>(p.C) + p.offC3[i3], o1 * p.ic1, tot, p, rdC);
        }
        return;
    } else if (ok1) {
        for (int64_t r = rbeg; r < rend; ++r) {
            const int64_t off = r_off(p, r);   // wave-uniform
            const T *q = rowA + off;
#pragma unroll
            for (int i = 0; i < kURows; ++i)
                if (o2b + 4 * i < p.e2) acc_add(acc[i], q[i * step2]);
        }
    }
    const bool rdC = p.beta[0] != 0.0 || p.beta[1] != 0.0;
    T *C = static_cast<T *>(p.C) + p.offC3[i3];
    if (p.S > 1) {
        // partials, numbered o1 + e1 (o2 + e2 i3)
        if (ok1)
#pragma unroll
            for (int i = 0; i < kURows; ++i) {
                const int64_t o2 = o2b + 4 * i;
                if (o2 < p.e2)
                    store_part<UT<PREC>::kCplx>(
                        p.ws + (int64_t)s * p.nO * (UT<PREC>::kCplx ? 2 : 1),
                        o1 + p.e1 * (o2 + p.e2 * i3), acc[i]);
            }
        return;
    }
    if constexpr (!TRANS) {
        if (ok1)
#pragma unroll
            for (int i = 0; i < kURows; ++i) {
                const int64_t o2 = o2b + 4 * i;
                if (o2 < p.e2)
                    store_out<PREC>(C, o1 * p.ic1 + o2 * p.ic2, acc[i], p, rdC);
            }
    } else {
        // through LDS: row (w + 4i) of O2, column lane of O1 ...
#pragma unroll
        for (int i = 0; i < kURows; ++i) {
            if constexpr (kCplx) lds[(w + 4 * i) * (kUT + 1) + lane] = acc[i];
            else lds[(w + 4 * i) * (kUT + 1) + lane] = acc[i].re;
        }
        __syncthreads();
        // ... read back with the lanes along O2
        const int64_t o2 = t2 * kUT + lane;
        if (o2 < p.e2) {
#pragma unroll
            for (int i = 0; i < kURows; ++i) {
                const int64_t c1 = t1 * kUT + w + 4 * i;
                if (c1 < p.e1) {
                    Acc2 v;
                    if constexpr (kCplx) v = lds[lane * (kUT + 1) + w + 4 * i];
                    else v = Acc2{lds[lane * (kUT + 1) + w + 4 * i], 0.0};
                    store_out<PREC>(C, c1 * p.ic1 + o2 * p.ic2, v, p, rdC);
                }
            }
        }
    }
}

template <int PREC>
__global__ __launch_bounds__(256) void unary_lanes_r_kernel(UnaryParams p) {
    using T = typename UT<PREC>::T;
    const T *A = static_cast<const T *>(p.A);
    T *C = static_cast<T *>(p.C);
    const int lane = threadIdx.x & 63;
    const int g = p.g;
    const int sub = lane & (g - 1);
    const int per = 64 / g;                       // outputs per wave and round
    const int64_t waves = (int64_t)gridDim.x * 4;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t items = p.nO * p.S;
    const bool rdC = p.beta[0] != 0.0 || p.beta[1] != 0.0;
    for (int64_t base = wave * per; base < items; base += waves * per) {
        const int64_t item = base + lane / g;
        const bool live = item < items;
        const int64_t o = live ? item % p.nO : 0;
        const int s = live ? (int)(item / p.nO) : 0;
        // output o = o1 + e1 (o2 + e2 i3)
        const int64_t o1 = o % p.e1, rest = o / p.e1;
        const int64_t o2 = rest % p.e2, i3 = rest / p.e2;
        Acc2 acc{0.0, 0.0};
        if (live) {
            const int64_t rbeg = (int64_t)s * p.rPer;
            const int64_t rend = min(p.nR, rbeg + p.rPer);
            const T *q = A + p.offA3[i3] + o1 * p.ia1 + o2 * p.ia2;
            // four partial sums (positions r, r + g, r + 2g, r + 3g of each
            // round of 4g), added in that order at the end
            Acc2 a4[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
            int64_t r = rbeg + sub;
            for (; r + 3 * (int64_t)g < rend; r += 4 * (int64_t)g) {
#pragma unroll
                for (int u = 0; u < 4; ++u) acc_add(a4[u], q[r_off(p, r + u * (int64_t)g)]);
            }
            for (int u = 0; r < rend; r += g, ++u) acc_add(a4[u], q[r_off(p, r)]);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                acc.re += a4[u].re;
                acc.im += a4[u].im;
            }
        }
        // add the g lanes' sums (the same tree for every output)
        for (int m = g >> 1; m >= 1; m >>= 1) {
            acc.re += __shfl_xor(acc.re, m, 64);
            acc.im += __shfl_xor(acc.im, m, 64);
        }
        if (live && sub == 0) {
            if (p.S > 1)
                store_part<UT<PREC>::kCplx>(p.ws + (int64_t)s * p.nO * (UT<PREC>::kCplx ? 2 : 1),
                                            o, acc);
            else
                store_out<PREC>(C, p.offC3[i3] + o1 * p.ic1 + o2 * p.ic2, acc, p,
                                              rdC);
        }
    }
}

template <int PREC>
__global__ __launch_bounds__(256) void unary_finish_kernel(UnaryParams p) {
    using T = typename UT<PREC>::T;
    constexpr int W = UT<PREC>::kCplx ? 2 : 1;
    T *C = static_cast<T *>(p.C);
    const bool rdC = p.beta[0] != 0.0 || p.beta[1] != 0.0;
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < p.nO;
         o += (int64_t)gridDim.x * blockDim.x) {
        Acc2 s{0.0, 0.0};
        for (int z = 0; z < p.S; ++z) {
            s.re += p.ws[W * ((int64_t)z * p.nO + o)];
            if (W == 2) s.im += p.ws[W * ((int64_t)z * p.nO + o) + 1];
        }
        const int64_t o1 = o % p.e1, r = o / p.e1;
        const int64_t o2 = r % p.e2, i3 = r / p.e2;
        const int64_t off = p.offC3[i3] + o1 * p.ic1 + o2 * p.ic2;
        store_out<PREC>(C, off, s, p, rdC);
    }
}

template <int PREC> static int tiled_prec(const UnaryParams &p, hipStream_t s) {
    const int64_t blocks = (int64_t)p.tiles1 * p.tiles2 * p.n3 * p.S;
    if (blocks < 1) return 0;
    if (blocks > INT32_MAX) return GETT_ERR_INTERNAL;
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    auto kern = p.trans ? unary_tiled_kernel<PREC, true, false>
                        : (p.e2 == 1 ? unary_tiled_kernel<PREC, false, true>
                                     : unary_tiled_kernel<PREC, false, false>);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, s, p);
    return launch_status();
}

template <int PREC> static int lanes_prec(const UnaryParams &p, hipStream_t s) {
    const int64_t items = p.nO * p.S;
    const int64_t per_block = 4 * (64 / p.g);
    int64_t blocks = (items + per_block - 1) / per_block;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) return 0;
    (void)hipGetLastError();
    hipLaunchKernelGGL(unary_lanes_r_kernel<PREC>, dim3((unsigned)blocks), dim3(256), 0, s, p);
    return launch_status();
}

template <int PREC> static int finish_prec(const UnaryParams &p, hipStream_t s) {
    int64_t blocks = (p.nO + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) return 0;
    (void)hipGetLastError();
    hipLaunchKernelGGL(unary_finish_kernel<PREC>, dim3((unsigned)blocks), dim3(256), 0, s, p);
    return launch_status();
}

int launch_unary_tiled(int prec, const UnaryParams &p, hipStream_t s) {
    switch (prec) {
    case 0: return tiled_prec<0>(p, s);
    case 1: return tiled_prec<1>(p, s);
    case 4: return tiled_prec<4>(p, s);
    case 5: return tiled_prec<5>(p, s);
    default: return GETT_ERR_INTERNAL;
    }
}

int launch_unary_lanes_r(int prec, const UnaryParams &p, hipStream_t s) {
    switch (prec) {
    case 0: return lanes_prec<0>(p, s);
    case 1: return lanes_prec<1>(p, s);
    case 4: return lanes_prec<4>(p, s);
    case 5: return lanes_prec<5>(p, s);
    default: return GETT_ERR_INTERNAL;
    }
}

int launch_unary_finish(int prec, const UnaryParams &p, hipStream_t s) {
    switch (prec) {
    case 0: return finish_prec<0>(p, s);
    case 1: return finish_prec<1>(p, s);
    case 4: return finish_prec<4>(p, s);
    case 5: return finish_prec<5>(p, s);
    default: return GETT_ERR_INTERNAL;
    }
}

}  // namespace gett
