// gett_scale.hip -- C <- beta * C over every output of a scaled call whose
// contracted sum is empty (a contracted extent of zero): the alpha * sum
// part vanishes, the beta * C_in part remains.
#include "gett_internal.h"

namespace gett {

template <class T> struct ScaleT;
template <> struct ScaleT<double> {
    static __device__ double apply(double c, double br, double, bool rd) { return rd ? br * c : 0.0; }
};
template <> struct ScaleT<float> {
    static __device__ float apply(float c, double br, double, bool rd) {
        return rd ? (float)br * c : 0.0f;
    }
};

template <class T>
__global__ __launch_bounds__(256) void scale_c_kernel(T *C, ScaleModes m, double br, double bi) {
    const bool rd = br != 0.0 || bi != 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m.total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = i, off = 0;
        for (int j = 0; j < m.n; ++j) {
            off += (r % m.ext[j]) * m.inc[j];
            r /= m.ext[j];
        }
        C[off] = ScaleT<T>::apply(rd ? C[off] : T(0), br, bi, rd);
    }
}

// Complex elements: (re, im) pairs of R.
template <class R>
__global__ __launch_bounds__(256) void scale_cz_kernel(R *C, ScaleModes m, double br, double bi) {
    const bool rd = br != 0.0 || bi != 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m.total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = i, off = 0;
        for (int j = 0; j < m.n; ++j) {
            off += (r % m.ext[j]) * m.inc[j];
            r /= m.ext[j];
        }
        R xr = 0, xi = 0;
        if (rd) {
            const R cr = C[2 * off], ci = C[2 * off + 1];
            xr = (R)br * cr - (R)bi * ci;
            xi = (R)br * ci + (R)bi * cr;
        }
        C[2 * off] = xr;
        C[2 * off + 1] = xi;
    }
}

int launch_scale_c(int prec, void *C, const ScaleModes &m, const double *beta, hipStream_t s) {
    int64_t blocks = (m.total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    const dim3 g((unsigned)blocks), b(256);
    switch (prec) {
    case kF64:
        hipLaunchKernelGGL(scale_c_kernel<double>, g, b, 0, s, static_cast<double *>(C), m,
                           beta[0], beta[1]);
        break;
    case kF32:
    case kBF3:
        hipLaunchKernelGGL(scale_c_kernel<float>, g, b, 0, s, static_cast<float *>(C), m, beta[0],
                           beta[1]);
        break;
    case kZ64:
        hipLaunchKernelGGL(scale_cz_kernel<double>, g, b, 0, s, static_cast<double *>(C), m,
                           beta[0], beta[1]);
        break;
    case kC32:
        hipLaunchKernelGGL(scale_cz_kernel<float>, g, b, 0, s, static_cast<float *>(C), m,
                           beta[0], beta[1]);
        break;
    default: return GETT_ERR_INTERNAL;
    }
    return launch_status();
}

}  // namespace gett
