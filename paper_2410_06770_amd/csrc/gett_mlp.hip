// gett_mlp.hip -- kernels of the schedule predictor: a small FP32 MLP
// (Linear + bias + ReLU layers, softmax cross-entropy over several heads,
// Adam).  The network is tiny (batch <= a few hundred, widths <= 128), so each
// kernel maps one thread to one output value and keeps every reduction in a
// fixed order: results do not depend on the launch and repeat bit for bit.
#include "gett_internal.h"

namespace gett {

// Y[b][o] = act(sum_i X[b][i] W[o][i] + bias[o]);  rows of W are contiguous.
__global__ void mlp_fwd_kernel(const float *__restrict__ X, const float *__restrict__ W,
                               const float *__restrict__ bias, float *__restrict__ Y, int64_t batch,
                               int64_t din, int64_t dout, int relu) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= batch * dout) return;
    const int64_t b = idx / dout, o = idx - b * dout;
    const float *x = X + b * din;
    const float *w = W + o * din;
    float s = 0.f;
    for (int64_t i = 0; i < din; ++i) s = fmaf(x[i], w[i], s);
    s += bias[o];
    Y[idx] = (relu && s < 0.f) ? 0.f : s;
}

__device__ __forceinline__ float dz_of(const float *Y, const float *dY, int64_t i, int relu) {
    const float g = dY[i];
    return (relu && !(Y[i] > 0.f)) ? 0.f : g;
}

// dW[o][i] = sum_b dZ[b][o] X[b][i];  db[o] = sum_b dZ[b][o]
__global__ void mlp_bwd_w_kernel(const float *__restrict__ X, const float *__restrict__ Y,
                                 const float *__restrict__ dY, float *__restrict__ dW,
                                 float *__restrict__ db, int64_t batch, int64_t din, int64_t dout,
                                 int relu) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nW = dout * din;
    if (idx < nW) {
        const int64_t o = idx / din, i = idx - o * din;
        float s = 0.f;
        for (int64_t b = 0; b < batch; ++b) s = fmaf(dz_of(Y, dY, b * dout + o, relu), X[b * din + i], s);
        dW[idx] = s;
    } else if (idx < nW + dout) {
        const int64_t o = idx - nW;
        float s = 0.f;
        for (int64_t b = 0; b < batch; ++b) s += dz_of(Y, dY, b * dout + o, relu);
        db[o] = s;
    }
}

// dX[b][i] = sum_o dZ[b][o] W[o][i]
__global__ void mlp_bwd_x_kernel(const float *__restrict__ W, const float *__restrict__ Y,
                                 const float *__restrict__ dY, float *__restrict__ dX,
                                 int64_t batch, int64_t din, int64_t dout, int relu) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= batch * din) return;
    const int64_t b = idx / din, i = idx - b * din;
    float s = 0.f;
    for (int64_t o = 0; o < dout; ++o) s = fmaf(dz_of(Y, dY, b * dout + o, relu), W[o * din + i], s);
    dX[idx] = s;
}

struct Heads {
    int32_t n;
    int32_t size[8];
};

// One workgroup: thread r handles rows r, r + 256, ...; per head a stable
// softmax; loss = mean over rows of -sum T log p; dZ = (p - T * sum T) / batch.
__global__ __launch_bounds__(256) void mlp_xent_kernel(const float *__restrict__ Z,
                                                       const float *__restrict__ T,
                                                       float *__restrict__ dZ,
                                                       float *__restrict__ loss, int64_t batch,
                                                       int64_t total, Heads heads) {
    __shared__ float part[256];
    float acc = 0.f;
    for (int64_t b = threadIdx.x; b < batch; b += blockDim.x) {
        const float *z = Z + b * total;
        const float *t = T + b * total;
        float *g = dZ + b * total;
        int64_t o = 0;
        for (int h = 0; h < heads.n; ++h) {
            const int n = heads.size[h];
            float mx = z[o];
            for (int i = 1; i < n; ++i) mx = fmaxf(mx, z[o + i]);
            float se = 0.f, ts = 0.f;
            for (int i = 0; i < n; ++i) {
                se += expf(z[o + i] - mx);
                ts += t[o + i];
            }
            const float lse = mx + logf(se);
            for (int i = 0; i < n; ++i) {
                const float lp = z[o + i] - lse;
                acc -= t[o + i] * lp;
                g[o + i] = (expf(lp) * ts - t[o + i]) / (float)batch;
            }
            o += n;
        }
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = part[0] / (float)batch;
}

__global__ void mlp_adam_kernel(float *__restrict__ P, const float *__restrict__ G,
                                float *__restrict__ m, float *__restrict__ v, int64_t n, float lr,
                                float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = G[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    P[i] = P[i] - lr * mh / (sqrtf(vh) + eps);
}

static int blocks_for(int64_t n) { return (int)((n + 255) / 256); }

int launch_mlp_linear_fwd(const float *X, const float *W, const float *b, float *Y, int64_t batch,
                          int64_t din, int64_t dout, int relu, hipStream_t s) {
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    hipLaunchKernelGGL(mlp_fwd_kernel, dim3(blocks_for(batch * dout)), dim3(256), 0, s, X, W, b, Y,
                       batch, din, dout, relu);
    return launch_status();
}

int launch_mlp_linear_bwd(const float *X, const float *W, const float *Y, const float *dY,
                          float *dX, float *dW, float *db, int64_t batch, int64_t din,
                          int64_t dout, int relu, hipStream_t s) {
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    hipLaunchKernelGGL(mlp_bwd_w_kernel, dim3(blocks_for(dout * din + dout)), dim3(256), 0, s, X, Y,
                       dY, dW, db, batch, din, dout, relu);
    if (launch_status()) return GETT_ERR_HIP;
    if (dX) {
        hipLaunchKernelGGL(mlp_bwd_x_kernel, dim3(blocks_for(batch * din)), dim3(256), 0, s, W, Y,
                           dY, dX, batch, din, dout, relu);
    }
    return launch_status();
}

int launch_mlp_xent(const float *Z, const float *T, float *dZ, float *loss, int64_t batch,
                    int64_t total, int64_t nheads, const int64_t *head_sizes, hipStream_t s) {
    Heads h;
    h.n = (int32_t)nheads;
    for (int i = 0; i < 8; ++i) h.size[i] = i < nheads ? (int32_t)head_sizes[i] : 0;
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    hipLaunchKernelGGL(mlp_xent_kernel, dim3(1), dim3(256), 0, s, Z, T, dZ, loss, batch, total, h);
    return launch_status();
}

int launch_mlp_adam(float *P, const float *G, float *m, float *v, int64_t n, float lr, float b1,
                    float b2, float eps, int64_t t, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)t);
    const float c2 = 1.f - powf(b2, (float)t);
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    hipLaunchKernelGGL(mlp_adam_kernel, dim3(blocks_for(n)), dim3(256), 0, s, P, G, m, v, n, lr, b1,
                       b2, eps, c1, c2);
    return launch_status();
}

}  // namespace gett
