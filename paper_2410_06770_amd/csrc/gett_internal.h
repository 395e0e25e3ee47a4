// gett_internal.h -- launcher and status declarations shared by the host
// runtime and the gfx950 kernel files; the tile menus and launch descriptors
// are in gett_config.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gett.h"
#include "gett_config.h"

namespace gett {

// Status of the launch just made: 0, or GETT_ERR_HIP with the HIP error kept
// for gett_strerror (callers clear any stale error before launching).
int launch_status();
const char *last_hip_error_name();

// Output modes of C (extent > 1) for the scaling pass of calls whose
// contracted sum is empty; rank of C is at most 128, and at most 63 of its
// modes can have extent > 1 in an addressable tensor.
constexpr int kScaleModes = 64;
struct ScaleModes {
    int64_t ext[kScaleModes], inc[kScaleModes];
    int32_t n;
    int32_t pad_;
    int64_t total;
};
// C <- beta * C (beta = (re, im); zero writes zeros without reading C).
int launch_scale_c(int prec, void *C, const ScaleModes &m, const double *beta, hipStream_t s);

// The current device, checked once per device to be gfx950 (0, or
// GETT_ERR_HIP / GETT_ERR_DEVICE).
int current_device_checked(int *dev);
// Releases the unary operations' plan cache (gett_finalize).
void unary_release();
// Stream-ordered temporary buffer on the current device from the library's
// pool (0 or GETT_ERR_ALLOC), and its release on the same stream.
int work_alloc(void **p, size_t bytes, hipStream_t s);
int work_free(void *p, hipStream_t s);

// Kernel launchers (defined in the .hip files).
int launch_tile(int prec, int tile, bool aFastK, bool bFastK, const TileParams &p,
                hipStream_t s);
int launch_splitk_reduce(int prec, const TileParams &p, hipStream_t s);
// Persistent batch kernel: its workgroups claim items through *d_next, which
// must be 0 when the kernel starts.
int launch_batch(int prec, const BatchProblem *d_probs, int32_t nprobs, const int32_t *d_items,
                 int32_t nitems, int32_t *d_next, int32_t grid, hipStream_t s);
int batch_grid_size(int prec);
// C = C_in + sum of the FP64 slice partials for the listed batch problems
// (those cut along K), reading their descriptors on the device.
int launch_batch_reduce(int prec, const BatchProblem *d_probs, const int32_t *d_list, int32_t n,
                        hipStream_t s);
#ifdef GETT_ADDR_CHECK
// Checked build: out-of-range accesses counted by the kernels of one
// precision on the current device (optionally reset); negative on a HIP error.
int64_t addr_violations(int prec, bool reset);
#endif

// FP8 path: quantisation into canonical K-contiguous rows and the GEMM on them.
// rowsFast selects the loader whose lanes run along the rows (for operands
// whose rows, not their contracted positions, are the cheap direction); it
// walks the rows in the order of offR, and rowMap (NULL: identity) gives the
// output row of each.
// bs: contracted positions per scale, 128 or 32 (MX-style); E holds
// 128 / bs exponents per row and 128-block.  fmt: element format, numbered
// as the scaled MFMA's format operand (kElemE4M3 with either block size;
// kElemE2M3 / kElemE2M1 with bs 32); codes are one per byte either way.
constexpr int kElemE4M3 = 0, kElemE2M3 = 2, kElemE2M1 = 4;
int launch_fp8_quant(const float *X, const int64_t *offR, const int32_t *rowMap, int64_t rows,
                     int64_t rowsPad, const int64_t *offK, int64_t K, bool rowsFast, uint8_t *Q,
                     int32_t *E, hipStream_t s, int bs, int fmt);
int launch_fp8_gemm(int tile, const uint8_t *QA, const int32_t *EA, const uint8_t *QB,
                    const int32_t *EB, float *C, const int64_t *offCM, const int64_t *offCN,
                    int64_t M, int64_t N, int64_t K, hipStream_t s, int bs, int fmt);

// MLP kernels.
int launch_mlp_linear_fwd(const float *X, const float *W, const float *b, float *Y, int64_t batch,
                          int64_t din, int64_t dout, int relu, hipStream_t s);
int launch_mlp_linear_bwd(const float *X, const float *W, const float *Y, const float *dY,
                          float *dX, float *dW, float *db, int64_t batch, int64_t din,
                          int64_t dout, int relu, hipStream_t s);
int launch_mlp_xent(const float *Z, const float *T, float *dZ, float *loss, int64_t batch,
                    int64_t total, int64_t nheads, const int64_t *head_sizes, hipStream_t s);
int launch_mlp_adam(float *P, const float *G, float *m, float *v, int64_t n, float lr, float b1,
                    float b2, float eps, int64_t t, hipStream_t s);

}  // namespace gett
