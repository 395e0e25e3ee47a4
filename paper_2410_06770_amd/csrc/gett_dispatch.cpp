// gett_dispatch.cpp -- routes launches to the per-precision tile objects.
#include "gett_internal.h"

namespace gett {

static thread_local hipError_t t_last_hip_error = hipSuccess;

int launch_status() {
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return 0;
    t_last_hip_error = e;
    return GETT_ERR_HIP;
}

const char *last_hip_error_name() {
    return t_last_hip_error == hipSuccess ? "" : hipGetErrorName(t_last_hip_error);
}

#define GETT_DECLARE_PRECISION(SUFFIX)                                                             \
    int launch_tile_##SUFFIX(int tile, bool afk, bool bfk, const TileParams &p, hipStream_t s);    \
    int launch_splitk_reduce_##SUFFIX(const TileParams &p, hipStream_t s);                        \
    int batch_grid_size_##SUFFIX();                                                                \
    int launch_batch_##SUFFIX(const BatchProblem *d, const int32_t *it, int32_t n, int32_t *nx,    \
                              int32_t g, hipStream_t s);                                                      \
    int launch_batch_reduce_##SUFFIX(const BatchProblem *d, const int32_t *l, int32_t n,           \
                                     hipStream_t s);                                               \
    int64_t addr_violations_##SUFFIX(bool reset);
GETT_DECLARE_PRECISION(f64)
GETT_DECLARE_PRECISION(f32)
GETT_DECLARE_PRECISION(bf3)
#define GETT_DECLARE_TILE_PRECISION(SUFFIX)                                                        \
    int launch_tile_##SUFFIX(int tile, bool afk, bool bfk, const TileParams &p, hipStream_t s);    \
    int launch_splitk_reduce_##SUFFIX(const TileParams &p, hipStream_t s);                        \
    int64_t addr_violations_##SUFFIX(bool reset);
GETT_DECLARE_TILE_PRECISION(z64)
GETT_DECLARE_TILE_PRECISION(c32)

int launch_tile(int prec, int tile, bool aFastK, bool bFastK, const TileParams &p, hipStream_t s) {
    switch (prec) {
    case kF64: return launch_tile_f64(tile, aFastK, bFastK, p, s);
    case kF32: return launch_tile_f32(tile, aFastK, bFastK, p, s);
    case kBF3: return launch_tile_bf3(tile, aFastK, bFastK, p, s);
    case kZ64: return launch_tile_z64(tile, aFastK, bFastK, p, s);
    case kC32: return launch_tile_c32(tile, aFastK, bFastK, p, s);
    default: return GETT_ERR_INTERNAL;
    }
}

int launch_splitk_reduce(int prec, const TileParams &p, hipStream_t s) {
    switch (prec) {
    case kF64: return launch_splitk_reduce_f64(p, s);
    case kF32: return launch_splitk_reduce_f32(p, s);
    case kBF3: return launch_splitk_reduce_bf3(p, s);
    case kZ64: return launch_splitk_reduce_z64(p, s);
    case kC32: return launch_splitk_reduce_c32(p, s);
    default: return GETT_ERR_INTERNAL;
    }
}

int batch_grid_size(int prec) {
    switch (prec) {
    case kF64: return batch_grid_size_f64();
    case kF32: return batch_grid_size_f32();
    case kBF3: return batch_grid_size_bf3();
    default: return -1;
    }
}

int launch_batch(int prec, const BatchProblem *d_probs, int32_t nprobs, const int32_t *d_items,
                 int32_t nitems, int32_t *d_next, int32_t grid, hipStream_t s) {
    (void)nprobs;
    switch (prec) {
    case kF64: return launch_batch_f64(d_probs, d_items, nitems, d_next, grid, s);
    case kF32: return launch_batch_f32(d_probs, d_items, nitems, d_next, grid, s);
    case kBF3: return launch_batch_bf3(d_probs, d_items, nitems, d_next, grid, s);
    default: return GETT_ERR_INTERNAL;
    }
}

int launch_batch_reduce(int prec, const BatchProblem *d_probs, const int32_t *d_list, int32_t n,
                        hipStream_t s) {
    switch (prec) {
    case kF64: return launch_batch_reduce_f64(d_probs, d_list, n, s);
    case kF32: return launch_batch_reduce_f32(d_probs, d_list, n, s);
    case kBF3: return launch_batch_reduce_bf3(d_probs, d_list, n, s);
    default: return GETT_ERR_INTERNAL;
    }
}

#ifdef GETT_ADDR_CHECK
int64_t addr_violations(int prec, bool reset) {
    switch (prec) {
    case kF64: return addr_violations_f64(reset);
    case kF32: return addr_violations_f32(reset);
    case kBF3: return addr_violations_bf3(reset);
    case kZ64: return addr_violations_z64(reset);
    case kC32: return addr_violations_c32(reset);
    default: return -1;
    }
}
#endif

}  // namespace gett
