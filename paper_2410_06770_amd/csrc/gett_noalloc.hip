// gett_noalloc.hip -- device scratch of the allocation-free entry point
// (dgett_noalloc) and the kernel that writes a plan's offset tables into it.
//
// dgett_noalloc runs the same tile and split-K kernels as dgett, but its
// offset tables and its split-K partial sums live in one file-scope device
// array instead of library allocations.  Each GPU holds its own copy of the
// array (GETT_NOALLOC_SCRATCH_BYTES) until the process ends; every call on a
// GPU reuses it, so calls that overlap on one GPU (different streams or
// threads) race.
#include <mutex>

#include "gett_internal.h"
#include "gett_noalloc.h"

namespace gett {

// The scratch array.  In host code its name is a host-side stand-in, never a
// device address: host code uses the per-device address obtained below.
static __device__ __align__(256) unsigned char scratch[GETT_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

int noalloc_scratch(int dev, void **ptr, int64_t *bytes) {
    if (dev < 0 || dev >= kMaxDevices) return GETT_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        // Called with `dev` current (the caller checked the device): the
        // address of this device's copy of the array.
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return GETT_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    *bytes = GETT_NOALLOC_SCRATCH_BYTES;
    return 0;
}

// off_T[g] = sum_i inc_T,i * coord_i(g) for the six tables of a canonical
// form (M: A and C slots, N: B and C slots, K: A and B slots), first mode
// fastest, zero past the group's size (the padding the tiles rely on).
__global__ __launch_bounds__(256) void table_fill_kernel(FillGroups f, int64_t *__restrict__ out) {
    const int64_t total = 2 * (f.pad[0] + f.pad[1] + f.pad[2]);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = i;
        int grp = 0;
        while (r >= 2 * f.pad[grp]) {
            r -= 2 * f.pad[grp];
            ++grp;
        }
        const int slot = r >= f.pad[grp] ? 1 : 0;
        int64_t g = r - slot * f.pad[grp];
        int64_t off = 0;
        if (g < f.size[grp]) {
            const FillMode *md = f.modes[grp];
            for (int j = 0; j < f.nmodes[grp]; ++j) {
                const int64_t e = md[j].ext;
                const int64_t c = g % e;
                g /= e;
                off += c * (slot ? md[j].i1 : md[j].i0);
            }
        }
        out[i] = off;
    }
}

int launch_table_fill(const FillGroups &f, int64_t *out, hipStream_t s) {
    const int64_t total = 2 * (f.pad[0] + f.pad[1] + f.pad[2]);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    (void)hipGetLastError();   // clear a stale error left by other HIP users
    hipLaunchKernelGGL(table_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, f, out);
    return launch_status();
}

}  // namespace gett
