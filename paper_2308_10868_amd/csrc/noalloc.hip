// Block selection that allocates nothing: nrr_select_blocks with its scratch
// (one 64-bit ranking key per candidate block, the radix-select state and
// the compaction's per-tile counts) taken from a fixed device array of this
// library instead of a caller's workspace.  Every word of that scratch is
// written by the selection's own kernels before it is read, so nothing needs
// clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "nrr.h"
#include "nrr_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;  // up to ~4.19 million candidates
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends.  In host code this name is
// a host-side stand-in: the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch`, per device

}  // namespace

nrr_status nrr_select_blocks_static(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                                    int32_t block, int32_t stride, double fraction,
                                    int32_t *centers, int64_t capacity, int64_t *k_out,
                                    void *stream) {
    int32_t g[3];
    nrr_status s = nrr_grid_shape(dims, block, stride, g);
    if (s != NRR_OK) return s;
    // the plain selection's workspace (the selection variants need more)
    const size_t need = nrr::select_layout((int64_t)g[0] * g[1] * g[2]).total;
    if (need > kScratchBytes)
        return nrr::set_error(NRR_ERR_UNSUPPORTED,
                              "selection needs %zu bytes of scratch; the allocation-free "
                              "selection holds %zu (use nrr_select_blocks with a workspace)",
                              need, kScratchBytes);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return nrr::set_error(NRR_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return nrr::set_error(NRR_ERR_UNSUPPORTED, "device %d beyond the %d served", dev,
                              kMaxDevices);
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_scratch[dev]) {  // once per device, with that device current
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return nrr::set_error(NRR_ERR_HIP, "hipGetSymbolAddress(scratch): %s",
                                      hipGetErrorString(e));
            g_scratch[dev] = p;
        }
        ptr = g_scratch[dev];
    }
    return nrr_select_blocks(vol, dtype, dims, block, stride, fraction, centers, capacity, k_out,
                             ptr, kScratchBytes, stream);
}
