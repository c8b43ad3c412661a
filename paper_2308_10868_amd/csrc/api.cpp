// C ABI of libnrr.so (declared in include/nrr.h): argument validation,
// workspace sizing, status codes and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "nrr.h"
#include "nrr_internal.h"

namespace {

thread_local char g_err[512] = "";

nrr_status fail(nrr_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

nrr_status ok() {
    g_err[0] = '\0';
    return NRR_OK;
}

nrr_status check_grid(const int32_t dims[3], int32_t block, int32_t stride, int32_t grid[3]) {
    if (!dims) return fail(NRR_ERR_INVALID_ARG, "dims is NULL");
    if (block < 3 || block % 2 == 0)
        return fail(NRR_ERR_INVALID_ARG, "block must be odd and >= 3 (got %d)", block);
    if (stride < 1) return fail(NRR_ERR_INVALID_ARG, "stride must be >= 1 (got %d)", stride);
    for (int a = 0; a < 3; ++a) {
        if (dims[a] < block)
            return fail(NRR_ERR_INVALID_ARG, "dims[%d] = %d is smaller than block %d", a, dims[a],
                        block);
        grid[a] = (dims[a] - block) / stride + 1;
    }
    return NRR_OK;
}

nrr_status check_dtype(nrr_dtype dtype) {
    if (dtype != NRR_U16 && dtype != NRR_F32)
        return fail(NRR_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    return NRR_OK;
}

int64_t count_rule(int64_t n, double fraction) {
    double k = std::floor(0.5 + (double)n * fraction);
    if (k < 0) k = 0;
    if (k > (double)n) k = (double)n;
    return (int64_t)k;
}

nrr_status hip_status(hipError_t e, const char *what) {
    if (e == hipSuccess) return ok();
    return fail(NRR_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

extern "C" {

int32_t nrr_version(void) { return 10000; }

const char *nrr_status_string(nrr_status s) {
    switch (s) {
        case NRR_OK: return "ok";
        case NRR_ERR_INVALID_ARG: return "invalid argument";
        case NRR_ERR_BUFFER_TOO_SMALL: return "buffer too small";
        case NRR_ERR_HIP: return "HIP runtime error";
        case NRR_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *nrr_last_error(void) { return g_err; }

nrr_status nrr_grid_shape(const int32_t dims[3], int32_t block, int32_t stride, int32_t grid[3]) {
    if (!grid) return fail(NRR_ERR_INVALID_ARG, "grid is NULL");
    int32_t g[3];
    nrr_status s = check_grid(dims, block, stride, g);
    if (s != NRR_OK) return s;
    for (int a = 0; a < 3; ++a) grid[a] = g[a];
    return ok();
}

nrr_status nrr_select_count(const int32_t dims[3], int32_t block, int32_t stride, double fraction,
                            int64_t *k) {
    if (!k) return fail(NRR_ERR_INVALID_ARG, "k is NULL");
    int32_t g[3];
    nrr_status s = check_grid(dims, block, stride, g);
    if (s != NRR_OK) return s;
    if (!(fraction > 0.0) || fraction > 1.0)
        return fail(NRR_ERR_INVALID_ARG, "fraction must be in (0, 1] (got %g)", fraction);
    *k = count_rule((int64_t)g[0] * g[1] * g[2], fraction);
    return ok();
}

nrr_status nrr_select_workspace_bytes(const int32_t dims[3], int32_t block, int32_t stride,
                                      size_t *bytes) {
    if (!bytes) return fail(NRR_ERR_INVALID_ARG, "bytes is NULL");
    int32_t g[3];
    nrr_status s = check_grid(dims, block, stride, g);
    if (s != NRR_OK) return s;
    *bytes = nrr::select_layout((int64_t)g[0] * g[1] * g[2]).total;
    return ok();
}

nrr_status nrr_match_workspace_bytes(nrr_dtype dtype, const int32_t dims[3], int32_t block,
                                     size_t *bytes) {
    if (!bytes) return fail(NRR_ERR_INVALID_ARG, "bytes is NULL");
    nrr_status s = check_dtype(dtype);
    if (s != NRR_OK) return s;
    int32_t g[3];
    s = check_grid(dims, block, 1, g);
    if (s != NRR_OK) return s;
    *bytes = nrr::stats_layout(dtype, dims, block).total;
    return ok();
}

nrr_status nrr_match_supported(nrr_dtype dtype, int32_t block, int32_t window) {
    nrr_status s = check_dtype(dtype);
    if (s != NRR_OK) return s;
    if (block < 3 || block % 2 == 0)
        return fail(NRR_ERR_INVALID_ARG, "block must be odd and >= 3 (got %d)", block);
    if (window < 0) return fail(NRR_ERR_INVALID_ARG, "window must be >= 0 (got %d)", window);
    const char *why = nrr::match_unsupported_reason(dtype, block, window);
    if (why) return fail(NRR_ERR_UNSUPPORTED, "block %d window %d: %s", block, window, why);
    return ok();
}

nrr_status nrr_select_blocks(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                             int32_t block, int32_t stride, double fraction, int32_t *centers,
                             int64_t capacity, int64_t *k_out, void *workspace,
                             size_t workspace_bytes, void *stream) {
    nrr_status s = check_dtype(dtype);
    if (s != NRR_OK) return s;
    if (!k_out) return fail(NRR_ERR_INVALID_ARG, "k_out is NULL");
    int32_t g[3];
    s = check_grid(dims, block, stride, g);
    if (s != NRR_OK) return s;
    if (block > 15) return fail(NRR_ERR_UNSUPPORTED, "block edge above 15 is not built");
    if (!(fraction > 0.0) || fraction > 1.0)
        return fail(NRR_ERR_INVALID_ARG, "fraction must be in (0, 1] (got %g)", fraction);
    const int64_t n = (int64_t)g[0] * g[1] * g[2];
    const int64_t k = count_rule(n, fraction);
    *k_out = k;
    if (capacity < k)
        return fail(NRR_ERR_BUFFER_TOO_SMALL, "capacity %lld < K = %lld", (long long)capacity,
                    (long long)k);
    if (k == 0) return ok();
    if (!vol || !centers || !workspace)
        return fail(NRR_ERR_INVALID_ARG, "vol, centers and workspace must be non-NULL");
    const size_t need = nrr::select_layout(n).total;
    if (workspace_bytes < need)
        return fail(NRR_ERR_BUFFER_TOO_SMALL, "workspace %zu < %zu bytes", workspace_bytes, need);
    hipError_t e = nrr::launch_select(vol, dtype, dims, block, stride, g, k, centers, workspace,
                                      static_cast<hipStream_t>(stream));
    return hip_status(e, "nrr_select_blocks launch");
}

namespace {

// Shared validation of the matching entry points; fills the stats layout.
nrr_status check_match(const void *ref, const void *flt, nrr_dtype dtype, const int32_t dims[3],
                       const int32_t *centers, int64_t n, int32_t block, int32_t window,
                       const int32_t *disp, const float *ncc, const float *conf,
                       const void *workspace, size_t workspace_bytes, nrr::StatsLayout *L) {
    nrr_status s = check_dtype(dtype);
    if (s != NRR_OK) return s;
    int32_t g[3];
    s = check_grid(dims, block, 1, g);
    if (s != NRR_OK) return s;
    if (window < 0) return fail(NRR_ERR_INVALID_ARG, "window must be >= 0 (got %d)", window);
    if (n < 0) return fail(NRR_ERR_INVALID_ARG, "n must be >= 0 (got %lld)", (long long)n);
    if (n == 0) return ok();
    if (!ref || !flt || !centers || !disp || !ncc || !conf || !workspace)
        return fail(NRR_ERR_INVALID_ARG, "array and workspace pointers must be non-NULL");
    if ((int64_t)dims[0] * dims[1] * dims[2] >= (1ll << 40))
        return fail(NRR_ERR_UNSUPPORTED, "volume too large");
    *L = nrr::stats_layout(dtype, dims, block);
    if (workspace_bytes < L->total)
        return fail(NRR_ERR_BUFFER_TOO_SMALL, "workspace %zu < %zu bytes", workspace_bytes,
                    L->total);
    const char *why = nrr::match_unsupported_reason(dtype, block, window);
    if (why) return fail(NRR_ERR_UNSUPPORTED, "block %d window %d: %s", block, window, why);
    return NRR_OK;
}

nrr_status run_match(const void *ref, const void *flt, nrr_dtype dtype, const int32_t dims[3],
                     const int32_t *centers, int64_t n, int32_t block, int32_t window,
                     int32_t *disp, float *ncc, float *conf, const void *workspace,
                     const nrr::StatsLayout &L, hipStream_t st) {
    nrr::MatchArgs a;
    a.ref = ref;
    a.flt = flt;
    a.nx = dims[0];
    a.ny = dims[1];
    a.nz = dims[2];
    a.centers = centers;
    a.n = n;
    a.block = block;
    a.window = window;
    a.stats = workspace;
    a.pairs = L.pair_off ? reinterpret_cast<const uint32_t *>(
                               static_cast<const char *>(workspace) + L.pair_off)
                         : nullptr;
    a.ox = L.ox;
    a.oy = L.oy;
    a.disp = disp;
    a.ncc = ncc;
    a.conf = conf;
    return hip_status(nrr::launch_match(dtype, a, st), "block match launch");
}

}  // namespace

nrr_status nrr_window_stats(const void *flt, nrr_dtype dtype, const int32_t dims[3],
                            int32_t block, void *workspace, size_t workspace_bytes,
                            void *stream) {
    nrr_status s = check_dtype(dtype);
    if (s != NRR_OK) return s;
    int32_t g[3];
    s = check_grid(dims, block, 1, g);
    if (s != NRR_OK) return s;
    if (block > 15) return fail(NRR_ERR_UNSUPPORTED, "block edge above 15 is not built");
    if (!flt || !workspace) return fail(NRR_ERR_INVALID_ARG, "flt and workspace must be non-NULL");
    const nrr::StatsLayout L = nrr::stats_layout(dtype, dims, block);
    if (workspace_bytes < L.total)
        return fail(NRR_ERR_BUFFER_TOO_SMALL, "workspace %zu < %zu bytes", workspace_bytes,
                    L.total);
    return hip_status(nrr::launch_stats(flt, dtype, dims, block, workspace,
                                        static_cast<hipStream_t>(stream)),
                      "window statistics launch");
}

nrr_status nrr_block_match_prepared(const void *ref, const void *flt, nrr_dtype dtype,
                                    const int32_t dims[3], const int32_t *centers, int64_t n,
                                    int32_t block, int32_t window, int32_t *disp, float *ncc,
                                    float *conf, const void *workspace, size_t workspace_bytes,
                                    void *stream) {
    nrr::StatsLayout L;
    nrr_status s = check_match(ref, flt, dtype, dims, centers, n, block, window, disp, ncc, conf,
                               workspace, workspace_bytes, &L);
    if (s != NRR_OK || n == 0) return s;
    return run_match(ref, flt, dtype, dims, centers, n, block, window, disp, ncc, conf, workspace,
                     L, static_cast<hipStream_t>(stream));
}

nrr_status nrr_block_match(const void *ref, const void *flt, nrr_dtype dtype,
                           const int32_t dims[3], const int32_t *centers, int64_t n,
                           int32_t block, int32_t window, int32_t *disp, float *ncc, float *conf,
                           void *workspace, size_t workspace_bytes, void *stream) {
    nrr::StatsLayout L;
    nrr_status s = check_match(ref, flt, dtype, dims, centers, n, block, window, disp, ncc, conf,
                               workspace, workspace_bytes, &L);
    if (s != NRR_OK || n == 0) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = nrr::launch_stats(flt, dtype, dims, block, workspace, st);
    if (e != hipSuccess) return hip_status(e, "window statistics launch");
    return run_match(ref, flt, dtype, dims, centers, n, block, window, disp, ncc, conf, workspace,
                     L, st);
}

}  // extern "C"
