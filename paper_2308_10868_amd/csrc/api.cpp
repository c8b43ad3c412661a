// C ABI of libnrr.so (declared in include/nrr.h): argument validation,
// workspace sizing, status codes and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <numeric>
#include <unordered_map>
#include <vector>

#include "nrr.h"
#include "nrr_internal.h"
#include "stats_cols.h"

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

}  // namespace

// The thread-local detail of nrr_last_error, for the library's other files.
nrr_status nrr::set_error(nrr_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

namespace {

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
    *bytes = nrr::select_layout((int64_t)g[0] * g[1] * g[2], true).total;
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

nrr_status nrr_match_plan(nrr_dtype dtype, const int32_t dims[3], int32_t block, int32_t window,
                          nrr_tile_shape *shape) {
    if (!dims || !shape) return fail(NRR_ERR_INVALID_ARG, "dims and shape must be non-NULL");
    nrr_status s = nrr_match_supported(dtype, block, window);
    if (s != NRR_OK) return s;
    int32_t g[3];
    if ((s = check_grid(dims, block, 1, g)) != NRR_OK) return s;
    nrr::MatchArgs a{};
    a.nx = dims[0];
    a.ny = dims[1];
    a.nz = dims[2];
    a.block = block;
    a.window = window;
    a.ox = dims[0] - block + 1;
    a.oy = dims[1] - block + 1;
    nrr::TileShape t;
    if (!nrr::match_plan(dtype, a, &t))
        return fail(NRR_ERR_UNSUPPORTED, "no compiled shape for block %d window %d", block, window);
    *shape = nrr_tile_shape{t.arith, t.rx, t.ry, t.nt, t.pf, t.cz};
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
    if (n >= (1ll << 31))
        return fail(NRR_ERR_UNSUPPORTED, "%lld candidates (grids of 2^31 or more are not built)",
                    (long long)n);
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

nrr_status nrr_select_blocks_ex(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                                int32_t block, int32_t stride, double fraction,
                                const uint8_t *mask, int32_t connectivity, int32_t *centers,
                                int64_t capacity, int64_t *k_device, void *workspace,
                                size_t workspace_bytes, void *stream) {
    nrr_status s = check_dtype(dtype);
    if (s != NRR_OK) return s;
    int32_t g[3];
    if ((s = check_grid(dims, block, stride, g)) != NRR_OK) return s;
    if (!(fraction > 0.0 && fraction <= 1.0))
        return fail(NRR_ERR_INVALID_ARG, "fraction must be in (0, 1] (got %g)", fraction);
    if (connectivity != 0 && connectivity != 6 && connectivity != 18 && connectivity != 26)
        return fail(NRR_ERR_INVALID_ARG, "connectivity must be 0, 6, 18 or 26 (got %d)",
                    connectivity);
    if (!vol || !centers || !k_device || !workspace)
        return fail(NRR_ERR_INVALID_ARG, "vol, centers, k_device and workspace must be non-NULL");
    const int64_t n = (int64_t)g[0] * g[1] * g[2];
    if (n >= (1ll << 31))
        return fail(NRR_ERR_UNSUPPORTED, "%lld candidates (limit 2^31)", (long long)n);
    const int64_t kmax = count_rule(n, fraction);
    if (capacity < kmax)
        return fail(NRR_ERR_BUFFER_TOO_SMALL, "capacity %lld < %lld", (long long)capacity,
                    (long long)kmax);
    const nrr::SelectLayout L = nrr::select_layout(n, true);
    if (workspace_bytes < L.total)
        return fail(NRR_ERR_BUFFER_TOO_SMALL, "workspace %zu < %zu bytes", workspace_bytes,
                    L.total);
    return hip_status(nrr::launch_select_ex(vol, dtype, dims, block, stride, g, fraction, mask,
                                            connectivity, centers, k_device, workspace,
                                            static_cast<hipStream_t>(stream)),
                      "nrr_select_blocks_ex launch");
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

nrr::MatchArgs match_args(const void *ref, const void *flt, const int32_t dims[3],
                          const int32_t *centers, int64_t n, int32_t block, int32_t window,
                          int32_t *disp, float *ncc, float *conf, const void *workspace,
                          const nrr::StatsLayout &L) {
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
    return a;
}

// Whether a search workspace holds the plane-pair volume of 12-bit data (the
// dot2 form reads it; the other forms do not), as the last statistics call
// on that workspace left it.  Workspaces never filled by nrr_window_stats_for
// count as holding it (nrr_window_stats always writes it).
std::mutex g_pairs_mu;
std::unordered_map<const void *, bool> g_pairs;

void note_pairs(const void *ws, bool has) {
    std::lock_guard<std::mutex> lk(g_pairs_mu);
    if (has)
        g_pairs.erase(ws);
    else
        g_pairs[ws] = false;
}

bool holds_pairs(const void *ws) {
    std::lock_guard<std::mutex> lk(g_pairs_mu);
    return g_pairs.find(ws) == g_pairs.end();
}

// Does the search planned for these sizes read the plane-pair volume?
bool plan_reads_pairs(nrr_dtype dtype, const nrr::MatchArgs &a) {
    if (dtype != NRR_U16) return false;
    nrr::TileShape t;
    return !nrr::match_plan(dtype, a, &t) || t.arith == 0;
}

nrr_status run_match(const void *ref, const void *flt, nrr_dtype dtype, const int32_t dims[3],
                     const int32_t *centers, int64_t n, int32_t block, int32_t window,
                     int32_t *disp, float *ncc, float *conf, const void *workspace,
                     const nrr::StatsLayout &L, hipStream_t st) {
    const nrr::MatchArgs a =
        match_args(ref, flt, dims, centers, n, block, window, disp, ncc, conf, workspace, L);
    if (L.pair_off && plan_reads_pairs(dtype, a) && !holds_pairs(workspace)) {
        // statistics made for another plan: add the pair volume now
        hipError_t e = nrr::launch_pair_volume(static_cast<const uint16_t *>(flt), dims,
                                               const_cast<uint32_t *>(a.pairs), st);
        if (e != hipSuccess) return hip_status(e, "pair volume launch");
        note_pairs(workspace, true);
    }
    return hip_status(nrr::launch_match(dtype, a, st), "block match launch");
}

// Sizes, plans and workspace regions of a batched search.
struct BatchLayout {
    std::vector<int64_t> ncand, k, off;  // per set (off: nsets + 1 rows offsets)
    std::vector<int32_t> grid;           // per set, 3 values
    std::vector<int32_t> variant, cz;
    std::vector<double> cost;            // per set: K times the per-block cost
    std::vector<int32_t> bvals;          // distinct block sizes
    std::vector<size_t> stats_off;       // per distinct block size
    size_t sel_off = 0, sets_off = 0, keys_off = 0, total = 0, lds = 0;
    int64_t nitems = 0, max_cand = 0, sum_cand = 0;
};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

nrr_status batch_layout(nrr_dtype dtype, const int32_t dims[3], const nrr_param_set *sets,
                        int32_t nsets, BatchLayout *L) {
    nrr_status s = check_dtype(dtype);
    if (s != NRR_OK) return s;
    if (nsets < 0) return fail(NRR_ERR_INVALID_ARG, "nsets must be >= 0 (got %d)", nsets);
    if (nsets > 0 && !sets) return fail(NRR_ERR_INVALID_ARG, "sets is NULL");
    L->off.assign(1, 0);
    for (int i = 0; i < nsets; ++i) {
        const nrr_param_set &q = sets[i];
        int32_t g[3];
        if ((s = check_grid(dims, q.block, q.stride, g)) != NRR_OK) return s;
        if (!(q.fraction > 0.0 && q.fraction <= 1.0))
            return fail(NRR_ERR_INVALID_ARG, "set %d: fraction must be in (0, 1]", i);
        if (q.window < 0) return fail(NRR_ERR_INVALID_ARG, "set %d: window must be >= 0", i);
        if (q.window > 64) return fail(NRR_ERR_UNSUPPORTED, "set %d: window above 64", i);
        const int64_t nc = (int64_t)g[0] * g[1] * g[2];
        if (nc > nrr::kBatchCand)
            return fail(NRR_ERR_UNSUPPORTED, "set %d: %lld candidate blocks (batched limit %d)", i,
                        (long long)nc, nrr::kBatchCand);
        int32_t var = 0, cz = 0;
        size_t lds = 0;
        double per = 0.0;
        if (!nrr::plan_batch_set(dtype, q.block, q.window, &var, &cz, &lds, &per))
            return fail(NRR_ERR_UNSUPPORTED, "set %d: no batched shape for block %d window %d", i,
                        q.block, q.window);
        const int64_t k = count_rule(nc, q.fraction);
        L->ncand.push_back(nc);
        L->k.push_back(k);
        L->off.push_back(L->off.back() + k);
        L->grid.insert(L->grid.end(), g, g + 3);
        L->variant.push_back(var);
        L->cz.push_back(cz);
        L->cost.push_back(per * (double)k);
        L->lds = std::max(L->lds, lds);
        L->nitems += k;
        L->max_cand = std::max(L->max_cand, nc);
        L->sum_cand += nc;
        if (std::find(L->bvals.begin(), L->bvals.end(), q.block) == L->bvals.end())
            L->bvals.push_back(q.block);
    }
    size_t at = 0;
    for (int32_t b : L->bvals) {
        L->stats_off.push_back(at);
        at += align256(nrr::stats_layout(dtype, dims, b).total);
    }
    L->sel_off = at;
    at += align256(sizeof(nrr::BatchSelectSet) * (size_t)std::max(nsets, 1));
    L->sets_off = at;
    at += align256(sizeof(nrr::BatchSet) * (size_t)std::max(nsets, 1));
    L->keys_off = at;
    at += align256(sizeof(uint64_t) * (size_t)std::max<int64_t>(L->sum_cand, 1));
    L->total = at;
    return NRR_OK;
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
    note_pairs(workspace, true);
    return hip_status(nrr::launch_stats(flt, dtype, dims, block, workspace,
                                        static_cast<hipStream_t>(stream)),
                      "window statistics launch");
}

nrr_status nrr_window_stats_for(const void *flt, nrr_dtype dtype, const int32_t dims[3],
                                int32_t block, int32_t window, void *workspace,
                                size_t workspace_bytes, void *stream) {
    nrr_status s = check_dtype(dtype);
    if (s != NRR_OK) return s;
    int32_t g[3];
    if ((s = check_grid(dims, block, 1, g)) != NRR_OK) return s;
    if (block > 15) return fail(NRR_ERR_UNSUPPORTED, "block edge above 15 is not built");
    if (window < 0) return fail(NRR_ERR_INVALID_ARG, "window must be >= 0 (got %d)", window);
    if (!flt || !workspace) return fail(NRR_ERR_INVALID_ARG, "flt and workspace must be non-NULL");
    const nrr::StatsLayout L = nrr::stats_layout(dtype, dims, block);
    if (workspace_bytes < L.total)
        return fail(NRR_ERR_BUFFER_TOO_SMALL, "workspace %zu < %zu bytes", workspace_bytes,
                    L.total);
    const nrr::MatchArgs a = match_args(nullptr, flt, dims, nullptr, 0, block, window, nullptr,
                                        nullptr, nullptr, workspace, L);
    const bool pairs = plan_reads_pairs(dtype, a);
    note_pairs(workspace, pairs);
    const int32_t b3[3] = {block, block, block};
    return hip_status(nrr::launch_stats(flt, dtype, dims, b3, pairs, workspace,
                                        static_cast<hipStream_t>(stream)),
                      "window statistics launch");
}

namespace {

// The library's second stream and fork/join events, one set per device,
// created on first use; the mutex makes each call's record/wait sequence
// atomic, so the reused events always pair with the call that recorded them.
struct ForkSet {
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex g_fork_mu;
ForkSet g_fork[64];

// The current device's fork set, created on first use (call with g_fork_mu
// held: the caller's record/wait sequence then owns the events).
hipError_t fork_set(ForkSet **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    ForkSet &fs = g_fork[dev];
    if (!fs.side) {
        e = hipStreamCreateWithFlags(&fs.side, hipStreamNonBlocking);  // default priority
        // the events order work of this device only: no system-scope fences
        const unsigned fl = hipEventDisableTiming | hipEventDisableSystemFence;
        if (e == hipSuccess) e = hipEventCreateWithFlags(&fs.fork, fl);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&fs.join, fl);
        if (e != hipSuccess) return e;
    }
    *out = &fs;
    return hipSuccess;
}

}  // namespace

nrr_status nrr_select_and_window_stats(const void *ref, const void *flt, nrr_dtype dtype,
                                       const int32_t dims[3], int32_t block, int32_t stride,
                                       double fraction, int32_t window, int32_t *centers,
                                       int64_t capacity, int64_t *k_out, void *select_workspace,
                                       size_t select_workspace_bytes, void *match_workspace,
                                       size_t match_workspace_bytes, void *stream) {
    nrr_status s = check_dtype(dtype);
    if (s != NRR_OK) return s;
    if (!k_out) return fail(NRR_ERR_INVALID_ARG, "k_out is NULL");
    int32_t g[3];
    if ((s = check_grid(dims, block, stride, g)) != NRR_OK) return s;
    if (block > 15) return fail(NRR_ERR_UNSUPPORTED, "block edge above 15 is not built");
    if (!(fraction > 0.0) || fraction > 1.0)
        return fail(NRR_ERR_INVALID_ARG, "fraction must be in (0, 1] (got %g)", fraction);
    if (window < 0) return fail(NRR_ERR_INVALID_ARG, "window must be >= 0 (got %d)", window);
    const int64_t n = (int64_t)g[0] * g[1] * g[2];
    if (n >= (1ll << 31))
        return fail(NRR_ERR_UNSUPPORTED, "%lld candidates (grids of 2^31 or more are not built)",
                    (long long)n);
    const int64_t k = count_rule(n, fraction);
    *k_out = k;
    if (capacity < k)
        return fail(NRR_ERR_BUFFER_TOO_SMALL, "capacity %lld < K = %lld", (long long)capacity,
                    (long long)k);
    if (!ref || !flt || !match_workspace || (k > 0 && (!centers || !select_workspace)))
        return fail(NRR_ERR_INVALID_ARG, "volumes, centers and workspaces must be non-NULL");
    const size_t need = nrr::select_layout(n).total;
    if (k > 0 && select_workspace_bytes < need)
        return fail(NRR_ERR_BUFFER_TOO_SMALL, "selection workspace %zu < %zu bytes",
                    select_workspace_bytes, need);
    const nrr::StatsLayout L = nrr::stats_layout(dtype, dims, block);
    if (match_workspace_bytes < L.total)
        return fail(NRR_ERR_BUFFER_TOO_SMALL, "match workspace %zu < %zu bytes",
                    match_workspace_bytes, L.total);
    const nrr::MatchArgs a = match_args(nullptr, flt, dims, nullptr, 0, block, window, nullptr,
                                        nullptr, nullptr, match_workspace, L);
    const bool pairs = plan_reads_pairs(dtype, a);
    note_pairs(match_workspace, pairs);
    const int32_t b3[3] = {block, block, block};
    hipStream_t st = static_cast<hipStream_t>(stream);
    const nrr::BoxGrid G = nrr::cubic_grid(block, stride, g);
    const nrr::SelectLayout SL = nrr::select_layout(n);
    char *sws = static_cast<char *>(select_workspace);
    uint64_t *keys = k > 0 ? reinterpret_cast<uint64_t *>(sws + SL.keys_off) : nullptr;
    if (nrr::select_stats_fusable(dtype, n, k, block)) {
        // one stream: the keys, then the select and the statistics in one
        // launch (the select's workgroup first), then the plane-pair words
        // if the plan reads them
        nrr::launch_keys(ref, dtype, dims, G, n, keys, st);
        const nrr::StatsLayout L2 = nrr::stats_layout(dtype, dims, b3, pairs);
        hipError_t e = nrr::launch_select_stats(keys, n, G, k, centers, SL, sws,
                                                static_cast<const uint16_t *>(flt), dims, block,
                                                L2, match_workspace, st);
        if (e == hipSuccess && L2.pair_off)
            e = nrr::launch_pair_volume(
                static_cast<const uint16_t *>(flt), dims,
                reinterpret_cast<uint32_t *>(static_cast<char *>(match_workspace) + L2.pair_off),
                st);
        return hip_status(e, "selection and window statistics launch");
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "device query");
    if (dev < 0 || dev >= 64) return fail(NRR_ERR_UNSUPPORTED, "device index %d (0..63 built)", dev);
    std::lock_guard<std::mutex> lk(g_fork_mu);
    ForkSet *fsp = nullptr;
    e = fork_set(&fsp);
    if (e != hipSuccess) return hip_status(e, "second stream creation");
    ForkSet &fs = *fsp;
    // keys on `stream`; then the statistics on the second stream (forked
    // here, so the selection's one-workgroup kernel, next on `stream`, is
    // placed before the statistics fill the device); `stream` joins them
    if (k > 0) nrr::launch_keys(ref, dtype, dims, G, n, keys, st);
    e = hipEventRecord(fs.fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(fs.side, fs.fork, 0);
    if (e == hipSuccess) e = nrr::launch_stats(flt, dtype, dims, b3, pairs, match_workspace, fs.side);
    if (e == hipSuccess) e = hipEventRecord(fs.join, fs.side);
    if (e == hipSuccess && k > 0) {
        nrr::select_from_keys(keys, n, G, k, nullptr, centers, SL, sws, st);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamWaitEvent(st, fs.join, 0);
    return hip_status(e, "selection and window statistics launch");
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
    // the plane-pair volume only when the planned search reads it
    const nrr::MatchArgs a =
        match_args(ref, flt, dims, centers, n, block, window, disp, ncc, conf, workspace, L);
    const bool pairs = plan_reads_pairs(dtype, a);
    note_pairs(workspace, pairs);
    const int32_t b3[3] = {block, block, block};
    hipError_t e = nrr::launch_stats(flt, dtype, dims, b3, pairs, workspace, st);
    if (e != hipSuccess) return hip_status(e, "window statistics launch");
    return run_match(ref, flt, dtype, dims, centers, n, block, window, disp, ncc, conf, workspace,
                     L, st);
}

nrr_status nrr_block_match_surface(const void *ref, const void *flt, nrr_dtype dtype,
                                   const int32_t dims[3], const int32_t *centers, int64_t n,
                                   int32_t block, int32_t window, int32_t arith, int32_t *disp,
                                   float *ncc, float *conf, float *surface, void *workspace,
                                   size_t workspace_bytes, void *stream) {
    nrr::StatsLayout L;
    nrr_status s = check_match(ref, flt, dtype, dims, centers, n, block, window, disp, ncc, conf,
                               workspace, workspace_bytes, &L);
    if (s != NRR_OK || n == 0) return s;
    if (!surface) return fail(NRR_ERR_INVALID_ARG, "surface is NULL");
    if (arith < -1 || arith > 2) return fail(NRR_ERR_INVALID_ARG, "arith must be -1..2");
    const nrr::MatchArgs a =
        match_args(ref, flt, dims, centers, n, block, window, disp, ncc, conf, workspace, L);
    if (arith < 0) {
        nrr::TileShape t;
        if (!nrr::match_plan(dtype, a, &t))
            return fail(NRR_ERR_UNSUPPORTED, "no compiled shape for block %d window %d", block,
                        window);
        arith = t.arith;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t side = 2 * (int64_t)window + 1;
    hipError_t e = nrr::launch_fill(surface, n * side * side * side, NAN, st);
    if (e != hipSuccess) return hip_status(e, "surface fill");
    note_pairs(workspace, true);
    if ((e = nrr::launch_stats(flt, dtype, dims, block, workspace, st)) != hipSuccess)
        return hip_status(e, "window statistics launch");
    e = nrr::launch_match_surface(dtype, arith, a, surface, st);
    if (e == hipErrorNotSupported)
        return fail(NRR_ERR_UNSUPPORTED, "no surface form %d for block %d window %d", arith, block,
                    window);
    return hip_status(e, "surface search launch");
}

// ------------------------------------------------------- per-axis sizes

namespace {

// Per-axis block edges (odd, 1..15), strides (>= 1, may be NULL) and the
// candidate grid they give.
nrr_status check_box(const int32_t dims[3], const int32_t block[3], const int32_t stride[3],
                     nrr::BoxGrid *G) {
    if (!dims || !block) return fail(NRR_ERR_INVALID_ARG, "dims and block must be non-NULL");
    for (int a = 0; a < 3; ++a) {
        const int32_t b = block[a], st = stride ? stride[a] : 1;
        if (b < 1 || b % 2 == 0)
            return fail(NRR_ERR_INVALID_ARG, "block[%d] must be odd and >= 1 (got %d)", a, b);
        if (b > 15) return fail(NRR_ERR_UNSUPPORTED, "block[%d] = %d: edges above 15 are not built",
                                a, b);
        if (st < 1) return fail(NRR_ERR_INVALID_ARG, "stride[%d] must be >= 1 (got %d)", a, st);
        if (dims[a] < b)
            return fail(NRR_ERR_INVALID_ARG, "dims[%d] = %d is smaller than block[%d] = %d", a,
                        dims[a], a, b);
        G->b[a] = b;
        G->s[a] = st;
        G->g[a] = (dims[a] - b) / st + 1;
    }
    return NRR_OK;
}

}  // namespace

nrr_status nrr_aniso_workspace_bytes(nrr_dtype dtype, const int32_t dims[3],
                                     const int32_t block[3], const int32_t stride[3],
                                     size_t *select_bytes, size_t *match_bytes) {
    nrr_status s = check_dtype(dtype);
    if (s != NRR_OK) return s;
    nrr::BoxGrid G;
    if ((s = check_box(dims, block, stride, &G)) != NRR_OK) return s;
    if (select_bytes)
        *select_bytes = nrr::select_layout((int64_t)G.g[0] * G.g[1] * G.g[2], true).total;
    if (match_bytes) *match_bytes = nrr::stats_layout(dtype, dims, block, false).total;
    return ok();
}

nrr_status nrr_select_blocks_aniso(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                                   const int32_t block[3], const int32_t stride[3],
                                   double fraction, int32_t *centers, int64_t capacity,
                                   int64_t *k_out, void *workspace, size_t workspace_bytes,
                                   void *stream) {
    nrr_status s = check_dtype(dtype);
    if (s != NRR_OK) return s;
    if (!k_out || !stride) return fail(NRR_ERR_INVALID_ARG, "k_out and stride must be non-NULL");
    nrr::BoxGrid G;
    if ((s = check_box(dims, block, stride, &G)) != NRR_OK) return s;
    if (!(fraction > 0.0) || fraction > 1.0)
        return fail(NRR_ERR_INVALID_ARG, "fraction must be in (0, 1] (got %g)", fraction);
    const int64_t n = (int64_t)G.g[0] * G.g[1] * G.g[2];
    if (n >= (1ll << 31))
        return fail(NRR_ERR_UNSUPPORTED, "%lld candidates (grids of 2^31 or more are not built)",
                    (long long)n);
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
    return hip_status(nrr::launch_select(vol, dtype, dims, G, k, centers, workspace,
                                         static_cast<hipStream_t>(stream)),
                      "nrr_select_blocks_aniso launch");
}

nrr_status nrr_select_count_aniso(const int32_t dims[3], const int32_t block[3],
                                  const int32_t stride[3], double fraction, int32_t grid[3],
                                  int64_t *k) {
    if (!stride || !k) return fail(NRR_ERR_INVALID_ARG, "stride and k must be non-NULL");
    nrr::BoxGrid G;
    nrr_status s = check_box(dims, block, stride, &G);
    if (s != NRR_OK) return s;
    if (!(fraction > 0.0) || fraction > 1.0)
        return fail(NRR_ERR_INVALID_ARG, "fraction must be in (0, 1] (got %g)", fraction);
    if (grid)
        for (int a = 0; a < 3; ++a) grid[a] = G.g[a];
    *k = count_rule((int64_t)G.g[0] * G.g[1] * G.g[2], fraction);
    return ok();
}

nrr_status nrr_select_blocks_aniso_ex(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                                      const int32_t block[3], const int32_t stride[3],
                                      double fraction, const uint8_t *mask, int32_t connectivity,
                                      int32_t *centers, int64_t capacity, int64_t *k_device,
                                      void *workspace, size_t workspace_bytes, void *stream) {
    nrr_status s = check_dtype(dtype);
    if (s != NRR_OK) return s;
    if (!stride) return fail(NRR_ERR_INVALID_ARG, "stride must be non-NULL");
    nrr::BoxGrid G;
    if ((s = check_box(dims, block, stride, &G)) != NRR_OK) return s;
    if (!(fraction > 0.0) || fraction > 1.0)
        return fail(NRR_ERR_INVALID_ARG, "fraction must be in (0, 1] (got %g)", fraction);
    if (connectivity != 0 && connectivity != 6 && connectivity != 18 && connectivity != 26)
        return fail(NRR_ERR_INVALID_ARG, "connectivity must be 0, 6, 18 or 26 (got %d)",
                    connectivity);
    if (!vol || !centers || !k_device || !workspace)
        return fail(NRR_ERR_INVALID_ARG, "vol, centers, k_device and workspace must be non-NULL");
    const int64_t n = (int64_t)G.g[0] * G.g[1] * G.g[2];
    if (n >= (1ll << 31))
        return fail(NRR_ERR_UNSUPPORTED, "%lld candidates (limit 2^31)", (long long)n);
    const int64_t kmax = count_rule(n, fraction);
    if (capacity < kmax)
        return fail(NRR_ERR_BUFFER_TOO_SMALL, "capacity %lld < %lld", (long long)capacity,
                    (long long)kmax);
    const nrr::SelectLayout L = nrr::select_layout(n, true);
    if (workspace_bytes < L.total)
        return fail(NRR_ERR_BUFFER_TOO_SMALL, "workspace %zu < %zu bytes", workspace_bytes,
                    L.total);
    return hip_status(nrr::launch_select_ex(vol, dtype, dims, G, fraction, mask, connectivity,
                                            centers, k_device, workspace,
                                            static_cast<hipStream_t>(stream)),
                      "nrr_select_blocks_aniso_ex launch");
}

namespace {

// Validation shared by the per-axis search entry points; fills the layout.
nrr_status check_aniso(const void *ref, const void *flt, nrr_dtype dtype, const int32_t dims[3],
                       const int32_t *centers, int64_t n, const int32_t block[3],
                       const int32_t window[3], const int32_t *disp, const float *ncc,
                       const float *conf, const void *workspace, size_t workspace_bytes,
                       nrr::StatsLayout *L) {
    nrr_status s = check_dtype(dtype);
    if (s != NRR_OK) return s;
    nrr::BoxGrid G;
    if ((s = check_box(dims, block, nullptr, &G)) != NRR_OK) return s;
    if (!window) return fail(NRR_ERR_INVALID_ARG, "window is NULL");
    for (int a = 0; a < 3; ++a)
        if (window[a] < 0)
            return fail(NRR_ERR_INVALID_ARG, "window[%d] must be >= 0 (got %d)", a, window[a]);
    if (n < 0) return fail(NRR_ERR_INVALID_ARG, "n must be >= 0 (got %lld)", (long long)n);
    if (n > INT32_MAX) return fail(NRR_ERR_UNSUPPORTED, "more than 2^31 - 1 blocks");
    const char *why = nrr::aniso_unsupported_reason(block, window);
    if (why)
        return fail(NRR_ERR_UNSUPPORTED, "block (%d,%d,%d) window (%d,%d,%d): %s", block[0],
                    block[1], block[2], window[0], window[1], window[2], why);
    if (n == 0) return NRR_OK;
    if (!ref || !flt || !centers || !disp || !ncc || !conf || !workspace)
        return fail(NRR_ERR_INVALID_ARG, "array and workspace pointers must be non-NULL");
    if ((int64_t)dims[0] * dims[1] * dims[2] >= (1ll << 40))
        return fail(NRR_ERR_UNSUPPORTED, "volume too large");
    *L = nrr::stats_layout(dtype, dims, block, false);
    if (workspace_bytes < L->total)
        return fail(NRR_ERR_BUFFER_TOO_SMALL, "workspace %zu < %zu bytes", workspace_bytes,
                    L->total);
    return NRR_OK;
}

nrr_status run_aniso(const void *ref, const void *flt, nrr_dtype dtype, const int32_t dims[3],
                     const int32_t *centers, int64_t n, const int32_t block[3],
                     const int32_t window[3], int32_t *disp, float *ncc, float *conf,
                     const void *workspace, const nrr::StatsLayout &L, hipStream_t st) {
    nrr::AnisoArgs a;
    a.ref = ref;
    a.flt = flt;
    a.nx = dims[0];
    a.ny = dims[1];
    a.nz = dims[2];
    a.centers = centers;
    a.n = n;
    for (int i = 0; i < 3; ++i) {
        a.b[i] = block[i];
        a.w[i] = window[i];
    }
    a.stats = workspace;
    a.ox = L.ox;
    a.oy = L.oy;
    a.disp = disp;
    a.ncc = ncc;
    a.conf = conf;
    a.cz = 0;
    return hip_status(nrr::launch_match_aniso(dtype, a, st), "per-axis search launch");
}

}  // namespace

nrr_status nrr_block_match_aniso(const void *ref, const void *flt, nrr_dtype dtype,
                                 const int32_t dims[3], const int32_t *centers, int64_t n,
                                 const int32_t block[3], const int32_t window[3], int32_t *disp,
                                 float *ncc, float *conf, void *workspace, size_t workspace_bytes,
                                 void *stream) {
    nrr::StatsLayout L;
    nrr_status s = check_aniso(ref, flt, dtype, dims, centers, n, block, window, disp, ncc, conf,
                               workspace, workspace_bytes, &L);
    if (s != NRR_OK || n == 0) return s == NRR_OK ? ok() : s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = nrr::launch_stats(flt, dtype, dims, block, false, workspace, st);
    if (e != hipSuccess) return hip_status(e, "window statistics launch");
    return run_aniso(ref, flt, dtype, dims, centers, n, block, window, disp, ncc, conf, workspace,
                     L, st);
}

nrr_status nrr_window_stats_aniso(const void *flt, nrr_dtype dtype, const int32_t dims[3],
                                  const int32_t block[3], void *workspace,
                                  size_t workspace_bytes, void *stream) {
    nrr_status s = check_dtype(dtype);
    if (s != NRR_OK) return s;
    nrr::BoxGrid G;
    if ((s = check_box(dims, block, nullptr, &G)) != NRR_OK) return s;
    if (!flt || !workspace) return fail(NRR_ERR_INVALID_ARG, "flt and workspace must be non-NULL");
    const nrr::StatsLayout L = nrr::stats_layout(dtype, dims, block, false);
    if (workspace_bytes < L.total)
        return fail(NRR_ERR_BUFFER_TOO_SMALL, "workspace %zu < %zu bytes", workspace_bytes,
                    L.total);
    return hip_status(nrr::launch_stats(flt, dtype, dims, block, false, workspace,
                                        static_cast<hipStream_t>(stream)),
                      "window statistics launch");
}

nrr_status nrr_block_match_aniso_prepared(const void *ref, const void *flt, nrr_dtype dtype,
                                          const int32_t dims[3], const int32_t *centers,
                                          int64_t n, const int32_t block[3],
                                          const int32_t window[3], int32_t *disp, float *ncc,
                                          float *conf, const void *workspace,
                                          size_t workspace_bytes, void *stream) {
    nrr::StatsLayout L;
    nrr_status s = check_aniso(ref, flt, dtype, dims, centers, n, block, window, disp, ncc, conf,
                               workspace, workspace_bytes, &L);
    if (s != NRR_OK || n == 0) return s == NRR_OK ? ok() : s;
    return run_aniso(ref, flt, dtype, dims, centers, n, block, window, disp, ncc, conf, workspace,
                     L, static_cast<hipStream_t>(stream));
}

nrr_status nrr_check_volume(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                            int64_t *bad_device, void *stream) {
    nrr_status s = check_dtype(dtype);
    if (s != NRR_OK) return s;
    if (!dims || !vol || !bad_device)
        return fail(NRR_ERR_INVALID_ARG, "vol, dims and bad_device must be non-NULL");
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 1) return fail(NRR_ERR_INVALID_ARG, "dims[%d] must be >= 1", a);
    const int64_t n = (int64_t)dims[0] * dims[1] * dims[2];
    return hip_status(nrr::launch_check_volume(vol, dtype, n, bad_device,
                                               static_cast<hipStream_t>(stream)),
                      "volume check launch");
}

nrr_status nrr_structure_confidence(const void *ref, nrr_dtype dtype, const int32_t dims[3],
                                    const int32_t *centers, int64_t n, int32_t block,
                                    const float *conf, float *out, void *stream) {
    nrr_status s = check_dtype(dtype);
    if (s != NRR_OK) return s;
    int32_t g[3];
    if ((s = check_grid(dims, block, 1, g)) != NRR_OK) return s;
    if (n < 0) return fail(NRR_ERR_INVALID_ARG, "n must be >= 0");
    if (n == 0) return ok();
    if (!ref || !centers || !conf || !out)
        return fail(NRR_ERR_INVALID_ARG, "ref, centers, conf and out must be non-NULL");
    return hip_status(nrr::launch_structure_conf(ref, dtype, dims, centers, n, block, conf, out,
                                                 static_cast<hipStream_t>(stream)),
                      "structure confidence launch");
}

// ------------------------------------------------------------------ tuning

nrr_status nrr_tune_match(const void *ref, const void *flt, nrr_dtype dtype,
                          const int32_t dims[3], const int32_t *centers, int64_t n, int32_t block,
                          int32_t window, int32_t *disp, float *ncc, float *conf,
                          const void *workspace, size_t workspace_bytes, int32_t reps,
                          nrr_tile_shape *best, double *best_us, void *stream) {
    if (reps < 1) return fail(NRR_ERR_INVALID_ARG, "reps must be >= 1 (got %d)", reps);
    nrr::StatsLayout L;
    nrr_status s = check_match(ref, flt, dtype, dims, centers, n, block, window, disp, ncc, conf,
                               workspace, workspace_bytes, &L);
    if (s != NRR_OK) return s;
    if (n == 0) return fail(NRR_ERR_INVALID_ARG, "n must be > 0 to time the search");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const nrr::MatchArgs a =
        match_args(ref, flt, dims, centers, n, block, window, disp, ncc, conf, workspace, L);
    nrr::TileShape shapes[64];
    const int ns = nrr::match_shapes(dtype, block, window, shapes, 64);
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return hip_status(e, "tuner event");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        hipEventDestroy(e0);
        return hip_status(e, "tuner event");
    }
    double bt = std::numeric_limits<double>::infinity();
    int bi = -1;
    for (int i = 0; i < ns && e == hipSuccess; ++i) {
        if ((e = nrr::launch_match(dtype, a, st, &shapes[i])) != hipSuccess) break;  // warm-up
        if ((e = hipEventRecord(e0, st)) != hipSuccess) break;
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = nrr::launch_match(dtype, a, st, &shapes[i]);
        if (e != hipSuccess) break;
        if ((e = hipEventRecord(e1, st)) != hipSuccess) break;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0.0f;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        const double us = 1000.0 * ms / reps;
        if (us < bt) {
            bt = us;
            bi = i;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess) return hip_status(e, "tuner trial");
    if (bi < 0) return fail(NRR_ERR_UNSUPPORTED, "no compiled shape for block %d window %d", block,
                            window);
    // leave the outputs as the chosen shape computes them
    nrr::set_tuned_shape(dtype, block, window, shapes[bi]);
    if ((e = nrr::launch_match(dtype, a, st, &shapes[bi])) != hipSuccess)
        return hip_status(e, "block match launch");
    if (best) {
        const nrr::TileShape &t = shapes[bi];
        *best = nrr_tile_shape{t.arith, t.rx, t.ry, t.nt, t.pf, t.cz};
    }
    if (best_us) *best_us = bt;
    return ok();
}

nrr_status nrr_tuned_shape(nrr_dtype dtype, int32_t block, int32_t window, nrr_tile_shape *out) {
    nrr::TileShape t;
    if (!out) return fail(NRR_ERR_INVALID_ARG, "out is NULL");
    if (!nrr::tuned_shape(dtype, block, window, &t))
        return fail(NRR_ERR_UNSUPPORTED, "no tuned shape for block %d window %d", block, window);
    *out = nrr_tile_shape{t.arith, t.rx, t.ry, t.nt, t.pf, t.cz};
    return ok();
}

nrr_status nrr_clear_tuning(void) {
    nrr::clear_tuned_shapes();
    return ok();
}

nrr_status nrr_match_shapes(nrr_dtype dtype, int32_t block, int32_t window, nrr_tile_shape *out,
                            int32_t cap, int32_t *count) {
    if (!count || (cap > 0 && !out))
        return fail(NRR_ERR_INVALID_ARG, "count (and out when cap > 0) must be non-NULL");
    nrr_status s = nrr_match_supported(dtype, block, window);
    if (s != NRR_OK) return s;
    nrr::TileShape shapes[64];
    const int ns = nrr::match_shapes(dtype, block, window, shapes, 64);
    for (int i = 0; i < ns && i < cap; ++i) {
        const nrr::TileShape &t = shapes[i];
        out[i] = nrr_tile_shape{t.arith, t.rx, t.ry, t.nt, t.pf, t.cz};
    }
    *count = ns;
    return ok();
}

nrr_status nrr_set_tuned_shape(nrr_dtype dtype, int32_t block, int32_t window,
                               const nrr_tile_shape *shape) {
    if (!shape) return fail(NRR_ERR_INVALID_ARG, "shape is NULL");
    nrr_status s = nrr_match_supported(dtype, block, window);
    if (s != NRR_OK) return s;
    const nrr::TileShape t{shape->arith, shape->rx, shape->ry, shape->nt, shape->pf, shape->cz};
    if (t.cz < 0) return fail(NRR_ERR_INVALID_ARG, "cz must be >= 0 (got %d)", t.cz);
    if (!nrr::shape_known(dtype, block, window, t))
        return fail(NRR_ERR_UNSUPPORTED,
                    "shape (arith %d, %dx%d, %d threads, pf %d) is not compiled for block %d "
                    "window %d", t.arith, t.rx, t.ry, t.nt, t.pf, block, window);
    nrr::set_tuned_shape(dtype, block, window, t);
    return ok();
}

}  // extern "C"

// ---------------------------------------------------------- batched search

struct nrr_batch_plan {
    const void *ref = nullptr, *flt = nullptr;
    nrr_dtype dtype = NRR_F32;
    int32_t dims[3] = {0, 0, 0};
    BatchLayout L;
    char *ws = nullptr;
    int32_t nsets = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// The window statistics of every block size of a batch on `st`.
hipError_t batch_stats(const nrr_batch_plan &P, hipStream_t st) {
    const size_t nb = P.L.bvals.size();
    if (P.dtype == NRR_F32 && nb >= 1 && nb <= (size_t)nrr::kStatsJobs) {
        void *outs[nrr::kStatsJobs];
        for (size_t i = 0; i < nb; ++i) outs[i] = P.ws + P.L.stats_off[i];
        return nrr::launch_stats_f32_multi(static_cast<const float *>(P.flt), P.dims,
                                           P.L.bvals.data(), outs, (int)nb, st);
    }
    for (size_t i = 0; i < nb; ++i) {
        hipError_t e = nrr::launch_stats(P.flt, P.dtype, P.dims, P.L.bvals[i],
                                         P.ws + P.L.stats_off[i], st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The launches of one batch on `st`: the window statistics (read `flt`) on the
// library's second stream, beside the batched selection (reads `ref`) on
// `st`; `st` joins them before the persistent search.
hipError_t batch_enqueue(const nrr_batch_plan &P, hipStream_t st) {
    if (P.nsets == 0) return batch_stats(P, st);
    std::lock_guard<std::mutex> lk(g_fork_mu);
    ForkSet *fs = nullptr;
    hipError_t e = fork_set(&fs);
    if (e == hipSuccess) e = hipEventRecord(fs->fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(fs->side, fs->fork, 0);
    if (e == hipSuccess) e = batch_stats(P, fs->side);
    if (e == hipSuccess) e = hipEventRecord(fs->join, fs->side);
    if (e == hipSuccess)
        e = nrr::launch_select_batch(
            P.ref, P.dtype, P.dims,
            reinterpret_cast<const nrr::BatchSelectSet *>(P.ws + P.L.sel_off), P.nsets,
            P.L.max_cand, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, fs->join, 0);
    if (e != hipSuccess) return e;
    return nrr::launch_match_batch(P.dtype,
                                   reinterpret_cast<const nrr::BatchSet *>(P.ws + P.L.sets_off),
                                   P.nsets, P.L.nitems, P.L.lds, st);
}

}  // namespace

extern "C" {

nrr_status nrr_batch_layout(nrr_dtype dtype, const int32_t dims[3], const nrr_param_set *sets,
                            int32_t nsets, int64_t *offsets, size_t *workspace_bytes) {
    BatchLayout L;
    nrr_status s = batch_layout(dtype, dims, sets, nsets, &L);
    if (s != NRR_OK) return s;
    if (offsets) std::copy(L.off.begin(), L.off.end(), offsets);
    if (workspace_bytes) *workspace_bytes = L.total;
    return ok();
}

nrr_status nrr_batch_shapes(nrr_dtype dtype, const int32_t dims[3], const nrr_param_set *sets,
                            int32_t nsets, nrr_tile_shape *out) {
    BatchLayout L;
    nrr_status s = batch_layout(dtype, dims, sets, nsets, &L);
    if (s != NRR_OK) return s;
    if (nsets > 0 && !out) return fail(NRR_ERR_INVALID_ARG, "out is NULL");
    for (int32_t i = 0; i < nsets; ++i) {
        nrr::TileShape t;
        if (!nrr::batch_variant_shape(dtype, L.variant[i], L.cz[i], &t))
            return fail(NRR_ERR_UNSUPPORTED, "set %d: no batched shape", i);
        out[i] = nrr_tile_shape{t.arith, t.rx, t.ry, t.nt, t.pf, t.cz};
    }
    return ok();
}

nrr_status nrr_batch_plan_create(const void *ref, const void *flt, nrr_dtype dtype,
                                 const int32_t dims[3], const nrr_param_set *sets, int32_t nsets,
                                 int32_t *centers, int32_t *disp, float *ncc, float *conf,
                                 void *workspace, size_t workspace_bytes, int32_t use_graph,
                                 void *stream, nrr_batch_plan **plan) {
    if (!plan) return fail(NRR_ERR_INVALID_ARG, "plan is NULL");
    *plan = nullptr;
    nrr_batch_plan *P = new nrr_batch_plan;
    nrr_status s = batch_layout(dtype, dims, sets, nsets, &P->L);
    if (s != NRR_OK) {
        delete P;
        return s;
    }
    const int64_t rows = P->L.off.back();
    if (!ref || !flt || !workspace || (rows > 0 && (!centers || !disp || !ncc || !conf))) {
        delete P;
        return fail(NRR_ERR_INVALID_ARG, "volume, output and workspace pointers must be non-NULL");
    }
    if (workspace_bytes < P->L.total) {
        const size_t need = P->L.total;
        delete P;
        return fail(NRR_ERR_BUFFER_TOO_SMALL, "workspace %zu < %zu bytes", workspace_bytes, need);
    }
    P->ref = ref;
    P->flt = flt;
    P->dtype = dtype;
    std::copy(dims, dims + 3, P->dims);
    P->ws = static_cast<char *>(workspace);
    P->nsets = nsets;
    // set tables: selection in the caller's order, search by falling cost
    std::vector<nrr::BatchSelectSet> sel(nsets);
    std::vector<nrr::BatchSet> bs(nsets);
    std::vector<int> order(nsets);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return P->L.cost[x] > P->L.cost[y]; });
    int64_t item = 0;
    std::vector<int64_t> key_at(nsets + 1, 0);
    for (int i = 0; i < nsets; ++i) key_at[i + 1] = key_at[i] + P->L.ncand[i];
    for (int j = 0; j < nsets; ++j) {
        const int i = order[j];
        const nrr_param_set &q = sets[i];
        const int64_t off = P->L.off[i];
        nrr::BatchSelectSet &t = sel[i];
        t.b = q.block;
        t.stride = q.stride;
        t.gx = P->L.grid[3 * i];
        t.gy = P->L.grid[3 * i + 1];
        t.gz = P->L.grid[3 * i + 2];
        t.pad = 0;
        t.ncand = P->L.ncand[i];
        t.k = P->L.k[i];
        t.centers = centers ? centers + 3 * off : nullptr;
        t.keys = reinterpret_cast<uint64_t *>(P->ws + P->L.keys_off) + key_at[i];
        const size_t bi =
            std::find(P->L.bvals.begin(), P->L.bvals.end(), q.block) - P->L.bvals.begin();
        const nrr::StatsLayout SL = nrr::stats_layout(dtype, dims, q.block);
        const char *stats = P->ws + P->L.stats_off[bi];
        nrr::BatchSet &b = bs[j];
        b.a = match_args(ref, flt, dims, t.centers, t.k, q.block, q.window,
                         disp ? disp + 3 * off : nullptr, ncc ? ncc + off : nullptr,
                         conf ? conf + off : nullptr, stats, SL);
        b.cz = P->L.cz[i];
        b.variant = P->L.variant[i];
        b.first_item = item;
        item += t.k;
    }
    hipError_t e = hipSuccess;
    if (nsets > 0) {
        e = hipMemcpy(P->ws + P->L.sel_off, sel.data(), sizeof(nrr::BatchSelectSet) * nsets,
                      hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(P->ws + P->L.sets_off, bs.data(), sizeof(nrr::BatchSet) * nsets,
                          hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && use_graph) {
        {  // the second stream exists before the capture begins
            std::lock_guard<std::mutex> lk(g_fork_mu);
            ForkSet *fs = nullptr;
            e = fork_set(&fs);
        }
        hipStream_t cs = nullptr;
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) {
            e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                const hipError_t ee = batch_enqueue(*P, cs);
                e = hipStreamEndCapture(cs, &P->graph);
                if (ee != hipSuccess) e = ee;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
            hipStreamDestroy(cs);
        }
    }
    (void)stream;
    if (e != hipSuccess) {
        nrr_batch_plan_destroy(P);
        return hip_status(e, "batch plan");
    }
    *plan = P;
    return ok();
}

nrr_status nrr_batch_plan_run(nrr_batch_plan *plan, void *stream) {
    if (!plan) return fail(NRR_ERR_INVALID_ARG, "plan is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (plan->exec) return hip_status(hipGraphLaunch(plan->exec, st), "batch graph launch");
    return hip_status(batch_enqueue(*plan, st), "batch launch");
}

nrr_status nrr_batch_plan_destroy(nrr_batch_plan *plan) {
    if (!plan) return ok();
    if (plan->exec) hipGraphExecDestroy(plan->exec);
    if (plan->graph) hipGraphDestroy(plan->graph);
    delete plan;
    return ok();
}

}  // extern "C"
