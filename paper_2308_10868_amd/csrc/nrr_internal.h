// Internal declarations shared by the C-ABI layer and the HIP kernels of
// libnrr.so.  Not installed; the public interface is include/nrr.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "nrr.h"

namespace nrr {

// ------------------------------------------------------------- selection
// Workspace of the selection: one 64-bit ranking key per candidate block,
// the radix-select state and per-tile counts for the ordered compaction.
constexpr int kSelectTile = 2048;  // candidates per compaction workgroup

struct SelectLayout {
    size_t keys_off, state_off, tiles_off, total;
    int64_t n_tiles;
};
SelectLayout select_layout(int64_t n_candidates);

hipError_t launch_select(const void *vol, nrr_dtype dtype, const int32_t dims[3], int32_t block,
                         int32_t stride, const int32_t grid[3], int64_t k, int32_t *centers,
                         void *workspace, hipStream_t stream);

// ---------------------------------------------------------- window stats
// Per-voxel statistics of the displaced block whose origin (lowest corner)
// is that voxel, over the origin grid O = dims - block + 1, one record per
// origin (interleaved so the search reads one record per displacement):
//   u16: s = sum (F - 2048) (exact), r = 1/sqrt(N*sum (F-2048)^2 - s^2)
//        (ranking only; 0 for a flat block)
//   f32: s = sum F, r = 1/sqrt(N*sum F^2 - s^2) (0 for a flat block)
struct StatU16 {
    int32_t s;
    float r;
};
struct StatF32 {
    double s;
    double r;
};
// 12-bit volumes also get a plane-pair copy of `flt` for the dot2 search:
// pairs[z][y][x] = (F(z) - 2048) | (F(z+1) - 2048) << 16 as two int16 halves
// (upper half 0 on the last plane), 4 bytes per voxel at byte `pair_off`.
constexpr int kTileSlack = 16;  // >= the largest search tile edge
struct StatsLayout {
    size_t total;
    size_t pair_off;  // 0: no pair volume (float data)
    int32_t ox, oy, oz;
};
StatsLayout stats_layout(nrr_dtype dtype, const int32_t dims[3], int32_t block);

hipError_t launch_stats(const void *flt, nrr_dtype dtype, const int32_t dims[3], int32_t block,
                        void *workspace, hipStream_t stream);

// -------------------------------------------------------------- matching
struct MatchArgs {
    const void *ref;
    const void *flt;
    int32_t nx, ny, nz;
    const int32_t *centers;
    int64_t n;
    int32_t block, window;
    const void *stats;   // StatU16 or StatF32 records, [oz][oy][ox]
    const uint32_t *pairs;  // plane-pair volume (12-bit data), else nullptr
    int32_t ox, oy;      // origin-grid extents (x, y) of the stats arrays
    int32_t *disp;
    float *ncc;
    float *conf;
};

// Returns 0 when supported, else a static reason string.
const char *match_unsupported_reason(nrr_dtype dtype, int32_t block, int32_t window);

hipError_t launch_match(nrr_dtype dtype, const MatchArgs &a, hipStream_t stream);

// LDS bytes per workgroup available on the current device (cached).
size_t device_lds_limit();

}  // namespace nrr
