// Internal declarations shared by the C-ABI layer and the HIP kernels of
// libnrr.so.  Not installed; the public interface is include/nrr.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "nrr.h"

namespace nrr {

// Records the detail nrr_last_error returns (printf format); returns s.
nrr_status set_error(nrr_status s, const char *fmt, ...);

// ------------------------------------------------------------- selection
// Workspace of the selection: one 64-bit ranking key per candidate block,
// the radix-select state and per-tile counts for the ordered compaction.
constexpr int kSelectTile = 2048;  // candidates per compaction workgroup

struct SelectLayout {
    size_t keys_off, state_off, tiles_off, total;
    size_t radix_rows_off;                          // 0: one-workgroup radix select
    size_t ex_ctr_off, ex_state_off, ex_above_off;  // selection variants, large grids
    int64_t n_tiles;
};
// Grids of more candidates take the multi-workgroup radix select.
constexpr int64_t kRadixMultiMin = 1 << 15;
// variants: room for the selection variants on large grids as well
SelectLayout select_layout(int64_t n_candidates, bool variants = false);

// Candidate grid: per-axis block edge b, stride s and candidate count g
// (x, y, z); centre of candidate i on an axis = i * s + (b - 1) / 2.
struct BoxGrid {
    int32_t b[3], s[3], g[3];
};
BoxGrid cubic_grid(int32_t block, int32_t stride, const int32_t grid[3]);
// Ranking keys (selection order) of every candidate of G into keys[n].
void launch_keys(const void *vol, nrr_dtype dtype, const int32_t dims[3], const BoxGrid &G,
                 int64_t n, uint64_t *keys, hipStream_t stream);

hipError_t launch_select(const void *vol, nrr_dtype dtype, const int32_t dims[3], int32_t block,
                         int32_t stride, const int32_t grid[3], int64_t k, int32_t *centers,
                         void *workspace, hipStream_t stream);
hipError_t launch_select(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                         const BoxGrid &G, int64_t k, int32_t *centers, void *workspace,
                         hipStream_t stream);

// Selection with a candidate mask and a connectivity pattern (0, 6, 18, 26);
// the number taken goes to *k_device.  Grids of at most kSelectExCand
// candidates run in one workgroup (asynchronously); larger grids in round
// launches with a wait on the stream after each.
constexpr int64_t kSelectExCand = 24576;
hipError_t launch_select_ex(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                            int32_t block, int32_t stride, const int32_t grid[3], double fraction,
                            const uint8_t *mask, int32_t connectivity, int32_t *centers,
                            int64_t *k_device, void *workspace, hipStream_t stream);
hipError_t launch_select_ex(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                            const BoxGrid &G, double fraction, const uint8_t *mask,
                            int32_t connectivity, int32_t *centers, int64_t *k_device,
                            void *workspace, hipStream_t stream);
hipError_t launch_select_ex_large(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                                  const BoxGrid &G, double fraction, const uint8_t *mask,
                                  int32_t connectivity, int32_t *centers, int64_t *k_device,
                                  void *workspace, hipStream_t stream);
// The K best keys' candidates as centres in ascending grid index (K = k, or
// *kd when kd is given).
void select_from_keys(const uint64_t *keys, int64_t n, const BoxGrid &G, int64_t k,
                      const int64_t *kd, int32_t *centers, const SelectLayout &L, char *ws,
                      hipStream_t stream);

// Batched selection (one workgroup per parameter set) for candidate grids of
// at most kBatchCand blocks; `centers` points at the set's K output rows.
constexpr int kBatchCand = 4096;
struct BatchSelectSet {
    int32_t b, stride, gx, gy, gz;
    int32_t pad;
    int64_t ncand, k;
    uint64_t *keys;  // scratch, ncand ranking keys
    int32_t *centers;
};
// max_cand: the largest ncand of the sets (sizes the key launch).
hipError_t launch_select_batch(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                               const BatchSelectSet *sets, int nsets, int64_t max_cand,
                               hipStream_t stream);

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

// Count of voxels outside the dtype's contract into the device int64 *bad.
hipError_t launch_check_volume(const void *vol, nrr_dtype dtype, int64_t n, int64_t *bad,
                               hipStream_t stream);
// The plane-pair volume of a 12-bit volume alone (what the dot2 search reads).
hipError_t launch_pair_volume(const uint16_t *flt, const int32_t dims[3], uint32_t *pairs,
                              hipStream_t stream);
hipError_t launch_stats(const void *flt, nrr_dtype dtype, const int32_t dims[3], int32_t block,
                        void *workspace, hipStream_t stream);
// Per-axis block (bx, by, bz); `pairs`: also the plane-pair volume (12-bit).
StatsLayout stats_layout(nrr_dtype dtype, const int32_t dims[3], const int32_t block[3],
                         bool pairs);
hipError_t launch_stats(const void *flt, nrr_dtype dtype, const int32_t dims[3],
                        const int32_t block[3], bool pairs, void *workspace, hipStream_t stream);

// Directional confidence per block: out[n][6] = conf * J / trace(J).
hipError_t launch_structure_conf(const void *ref, nrr_dtype dtype, const int32_t dims[3],
                                 const int32_t *centers, int64_t n, int32_t block,
                                 const float *conf, float *out, hipStream_t stream);

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

// Search with per-axis block edges b and half windows w (x, y, z); `stats`
// is the statistics table of the bx x by x bz block (no plane-pair volume);
// cz is set by the launcher.
struct AnisoArgs {
    const void *ref;
    const void *flt;
    int32_t nx, ny, nz;
    const int32_t *centers;
    int64_t n;
    int32_t b[3], w[3];
    const void *stats;
    int32_t ox, oy;
    int32_t *disp;
    float *ncc;
    float *conf;
    int32_t cz;  // displacement planes per LDS run
};
const char *aniso_unsupported_reason(const int32_t block[3], const int32_t window[3]);
hipError_t launch_match_aniso(nrr_dtype dtype, const AnisoArgs &a, hipStream_t stream);

// ------------------------------------------------------- batched matching
// One parameter set of a batched search: its arguments (centres and outputs
// already offset to the set's rows), z-chunk, compiled tile shape and first
// work item (items = the set's blocks, sets ordered by falling cost).
struct BatchSet {
    MatchArgs a;
    int32_t cz, variant;
    int64_t first_item;
};
// Tile shape, z-chunk and LDS bytes of one set in the batched kernel; false
// when no compiled batched shape serves (dtype, block, window).
bool plan_batch_set(nrr_dtype dtype, int32_t block, int32_t window, int32_t *variant,
                    int32_t *cz, size_t *lds, double *cost_per_block);
// Persistent launch over all sets' blocks: `grid` workgroups stride the work
// items; `lds` is the largest set's need.
hipError_t launch_match_batch(nrr_dtype dtype, const BatchSet *sets, int32_t nsets,
                              int64_t nitems, size_t lds, hipStream_t stream);

// A compiled search shape: arithmetic (0 dot2, 1 FMA, 2 MFMA, -1 any), tile rx x ry
// (0: any), threads, record prefetch (-1 any) and z-chunk cap (0: planned).
struct TileShape {
    int32_t arith, rx, ry, nt, pf, cz;
};
// The search in form `arith` (0 dot2, 1 FMA, 2 MFMA) also writing the
// ranking NCC of every valid displacement to surface[n][2w+1]^3 (a
// diagnostic; hipErrorNotSupported when no such instantiation serves).
hipError_t launch_match_surface(nrr_dtype dtype, int32_t arith, const MatchArgs &a,
                                float *surface, hipStream_t stream);
// p[0..n) = v on the stream (a kernel, no memset).
hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t stream);
// The shape launch_match would use now (arith 0 dot2, 1 FMA, 2 MFMA); false
// when no compiled shape serves.
bool match_plan(nrr_dtype dtype, const MatchArgs &a, TileShape *out);
// Whether `sh` (cz ignored) is a compiled plain or batched shape for
// (dtype, block, window).
bool shape_known(nrr_dtype dtype, int32_t block, int32_t window, const TileShape &sh);
// The shape of a batched set planned as `variant` with z-chunk cz.
bool batch_variant_shape(nrr_dtype dtype, int32_t variant, int32_t cz, TileShape *out);
// `shape` (optional) forces the shape; else env overrides, tuned table, cost model.
hipError_t launch_match(nrr_dtype dtype, const MatchArgs &a, hipStream_t stream,
                        const TileShape *shape = nullptr);
// The shapes worth timing for (dtype, block, window); returns how many (<= cap).
int match_shapes(nrr_dtype dtype, int32_t block, int32_t window, TileShape *out, int cap);
// Process-wide table of tuned shapes used by every later launch.
bool tuned_shape(nrr_dtype dtype, int32_t block, int32_t window, TileShape *sh);
void set_tuned_shape(nrr_dtype dtype, int32_t block, int32_t window, const TileShape &sh);
void clear_tuned_shapes();

// The matrix-core form of the search (12-bit data, block edges 3-9, whole
// window in LDS): whether it serves (dtype, block, window), and its launch.
bool mfma_supported(nrr_dtype dtype, int32_t block, int32_t window);
bool mfma_fits(const MatchArgs &a);  // volume small enough for its 32-bit indices
// surface (optional): [n][2w+1]^3 ranking NCC of every valid displacement
// (a diagnostic instantiation; entries of invalid displacements untouched).
hipError_t launch_match_mfma(const MatchArgs &a, hipStream_t stream, float *surface = nullptr);
constexpr int32_t kArithMfma = 2;  // TileShape::arith of the matrix-core form

// LDS bytes per workgroup available on the current device (cached).
size_t device_lds_limit();

}  // namespace nrr
