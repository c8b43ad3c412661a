/*
 * nrr.h -- C ABI of libnrr.so: GPU block matching for physics-based
 * non-rigid registration (MI355X / gfx950).
 *
 * The library implements the data-parallel block-matching stage of the
 * registration method ("Physics-Based Non-Rigid Registration" section of
 * the paper): registration points are chosen where the intensity variance of
 * the surrounding block is high (selection, "Parallel feature selection"
 * paragraph of the HPC section), and for each point an exhaustive search
 * over a window of integer displacements finds the displacement that
 * maximises the normalised cross-correlation (the NCC equation) between the
 * pre-operative block and the displaced block of the intra-operative volume
 * (the GPU block-matching algorithm of the GPU section).
 *
 * Naming: `ref` is the pre-operative volume (blocks are taken from it),
 * `flt` the intra-operative volume (the search window lies in it).  With
 * flt(p) = ref(p - s) the displacement returned is +s.
 *
 * Conventions shared by every entry point:
 *  - volumes are dense C-order [z][y][x] arrays; dims = {nx, ny, nz};
 *  - vectors (centres, displacements) are int32 (x, y, z) triples;
 *  - `block` is the full odd block edge b (>= 3), h = (b-1)/2; a block
 *    centred at c covers c + o, o in [-h, h]^3;
 *  - the search window is +-`window` voxels per axis; only displacements
 *    whose displaced block lies fully inside the volume are evaluated;
 *  - NCC is the Pearson correlation over the block's voxels; it is 0 when
 *    the block or the displaced block is constant;
 *  - among equal NCC values the displacement with the smallest shift index
 *    ((dz+W)(2W+1) + (dy+W))(2W+1) + (dx+W) wins;
 *  - NRR_U16 volumes hold 12-bit intensities (0..4095); NRR_F32 volumes
 *    hold finite floats.
 *
 * Memory and streams: every array argument documented "device" is a device
 * pointer owned by the caller; apart from the registration server (one
 * allocation of the size given at nrr_server_create, freed by
 * nrr_server_destroy) and the fixed static array of the allocation-free
 * selection entry point, the library allocates no device memory, and it
 * keeps no reference to caller memory after returning.  Work is enqueued on `stream` (a
 * hipStream_t passed as void*, NULL = the default stream) and the call
 * returns without synchronising; outputs are valid after the caller
 * synchronises the stream, and inputs/workspace must stay alive until then.
 * Calls on different streams with different workspaces may run concurrently.
 *
 * Errors: every entry point returns an nrr_status and never aborts.  Host-
 * checkable argument errors are reported synchronously and nothing is
 * enqueued; nrr_last_error() then holds a thread-local message.
 */
#ifndef NRR_H
#define NRR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NRR_OK = 0,
    NRR_ERR_INVALID_ARG = 1,      /* bad size, null pointer, out-of-range parameter */
    NRR_ERR_BUFFER_TOO_SMALL = 2, /* output capacity or workspace too small */
    NRR_ERR_HIP = 3,              /* a HIP runtime call or kernel launch failed */
    NRR_ERR_UNSUPPORTED = 4       /* valid request outside the compiled limits */
} nrr_status;

typedef enum {
    NRR_U16 = 0, /* uint16 voxels, 12-bit values 0..4095 */
    NRR_F32 = 1  /* float32 voxels */
} nrr_dtype;

/* ------------------------------------------------------------------ helpers
 * Host-only: no device work, no synchronisation. */

/* Candidate grid of the selection: grid[a] = floor((dims[a]-block)/stride)+1
 * blocks per axis (origins g*stride, centres origin + h).  Errors:
 * INVALID_ARG if block is even or < 3, stride < 1, or dims[a] < block. */
nrr_status nrr_grid_shape(const int32_t dims[3], int32_t block, int32_t stride, int32_t grid[3]);

/* Number of blocks the selection keeps: K = floor(0.5 + N * fraction) with
 * N = grid[0]*grid[1]*grid[2] (the candidate count times the fraction plus
 * one half, the count rule of the parallel feature selection paragraph).  INVALID_ARG as nrr_grid_shape, or
 * fraction outside (0, 1]. */
nrr_status nrr_select_count(const int32_t dims[3], int32_t block, int32_t stride, double fraction,
                            int64_t *k);

/* Device workspace bytes nrr_select_blocks and nrr_select_blocks_ex need
 * for these sizes (the variants on grids of more than 24576 candidates take
 * 5 bytes per candidate more than the plain selection). */
nrr_status nrr_select_workspace_bytes(const int32_t dims[3], int32_t block, int32_t stride,
                                      size_t *bytes);

/* Device workspace bytes nrr_block_match needs (per-voxel window
 * statistics of `flt` for this block size). */
nrr_status nrr_match_workspace_bytes(nrr_dtype dtype, const int32_t dims[3], int32_t block,
                                     size_t *bytes);

/* NRR_OK if nrr_block_match supports this (dtype, block, window) on the
 * current device; NRR_ERR_UNSUPPORTED otherwise (e.g. the search window does
 * not fit in LDS), INVALID_ARG for malformed values. */
nrr_status nrr_match_supported(nrr_dtype dtype, int32_t block, int32_t window);

/* ---------------------------------------------------------------- selection
 * Variance-ranked block selection ("Parallel feature selection" paragraph:
 * each candidate block's intensity variance is computed, the candidates are
 * ordered by it and 0.5 + NFeatures x Fs of them are kept).
 *
 *  vol        device, dims[2]*dims[1]*dims[0] voxels of `dtype`.
 *  centers    device, int32 [capacity][3]: receives the K centres (x,y,z) in
 *             ascending linear grid index (gz*Gy+gy)*Gx+gx.
 *  k_out      host: receives K (also when capacity is too small).
 *  workspace  device, >= nrr_select_workspace_bytes() bytes, any content.
 *
 * Ranking: larger variance first; equal variance -> lower grid index first.
 * u16 uses the exact integer key N*sum(x^2)-(sum x)^2; f32 uses the FP64
 * two-pass variance summed in z, y, x order.
 * Errors: INVALID_ARG (bad sizes/fraction, null pointers), BUFFER_TOO_SMALL
 * (capacity < K with *k_out = K, or workspace too small), UNSUPPORTED (block
 * edge above 15, or a grid of 2^31 candidates or more), HIP.  K == 0 is a
 * valid no-op. */
nrr_status nrr_select_blocks(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                             int32_t block, int32_t stride, double fraction, int32_t *centers,
                             int64_t capacity, int64_t *k_out, void *workspace,
                             size_t workspace_bytes, void *stream);

/* nrr_select_blocks for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments and results without `workspace`; the
 * scratch comes from a 32 MiB array of this library that each GPU it runs
 * on holds until the process ends (its device address is looked up once per
 * device, on the first call with that device current).  No allocation, no
 * hipMemset: the selection writes every scratch word before reading it.
 *
 * Calls that overlap on one GPU (concurrent streams, or host threads
 * sharing a device) share that array and race: serialise them.  Errors as
 * nrr_select_blocks, plus UNSUPPORTED when the plain selection's workspace
 * for these sizes exceeds 32 MiB (about 4.19 million candidate blocks) or the
 * device index is 64 or more, HIP if the array's address cannot be found. */
nrr_status nrr_select_blocks_static(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                                    int32_t block, int32_t stride, double fraction,
                                    int32_t *centers, int64_t capacity, int64_t *k_out,
                                    void *stream);

/* Selection variants of the same paragraph: candidates restricted to a
 * region, and a connectivity pattern that keeps selected blocks apart.
 *
 *  mask          device, optional (NULL: every candidate): uint8 volume of
 *                dims; a candidate takes part iff the mask is nonzero at its
 *                centre.  N = number of candidates taking part, and the count
 *                is K = floor(0.5 + N * fraction).
 *  connectivity  0, 6, 18 or 26.  Candidates are visited in rank order (as
 *                nrr_select_blocks ranks them) and one is taken unless a
 *                candidate adjacent to it on the grid is already taken:
 *                adjacent = one grid step along one axis (6), along up to two
 *                axes (18) or up to three (26).  The visit stops at K taken
 *                (fewer when the candidates run out).  0: plain top-K among
 *                the candidates taking part.
 *  centers       device int32 [capacity][3]: the taken centres in ascending
 *                grid index; capacity >= floor(0.5 + grid count * fraction)
 *                (the count without a mask).
 *  k_device      device int64: receives the number taken.
 *  workspace     device, >= nrr_select_workspace_bytes().
 * Grids of up to 24576 candidates are selected by one workgroup and the call
 * returns without waiting.  Larger grids are selected in rounds (each settles
 * at least the best candidate still open) and the call waits on `stream`
 * after each round to see whether another is needed, so it returns when the
 * stream has reached the final selection kernels (not capturable in a graph).
 * Errors: INVALID_ARG (as nrr_select_blocks; connectivity not 0/6/18/26),
 * BUFFER_TOO_SMALL, UNSUPPORTED (2^31 candidates or more), HIP. */
nrr_status nrr_select_blocks_ex(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                                int32_t block, int32_t stride, double fraction,
                                const uint8_t *mask, int32_t connectivity, int32_t *centers,
                                int64_t capacity, int64_t *k_device, void *workspace,
                                size_t workspace_bytes, void *stream);

/* ----------------------------------------------------------------- matching
 * Exhaustive NCC block matching (NCC equation and the GPU block-matching
 * algorithm: every displacement of the window is evaluated and the maximum
 * with its displacement is kept; cost b^3 x (2W+1)^3 per point).
 *
 *  ref, flt   device volumes of `dtype`, same dims.
 *  centers    device, int32 [n][3] block centres (x,y,z) in `ref`.
 *  disp       device, int32 [n][3]: best displacement (dx,dy,dz).
 *  ncc        device, float [n]: NCC at that displacement.
 *  conf       device, float [n]: confidence weight max(0, ncc) for the
 *             downstream biomechanical solve (its S matrix).
 *  workspace  device, >= nrr_match_workspace_bytes() bytes, any content.
 *
 * A centre whose block is not inside the volume gets disp (0,0,0),
 * ncc NaN, conf 0; the other centres are unaffected.  Errors: INVALID_ARG,
 * BUFFER_TOO_SMALL (workspace), UNSUPPORTED (see nrr_match_supported), HIP.
 * n == 0 is a valid no-op. */
nrr_status nrr_block_match(const void *ref, const void *flt, nrr_dtype dtype,
                           const int32_t dims[3], const int32_t *centers, int64_t n,
                           int32_t block, int32_t window, int32_t *disp, float *ncc, float *conf,
                           void *workspace, size_t workspace_bytes, void *stream);

/* The two halves of nrr_block_match, for callers that search the same
 * intra-operative volume more than once with one block size (several block
 * lists, windows or parameter sets):
 *
 * nrr_window_stats writes into `workspace` the per-voxel statistics of every
 * b^3 block of `flt` (its sum and the reciprocal square root of its spread,
 * the denominator terms of the NCC equation).  nrr_block_match_prepared then
 * runs only the exhaustive search and reads that table: `workspace` must hold
 * the table written for the same flt contents, dtype, dims and block.  Same
 * argument rules and errors as nrr_block_match. */
nrr_status nrr_window_stats(const void *flt, nrr_dtype dtype, const int32_t dims[3],
                            int32_t block, void *workspace, size_t workspace_bytes,
                            void *stream);

/* Selection and window statistics of one step in one call: the plain
 * selection of `ref` (exactly nrr_select_blocks: the same K, centres and
 * errors) and the statistics of `flt` that the search for `window` reads
 * (exactly nrr_window_stats_for), the two running side by side.  For 12-bit
 * data, K > 0, grids of at most 32,768 candidates and block edges up to 9,
 * everything goes on `stream`: the keys, then one launch whose first
 * workgroup is the selection's radix select and whose other workgroups
 * compute the statistics (then the plane-pair words if the plan reads
 * them).  Otherwise the statistics go on a second stream of this library
 * (one per device, default priority, created on first use), forked from
 * `stream` after the keys, and `stream` waits for both before any later
 * work.  Safe under stream capture (a second stream joins the capture and is
 * joined back).  Concurrent calls on one device are serialised while they
 * enqueue on the second stream; such a call made while another host thread
 * captures a graph on the same device fails.  Errors as the two calls, plus
 * UNSUPPORTED for device indices of 64 or more. */
nrr_status nrr_select_and_window_stats(const void *ref, const void *flt, nrr_dtype dtype,
                                       const int32_t dims[3], int32_t block, int32_t stride,
                                       double fraction, int32_t window, int32_t *centers,
                                       int64_t capacity, int64_t *k_out, void *select_workspace,
                                       size_t select_workspace_bytes, void *match_workspace,
                                       size_t match_workspace_bytes, void *stream);

/* nrr_window_stats_for: as nrr_window_stats, for the search that nrr_block_match_prepared will run
 * with this window under the current plan (nrr_match_plan): the plane-pair
 * volume of 12-bit data is written only when that search reads it (the
 * dot2 form).  If the plan changes before the search (tuning, NRR_ARITH),
 * the prepared search adds the missing part itself. */
nrr_status nrr_window_stats_for(const void *flt, nrr_dtype dtype, const int32_t dims[3],
                                int32_t block, int32_t window, void *workspace,
                                size_t workspace_bytes, void *stream);

nrr_status nrr_block_match_prepared(const void *ref, const void *flt, nrr_dtype dtype,
                                    const int32_t dims[3], const int32_t *centers, int64_t n,
                                    int32_t block, int32_t window, int32_t *disp, float *ncc,
                                    float *conf, const void *workspace, size_t workspace_bytes,
                                    void *stream);

/* Per-axis block and window sizes.  The paper's parameter list gives the
 * half block size and the half search window separately for the three
 * axes ("Deep Learning Model Architecture" section), so blocks need not be
 * cubes.  block[3] = (bx, by, bz) are odd edges 1..15 (edge = 2 * half + 1),
 * stride[3] the candidate-grid steps, window[3] = (wx, wy, wz) half windows
 * 0..15.  Everything else is as in the cubic calls: the candidate grid per
 * axis, K = floor(0.5 + N * fraction), variance ranking with ties to the
 * lower grid index, centres in ascending grid index; displacements with
 * |d_a| <= w_a that keep the block inside the volume, shift index
 * ((dz+wz)(2wy+1) + (dy+wy))(2wx+1) + (dx+wx) breaking NCC ties, the flat
 * and outside rules.
 *
 * nrr_aniso_workspace_bytes: device workspace of the selection (grid of
 * block/stride; enough for the variants too) and of the search (block);
 * either output may be NULL, stride may be NULL (then 1).
 * nrr_select_count_aniso: the candidate grid (grid may be NULL) and K for
 * these sizes, on the host.
 * nrr_select_blocks_aniso: as nrr_select_blocks with per-axis sizes.
 * nrr_select_blocks_aniso_ex: as nrr_select_blocks_ex with per-axis sizes;
 * the mask is read at each candidate's centre (origin + (edge - 1) / 2 on
 * each axis) and grid neighbours are one grid step apart along an axis.
 * nrr_block_match_aniso: as nrr_block_match with per-axis sizes; the
 * workspace holds the window statistics of the bx x by x bz block.
 * Errors: INVALID_ARG, UNSUPPORTED (edge or half window above 15, window
 * region larger than the LDS), BUFFER_TOO_SMALL, HIP. */
nrr_status nrr_aniso_workspace_bytes(nrr_dtype dtype, const int32_t dims[3],
                                     const int32_t block[3], const int32_t stride[3],
                                     size_t *select_bytes, size_t *match_bytes);
nrr_status nrr_select_count_aniso(const int32_t dims[3], const int32_t block[3],
                                  const int32_t stride[3], double fraction, int32_t grid[3],
                                  int64_t *k);
nrr_status nrr_select_blocks_aniso(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                                   const int32_t block[3], const int32_t stride[3],
                                   double fraction, int32_t *centers, int64_t capacity,
                                   int64_t *k_out, void *workspace, size_t workspace_bytes,
                                   void *stream);
nrr_status nrr_select_blocks_aniso_ex(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                                      const int32_t block[3], const int32_t stride[3],
                                      double fraction, const uint8_t *mask, int32_t connectivity,
                                      int32_t *centers, int64_t capacity, int64_t *k_device,
                                      void *workspace, size_t workspace_bytes, void *stream);
nrr_status nrr_block_match_aniso(const void *ref, const void *flt, nrr_dtype dtype,
                                 const int32_t dims[3], const int32_t *centers, int64_t n,
                                 const int32_t block[3], const int32_t window[3], int32_t *disp,
                                 float *ncc, float *conf, void *workspace, size_t workspace_bytes,
                                 void *stream);
/* The two halves of nrr_block_match_aniso, for callers that search several
 * block sets against one moving volume: nrr_window_stats_aniso fills the
 * workspace with the statistics of the bx x by x bz block of `flt`;
 * nrr_block_match_aniso_prepared searches with that workspace (which must
 * come from the same flt, dtype, dims and block). */
nrr_status nrr_window_stats_aniso(const void *flt, nrr_dtype dtype, const int32_t dims[3],
                                  const int32_t block[3], void *workspace,
                                  size_t workspace_bytes, void *stream);
nrr_status nrr_block_match_aniso_prepared(const void *ref, const void *flt, nrr_dtype dtype,
                                          const int32_t dims[3], const int32_t *centers,
                                          int64_t n, const int32_t block[3],
                                          const int32_t window[3], int32_t *disp, float *ncc,
                                          float *conf, const void *workspace,
                                          size_t workspace_bytes, void *stream);

/* Every kernel relies on the dtype's contract (12-bit data: values 0..4095,
 * which the exact integer sums, the int16 offsets and the fp16 operands
 * need; float data: finite values) and does not check it: data outside it
 * give undefined results with NRR_OK.  nrr_check_volume counts, on
 * `stream`, the voxels of vol (device, dims[2]*dims[1]*dims[0] of dtype)
 * that break it into *bad_device (device int64), for callers that cannot
 * vouch for their data.  INVALID_ARG for NULL pointers or dims < 1. */
nrr_status nrr_check_volume(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                            int64_t *bad_device, void *stream);

/* Directional confidence for the biomechanical solve.  The FEM update
 * equation weights each block's displacement by a confidence matrix S; the
 * paper gives no formula for it.  This returns, per block centred at
 * centers[k] (block edge `block`), S = conf[k] * J / trace(J) with J the
 * structure tensor of `ref` over the block: the sum over its voxels of
 * g g^T, g the intensity gradient by central differences (one-sided first
 * differences on the volume's border planes).  S = 0 when trace(J) = 0 or
 * the block is not inside the volume.
 *
 *  ref      device volume of dtype; centers device int32 [n][3];
 *  conf     device float [n] (e.g. nrr_block_match's conf);
 *  out      device float [n][6] = S_xx, S_yy, S_zz, S_xy, S_xz, S_yz.
 * Errors: INVALID_ARG (bad block, null pointers with n > 0), HIP.  n == 0 is
 * a no-op. */
nrr_status nrr_structure_confidence(const void *ref, nrr_dtype dtype, const int32_t dims[3],
                                    const int32_t *centers, int64_t n, int32_t block,
                                    const float *conf, float *out, void *stream);

/* ------------------------------------------------------------------ tuning
 * Tile-shape autotuner.  The exhaustive search can run with several compiled
 * shapes (displacement tile per thread, threads per workgroup, prefetch of
 * the statistics records, number of displacement planes staged at once);
 * which is fastest depends on block, window and device.  The paper tunes
 * its GPU launch configuration by hand (its GPU timing discussion reports a
 * large gain from it); here the library times every shape it has for
 * (dtype, block, window) on the caller's own data and keeps the fastest for
 * every later search in this process with that (dtype, block, window):
 * nrr_block_match, nrr_block_match_prepared and the batched search.
 *
 *  A shape: arith 0 = dot2 (12-bit data), 1 = FMA, 2 = fp16 matrix cores
 *  (12-bit data, see nrr_match_plan); rx x ry displacements
 *  per thread; nt threads; pf 1 = records prefetched; cz displacement planes
 *  staged at once (0 in requests: as planned).
 *
 * nrr_tune_match takes the arguments of nrr_block_match_prepared (workspace
 * prepared by nrr_window_stats); the outputs hold the results of the last
 * trial (every shape computes the same results).  reps >= 1 timed launches
 * per shape after one warm-up.  It synchronises `stream`.  best (host,
 * optional) receives the chosen shape, best_us (host, optional) its mean
 * time in microseconds.  Errors as nrr_block_match_prepared, INVALID_ARG for
 * reps < 1. */
typedef struct {
    int32_t arith, rx, ry, nt, pf, cz;
} nrr_tile_shape;

nrr_status nrr_tune_match(const void *ref, const void *flt, nrr_dtype dtype,
                          const int32_t dims[3], const int32_t *centers, int64_t n, int32_t block,
                          int32_t window, int32_t *disp, float *ncc, float *conf,
                          const void *workspace, size_t workspace_bytes, int32_t reps,
                          nrr_tile_shape *best, double *best_us, void *stream);

/* The tuned shape for (dtype, block, window) (UNSUPPORTED if none yet), and
 * forgetting every tuned shape.  Host only. */
nrr_status nrr_tuned_shape(nrr_dtype dtype, int32_t block, int32_t window, nrr_tile_shape *out);
nrr_status nrr_clear_tuning(void);

/* Host-only views of the shape choice (no device work).
 *
 * nrr_match_plan: the shape nrr_block_match would launch now for these
 * arguments on the current device, with the NRR_ARITH (dot2 | fma | mfma)
 * and NRR_TILE overrides and tuned shapes taken into account.  arith 2 is
 * the fp16 matrix-core form (12-bit data, block edges 3-9, the window in
 * LDS; the default where it serves): products of exact 12-bit offsets with
 * FP32 sums, 256 threads; its rx, ry are 0 and pf -1.
 *
 * nrr_match_shapes: the compiled shapes nrr_tune_match times for (dtype,
 * block, window), each with a z-chunk cz; *count receives how many there are
 * (at most cap written to out).
 *
 * nrr_set_tuned_shape: pins `shape` for every later search of (dtype,
 * block, window) in this process, as nrr_tune_match does with the fastest;
 * cz 0 = as planned, else a cap on the z-chunk.  UNSUPPORTED if the shape is
 * not compiled for that block size (a shape of the batched search is
 * accepted and used there).
 *
 * nrr_batch_shapes: the shape each parameter set of a batched plan over
 * `sets` would run with (out[nsets]); errors as nrr_batch_layout.
 *
 * Errors: as nrr_match_supported, INVALID_ARG for NULL pointers. */
nrr_status nrr_match_plan(nrr_dtype dtype, const int32_t dims[3], int32_t block, int32_t window,
                          nrr_tile_shape *shape);
nrr_status nrr_match_shapes(nrr_dtype dtype, int32_t block, int32_t window, nrr_tile_shape *out,
                            int32_t cap, int32_t *count);
nrr_status nrr_set_tuned_shape(nrr_dtype dtype, int32_t block, int32_t window,
                               const nrr_tile_shape *shape);

/* ----------------------------------------------------------- batched search
 * The paper's intra-operative parametric search (block size, window and
 * selection fraction varied over one registration) as one batch: S
 * parameter sets over one volume pair, each a variance-ranked selection
 * (nrr_select_blocks with that set's block, stride and fraction) followed by
 * the exhaustive search of every selected block (nrr_block_match with that
 * set's window).  Results are identical to those S pairs of calls.
 *
 * The batch runs as one selection launch (a workgroup per set; each set's
 * candidate grid must have at most 4096 blocks), the window statistics of
 * each distinct block size, and ONE persistent search launch over the blocks
 * of every set (the sets of largest cost first, the tile shape of each set
 * from the tuned table or the cost model).  With use_graph the launches are
 * captured once into a HIP graph and each run replays it.
 *
 * nrr_batch_layout (host only): offsets[0..nsets] - set s owns output rows
 * offsets[s] .. offsets[s+1]-1 (K_s rows, in the order of `sets`) - and the
 * device workspace bytes of the plan.  Errors: INVALID_ARG (a malformed set:
 * rules of nrr_select_blocks and nrr_block_match), UNSUPPORTED (candidate
 * grid above 4096 blocks, or no compiled shape for a set).
 *
 * nrr_batch_plan_create: ref/flt device volumes; centers/disp int32
 * [rows][3], ncc/conf float [rows] device outputs; workspace device bytes as
 * nrr_batch_layout says.  All pointers stay owned by the caller and must
 * outlive the plan; every run rewrites the outputs and the workspace.  The
 * set tables are copied into the workspace during creation (synchronous).
 * *plan receives a host object released by nrr_batch_plan_destroy.
 *
 * nrr_batch_plan_run enqueues one batch on `stream` (asynchronous; a graph
 * launch when the plan holds one).  Runs of one plan must not overlap.  The
 * window statistics run on this library's second stream (the one
 * nrr_select_and_window_stats uses), forked from `stream` beside the
 * selection and joined back before the search, in eager runs and in the
 * captured graph alike; the same caveats hold (enqueues on one device are
 * serialised; a capture on another host thread at the same time fails). */
typedef struct {
    int32_t block, window, stride;
    double fraction;
} nrr_param_set;

typedef struct nrr_batch_plan nrr_batch_plan;

nrr_status nrr_batch_layout(nrr_dtype dtype, const int32_t dims[3], const nrr_param_set *sets,
                            int32_t nsets, int64_t *offsets, size_t *workspace_bytes);
nrr_status nrr_batch_shapes(nrr_dtype dtype, const int32_t dims[3], const nrr_param_set *sets,
                            int32_t nsets, nrr_tile_shape *out);

nrr_status nrr_batch_plan_create(const void *ref, const void *flt, nrr_dtype dtype,
                                 const int32_t dims[3], const nrr_param_set *sets, int32_t nsets,
                                 int32_t *centers, int32_t *disp, float *ncc, float *conf,
                                 void *workspace, size_t workspace_bytes, int32_t use_graph,
                                 void *stream, nrr_batch_plan **plan);

nrr_status nrr_batch_plan_run(nrr_batch_plan *plan, void *stream);

nrr_status nrr_batch_plan_destroy(nrr_batch_plan *plan);

/* ------------------------------------------------------------------ serving
 * A registration server for requests that arrive over time (the paper's
 * intra-operative setting: a registration must finish within the procedure,
 * while new scans keep arriving).  A request is one registration's block
 * matching: a volume pair and (block, stride, fraction, window); its result
 * is what nrr_select_blocks + nrr_block_match give for it.
 *
 * The server owns `device_bytes` of device memory (one allocation, made at
 * creation: the only device memory the library allocates itself) and `slots`
 * HIP streams, plus one stream for uploads of resident volumes.  A scheduler thread admits waiting
 * requests in arrival order as soon as a slot is free and the request's
 * device footprint (both volumes, selection and search workspaces, outputs:
 * nrr_request_footprint) fits in the free memory; a later request may pass
 * one that waits for memory if it fits, at most 8 times per waiting request.
 * Admitted requests run concurrently, each on its slot's stream: upload,
 * selection, window statistics, search, download.  Their memory returns to
 * the server when they complete.  Results do not depend on what else runs.
 *
 *  nrr_request.ref/flt   host or device volumes, dims[2]*dims[1]*dims[0]
 *                        voxels of dtype; read during the request's upload,
 *                        so they must stay unchanged until it completes.
 *  centers/disp/ncc/conf host or device outputs of >= K rows (K from
 *                        nrr_select_count; capacity = their rows), written
 *                        when the request completes.  Page-locked host
 *                        memory lets the copies overlap other work.  NULL
 *                        outputs are not copied out.
 *
 * nrr_server_submit (any host thread) validates and queues a request and
 * returns its ticket; INVALID_ARG / BUFFER_TOO_SMALL as the plain calls,
 * UNSUPPORTED when the footprint exceeds the server's memory or the search
 * is unsupported.  nrr_server_poll reports a ticket's state (0 queued,
 * 1 running, 2 done, 3 failed), its K, device bytes and times (queued, run,
 * submit-to-done) without blocking; nrr_server_wait blocks until it is done
 * and returns its status.  nrr_server_destroy finishes every submitted
 * request, then frees the server's memory and streams. */
typedef struct {
    const void *ref, *flt;
    nrr_dtype dtype;
    int32_t dims[3];
    int32_t block, stride, window;
    double fraction;
    int32_t *centers, *disp;
    float *ncc, *conf;
    int64_t capacity;
} nrr_request;

typedef struct {
    int32_t state, status;
    int64_t k, device_bytes;
    double queued_ms, run_ms, total_ms;
} nrr_request_info;

typedef struct {
    int64_t device_bytes, peak_bytes, used_bytes;
    int32_t slots, max_running;
    int64_t submitted, admitted, completed, pending;
    double wall_ms;     /* since creation */
    double busy_ms;     /* of wall_ms, time with at least one request running */
    int64_t volumes;    /* resident volumes */
    int64_t records;    /* request records not yet released */
} nrr_server_info;

typedef struct nrr_server nrr_server;

nrr_status nrr_request_footprint(const nrr_request *request, size_t *bytes);
nrr_status nrr_server_create(size_t device_bytes, int32_t slots, nrr_server **server);
nrr_status nrr_server_submit(nrr_server *server, const nrr_request *request, int64_t *ticket);

/* Resident volumes (the pre-operative volume of a procedure is registered
 * against every scan taken during it).  nrr_server_add_volume copies
 * dims[2]*dims[1]*dims[0] voxels of dtype from `data` (host or device; ready
 * when called, read before the call returns) into the server's memory and
 * returns its id (> 0); BUFFER_TOO_SMALL when the server's free memory cannot
 * hold it.  nrr_server_submit_resident submits a request whose ref and/or
 * flt is the resident volume `ref_volume` / `flt_volume` (0: the request's
 * own pointer, uploaded per request as by nrr_server_submit); the volume
 * must have the request's dtype and dims (INVALID_ARG otherwise).  A
 * resident ref keeps the block selection of each (block, stride, fraction)
 * it has been asked for: the first request computes it, later ones wait for
 * it on their own stream and reuse it.  nrr_server_remove_volume frees a
 * volume and its kept selections; INVALID_ARG while submitted requests that
 * name it have not finished. */
nrr_status nrr_server_add_volume(nrr_server *server, const void *data, nrr_dtype dtype,
                                 const int32_t dims[3], int64_t *volume);
nrr_status nrr_server_submit_resident(nrr_server *server, const nrr_request *request,
                                      int64_t ref_volume, int64_t flt_volume, int64_t *ticket);
nrr_status nrr_server_remove_volume(nrr_server *server, int64_t volume);

/* nrr_server_release drops the record of a finished (done or failed) request;
 * its ticket is unknown afterwards (INVALID_ARG for a ticket that has not
 * finished).  Records are kept until released or the server is destroyed. */
nrr_status nrr_server_release(nrr_server *server, int64_t ticket);
nrr_status nrr_server_poll(nrr_server *server, int64_t ticket, nrr_request_info *info);
nrr_status nrr_server_wait(nrr_server *server, int64_t ticket, nrr_request_info *info);
nrr_status nrr_server_stats(nrr_server *server, nrr_server_info *info);
nrr_status nrr_server_destroy(nrr_server *server);

/* ------------------------------------------------------------- diagnostics */

/* Static string for a status code. */
const char *nrr_status_string(nrr_status s);

/* Thread-local detail message of the last non-OK return on this thread
 * ("" if none).  Valid until the next call on the same thread. */
const char *nrr_last_error(void);

/* The search of nrr_block_match (window statistics included) that also
 * writes the NCC its ranking arithmetic gives every valid displacement: the
 * ranking key N cov / sqrt(N varF) of the NCC equation (section 3) divided
 * by sqrt(N varT), for checking that arithmetic's error against an exact
 * reference per displacement.  Diagnostic; slower than nrr_block_match.
 *
 *  arith      -1: the form nrr_block_match would use (see nrr_match_plan);
 *             0 dot2, 1 FMA, 2 fp16 matrix cores (each where compiled for
 *             this dtype and block edge, else UNSUPPORTED).
 *  surface    device, float [n][2W+1][2W+1][2W+1], indexed by the shift
 *             index ((dz+W)(2W+1) + (dy+W))(2W+1) + (dx+W); NaN for
 *             displacements whose block leaves the volume and for blocks
 *             outside the volume or flat (every NCC 0 by definition).
 *  others     as nrr_block_match (disp, ncc, conf written as it writes them).
 *
 * Errors as nrr_block_match, INVALID_ARG for a NULL surface or arith out of
 * range. */
nrr_status nrr_block_match_surface(const void *ref, const void *flt, nrr_dtype dtype,
                                   const int32_t dims[3], const int32_t *centers, int64_t n,
                                   int32_t block, int32_t window, int32_t arith, int32_t *disp,
                                   float *ncc, float *conf, float *surface, void *workspace,
                                   size_t workspace_bytes, void *stream);

/* ABI version (major*10000 + minor*100 + patch). */
int32_t nrr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NRR_H */
