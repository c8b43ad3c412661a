// The 12-bit window statistics by voxel columns, one wavefront's work:
// shared by the statistics kernel and the kernel that runs the statistics
// beside the one-workgroup selection (see stats.hip for the method).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "nrr_internal.h"

namespace nrr {

// Workgroup-free LDS ordering between the lanes of one wavefront: its LDS
// writes complete before the reads that follow.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int SC_RY = 8;        // origin rows per wavefront
constexpr int SC_LW = 64 + 16;  // LDS slots of a row: the lanes, then the x reach
constexpr int SC_WAVES = 8192;  // wavefronts a launch aims at (z-runs are cut to reach it)

// One wavefront of the 12-bit statistics by voxel columns.  BY: block edge
// in y; BC: the cubic block edge when it is known at compile time (then bx =
// bz = BY = BC), 0 when bx and bz come at run time.  The wavefront takes
// x-tile xw (origins 65 - bx per tile), y-tile yw (SC_RY origin rows) and
// z-run `run` (zc origin planes); lanes 0 .. 64 - bx hold origins x0 + lane.
// xch: this wavefront's LDS rows.
template <int BY, int BC>
__device__ __attribute__((always_inline)) inline void stats_cols_wave(
    const uint16_t *__restrict__ flt, int nx, int ny, int nz, int bx_rt, int bz_rt, int ox,
    int oy, int oz, int zc, StatU16 *__restrict__ out, int xw, int yw, int run,
    uint2 (&xch)[SC_RY][SC_LW]) {
    static_assert(BC == 0 || BC == BY, "a cubic block has one edge");
    constexpr int RY = SC_RY, NR = RY + BY - 1;  // origin rows, voxel rows
    // block sums of squares fit 32 bits when N 2048^2 < 2^32 (N <= 1023)
    constexpr bool Q32 = BC != 0 && BC * BC * BC <= 1023;
    using QT = typename std::conditional<Q32, uint32_t, uint64_t>::type;
    const int bx = BC ? BC : bx_rt, bz = BC ? BC : bz_rt;
    const int lane = threadIdx.x & 63;
    const int txw = 65 - bx;  // origins per wavefront in x
    const int x0 = xw * txw;
    const int y0 = yw * RY;
    if (y0 >= oy) return;  // whole wavefront leaves together
    const int z0 = run * zc, zend = min(z0 + zc, oz);
    const int x = min(x0 + lane, nx - 1);  // lanes past the volume read its last column
    const int64_t ps = (int64_t)nx * ny;
    // voxel row r of this wavefront in plane p (rows past the volume read its last)
    auto load_plane = [&](uint32_t(&v)[NR], int p) {
        const uint16_t *pl = flt + (int64_t)min(p, nz - 1) * ps + x;
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = pl[(int64_t)min(y0 + r, ny - 1) * nx];
    };
    int32_t zs[NR];
    uint32_t zq[NR];  // <= 15 squares of 2048^2: < 2^32
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        zs[r] = 0;
        zq[r] = 0;
    }
    auto add_plane = [&](const uint32_t(&v)[NR]) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int d = (int)v[r] - 2048;
            zs[r] += d;
            zq[r] += (uint32_t)(d * d);
        }
    };
    // the first origin plane's bz planes, the next plane in flight while one
    // is added (two buffers, so no register copy waits on a load)
    uint32_t va[NR], vb[NR];
    load_plane(va, z0);
    for (int p = 0; p < bz; p += 2) {
        load_plane(vb, z0 + p + 1);
        add_plane(va);
        load_plane(va, z0 + p + 2);
        if (p + 1 < bz) add_plane(vb);
    }
    const double n = (double)(bx * BY * bz);
    const bool xin = lane < txw && x0 + lane < ox;
    for (int z = z0; z < zend; ++z) {
        // the planes entering (z + bz) and leaving (z) at the next origin
        // plane, in flight while this one is summed
        load_plane(va, z + bz);
        load_plane(vb, z);
        // by-row sums (sliding over the rows, exact)
        int32_t vs[RY];
        uint32_t vq[RY];
        {
            int32_t a = 0;
            uint32_t b = 0;
#pragma unroll
            for (int k = 0; k < BY; ++k) {
                a += zs[k];
                b += zq[k];
            }
            vs[0] = a;
            vq[0] = b;
#pragma unroll
            for (int r = 1; r < RY; ++r) {
                a += zs[r + BY - 1] - zs[r - 1];
                b += zq[r + BY - 1] - zq[r - 1];
                vs[r] = a;
                vq[r] = b;
            }
        }
        // bx-column sums across lanes
        wave_lds_sync();  // the previous plane's reads are done
#pragma unroll
        for (int r = 0; r < RY; ++r) xch[r][lane] = make_uint2((uint32_t)vs[r], vq[r]);
        wave_lds_sync();
        StatU16 *orow = out + ((int64_t)z * oy + y0) * ox + x0;  // origin (x0, y0, z)
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const uint2 *row = &xch[r][lane];
            int32_t S = 0;
            QT Q = 0;
            if constexpr (BC != 0) {
#pragma unroll
                for (int k = 0; k < BC; ++k) {
                    const uint2 u = row[k];
                    S += (int32_t)u.x;
                    Q += u.y;
                }
            } else {
                for (int k = 0; k < bx; ++k) {
                    const uint2 u = row[k];
                    S += (int32_t)u.x;
                    Q += u.y;
                }
            }
            if (xin && y0 + r < oy) {
                // N q - s^2 < 2^53: exact in FP64, then rounded once to float
                // (the same value as rounding the integer)
                const double var = fma(n, (double)Q, -((double)S * (double)S));
                // r ranks displacements only (the reported NCC is recomputed exactly)
                StatU16 rec;
                rec.s = S;
                rec.r = var > 0.0 ? rsqrtf((float)var) : 0.0f;
                orow[(int64_t)r * ox + lane] = rec;
            }
        }
        // slide the z sums to the next origin plane
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            // (e - 2048)^2 - (l - 2048)^2 = (e - l)(e + l - 4096), |each| < 2^12
            const int t = (int)va[r] - (int)vb[r];
            zs[r] += t;
            zq[r] += (uint32_t)(t * ((int)va[r] + (int)vb[r] - 4096));
        }
    }
}

// Launch shape of the column statistics: x-tiles, y-tiles and z-runs of
// zc origin planes, runs cut so the launch has about `target` wavefronts.
struct ColsGrid {
    int64_t nwx, nwy, runs;
    int zc;
};

inline ColsGrid cols_grid(const StatsLayout &L, int bx, int64_t target = SC_WAVES) {
    ColsGrid c;
    const int txw = 65 - bx;
    c.nwx = (L.ox + txw - 1) / txw;
    c.nwy = (L.oy + SC_RY - 1) / SC_RY;
    int64_t runs = (target + c.nwx * c.nwy - 1) / (c.nwx * c.nwy);
    runs = runs < 1 ? 1 : (runs > L.oz ? L.oz : runs);
    c.zc = (int)((L.oz + runs - 1) / runs);
    c.runs = (L.oz + c.zc - 1) / c.zc;
    return c;
}

// The select and the column statistics in one launch (select.hip): for
// 12-bit data, K > 0, grids the one-workgroup select takes and cubic block
// edges up to 9 (select_stats_fusable).  keys: the grid's keys, already on
// `stream`; L: the statistics layout of `stats` (records only: the
// plane-pair volume, when the plan reads it, is a separate pass).
bool select_stats_fusable(nrr_dtype dtype, int64_t n, int64_t k, int32_t block);
hipError_t launch_select_stats(const uint64_t *keys, int64_t n, const BoxGrid &G, int64_t k,
                               int32_t *centers, const SelectLayout &SL, char *sws,
                               const uint16_t *flt, const int32_t dims[3], int32_t block,
                               const StatsLayout &L, void *stats, hipStream_t stream);

// Float window statistics of n (1..kStatsJobs) cubic block edges over one
// volume in one launch (stats.hip), edge blocks[i]'s records into outs[i]
// (each laid out as launch_stats lays out that edge's workspace).  Several
// short, latency-bound statistics passes then share the device.
constexpr int kStatsJobs = 4;
hipError_t launch_stats_f32_multi(const float *flt, const int32_t dims[3], const int32_t *blocks,
                                  void *const *outs, int n, hipStream_t stream);

}  // namespace nrr
