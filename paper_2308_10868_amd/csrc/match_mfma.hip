// Exhaustive NCC block matching of 12-bit volumes on the gfx950 matrix cores.
//
// The cross term of the NCC equation (section 3), X(d) = sum_o T(o) F(o + d)
// over the block's voxels o, is one sliding correlation per block: a single
// template against its search window.  A single template is a matrix-vector
// product, which matrix cores cannot use; this kernel gives it a second
// matrix dimension by letting the 16 columns of a 16x16x32 fp16 MFMA be a
// 4x4 patch of (dx, dy) displacement offsets, so the block operand is the
// block T written out once per offset (a zero-padded Toeplitz matrix):
//
//   C[m][n] = sum_{x', y', s} F(p_m + (x', y', s)) * T(x' - a_n, y' - b_n, s)
//
// where row m is a window base position p_m = (bx, by, dz) and column n the
// offset (a_n, b_n); C[m][n] is the cross term of displacement
// (bx + a_n, by + b_n, dz).  K runs over the plane s of the block and the
// 4-column by 2-row groups of (x', y') that any column of the patch touches.
//
// Exactness and precision: 12-bit voxels centred on an integer c are exact in
// fp16 when |v - c| <= 2048.  The block and its window take a constant each,
// both starting at the block's rounded mean: c_T clamped into [max - 2048,
// min + 2048] over the block, c_F into the same interval over the window
// (neither is ever empty for 12-bit data), so every product is exact and only
// the FP32 accumulation rounds.  T - c_T sums to at most about N/2 in
// magnitude, so the terms that cancel in N X - S_T S_F stay small even where
// the window holds values far from the block's (a single constant clamped
// over both would leave T - c far from zero mean there, and FP32 partial sums
// N times the covariance's size); F - c_F is centred for the displacements
// that look like the block, where the ranking has to be accurate.  The
// ranking key follows the exact integer window statistics, and the winner's
// NCC is recomputed in exact integer arithmetic from the staged operands.
//
// Data flow of one workgroup (one selected block):
//  * the block's clipped window is staged in LDS as fp16 (v - c), rows padded
//    so every base's reads stay inside, and T - c goes to a zero-bordered
//    fp16 table from which each wavefront builds its Toeplitz B operands once
//    (they stay in registers for the whole block);
//  * each wavefront sweeps the window planes for a tile of 16 bases: the A
//    operand loaded for plane p feeds the accumulators of every displacement
//    plane dz = p - s that uses it (s = 0..b-1), a ring of b accumulator
//    tiles indexed at compile time; the tile whose last plane was just added
//    is ranked (key = N cov * rsqrt(N varF) from the statistics table) and
//    its slot reused;
//  * bases cover the valid (dx, dy) range in steps of 4; the displacement
//    planes are split into phases so that tiles = ceil(bases * phases / 16)
//    balance over the workgroup's wavefronts;
//  * argmax: largest key, smallest shift index among equal keys, reduced over
//    lanes, wavefronts and the workgroup.
//
// One 256-thread workgroup per selected block, two co-resident per CU: the
// staging and ranking latencies of one are hidden behind the matrix work of
// the other.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>

#include "nrr_internal.h"

namespace nrr {
namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4), aligned(4)));
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 half4u __attribute__((ext_vector_type(4), aligned(2)));

constexpr int OFF = 3;  // zero border of the T table (offsets 0..3)

// Compile-time sizes of the K layout for block edge B.
template <int B>
struct KGeo {
    static constexpr int GX = (B + 3 + 3) / 4;   // x' groups of 4 (x' extent B + 3)
    static constexpr int GYP = (B + 3 + 1) / 2;  // y' row pairs (y' extent B + 3)
    static constexpr int NG = GX * GYP;          // k-groups of 8 per block plane
    static constexpr int NQ = (NG + 3) / 4;      // 32-wide K chunks per block plane
    static constexpr int TXW = 4 * GX + 4;       // T table row width (halves)
    static constexpr int TYW = 2 * GYP + OFF;    // T table rows per plane
    static constexpr int TT_HALVES = B * TYW * TXW;
    static constexpr int TT_BYTES = (TT_HALVES * 2 + 15) & ~15;
};

struct MfParams {
    const uint16_t *ref;
    const uint16_t *flt;
    int nx, ny, nz;
    const int32_t *centers;
    int64_t first;  // first block of this launch
    int w;
    const StatU16 *stats;
    int ox, oy;
    int rp, pl;  // LDS window row and plane pitch (halves)
    int32_t *disp;
    float *ncc;
    float *conf;
    // optional [n][2w+1]^3 ranking NCC of every valid displacement (the
    // diagnostic instantiation only)
    float *surface;
};

__device__ inline int64_t xcd_order(int64_t wg, int64_t n) {
    const int64_t q = n / 8, r = n % 8, k = wg % 8, j = wg / 8;
    return k * q + (k < r ? k : r) + j;
}

__device__ inline void keep_best(float &bk, int &bi, float k, int i) {
    const bool take = (k > bk) | ((k == bk) & (i < bi));  // no short-circuit branches
    bk = take ? k : bk;
    bi = take ? i : bi;
}

__device__ inline void put(const MfParams &p, int64_t blk, int dx, int dy, int dz, float v) {
    p.disp[3 * blk] = dx;
    p.disp[3 * blk + 1] = dy;
    p.disp[3 * blk + 2] = dz;
    p.ncc[blk] = v;
    p.conf[blk] = v > 0.0f ? v : 0.0f;
}

constexpr int MAX_NW = 4;  // wavefronts per workgroup
struct MfSmall {
    long long red[MAX_NW * 4];
    int mm[MAX_NW * 4];
    float key[MAX_NW];
    int idx[MAX_NW];
};

// Tile decomposition of one block's displacements: bases every 4 voxels in x
// and y; the displacement planes in `nph` phases of `tz` planes each, tz a
// multiple of the block edge so the sweep's ramps fall on whole unrolled
// blocks of steps (planes past the valid range are computed and masked).
struct Tiling {
    int nbx, nby, nxy, nph, tz, nrows, ntiles;
};

__device__ inline Tiling make_tiling(int dxn, int dyn, int dzn, int b, int nq, int nw) {
    Tiling t;
    t.nbx = (dxn + 3) / 4;
    t.nby = (dyn + 3) / 4;
    t.nxy = t.nbx * t.nby;
    // fewest wavefront rounds of (MFMAs of a tile + per-step overhead)
    int best = b;
    float bc = 3.0e38f;
    for (int tz = b; tz < dzn + b; tz += b) {
        const int ph = (dzn + tz - 1) / tz;
        const int tiles = (t.nxy * ph + 15) / 16;
        const int rounds = (tiles + nw - 1) / nw;
        const float c = rounds * ((float)tz * b * nq + 3.0f * (tz + b - 1));
        if (c < bc) {
            bc = c;
            best = tz;
        }
    }
    t.tz = best;
    t.nph = (dzn + best - 1) / best;
    t.nrows = t.nxy * t.nph;
    t.ntiles = (t.nrows + 15) / 16;
    return t;
}

// Search geometry of one block: valid displacement range per axis (the
// displaced block inside the volume), the window origin, and the staged
// region.  Rows are staged from the even element at or before the window's
// first column (4-byte aligned copies; volumes with an even row length), so
// window column x sits at LDS column x + px; the tiles' x bases are LDS
// columns 4i (8-byte aligned operand reads).
struct BGeo {
    int cx, cy, cz;
    bool inside;
    int lox, loy, loz, dxn, dyn, dzn;
    int wx0, wy0, wz0, ex, ey, ez, px;
    int rpb, pyb, cpr;  // LDS columns read, staged rows per plane, 8-column chunks per row
    Tiling tl;
};

template <int B>
__device__ inline BGeo block_geo(const MfParams &p, int64_t blk, int nw) {
    using G = KGeo<B>;
    constexpr int H = (B - 1) / 2;
    BGeo g;
    g.cx = p.centers[3 * blk];
    g.cy = p.centers[3 * blk + 1];
    g.cz = p.centers[3 * blk + 2];
    g.inside = g.cx - H >= 0 && g.cy - H >= 0 && g.cz - H >= 0 && g.cx + H <= p.nx - 1 &&
               g.cy + H <= p.ny - 1 && g.cz + H <= p.nz - 1;
    g.lox = max(-p.w, H - g.cx);
    g.loy = max(-p.w, H - g.cy);
    g.loz = max(-p.w, H - g.cz);
    g.dxn = min(p.w, p.nx - 1 - H - g.cx) - g.lox + 1;
    g.dyn = min(p.w, p.ny - 1 - H - g.cy) - g.loy + 1;
    g.dzn = min(p.w, p.nz - 1 - H - g.cz) - g.loz + 1;
    g.wx0 = g.cx - H + g.lox;
    g.wy0 = g.cy - H + g.loy;
    g.wz0 = g.cz - H + g.loz;
    g.ex = g.dxn + B - 1;
    g.ey = g.dyn + B - 1;
    g.ez = g.dzn + B - 1;
    g.px = (p.nx & 1) == 0 ? (g.wx0 & 1) : 0;
    g.tl = make_tiling(g.dxn + g.px, g.dyn, g.dzn, B, G::NQ, nw);
    g.rpb = 4 * (g.tl.nbx - 1) + 4 * G::GX;
    g.pyb = 4 * (g.tl.nby - 1) + 2 * G::GYP;
    g.cpr = (g.rpb + 7) / 8;
    return g;
}

// Global element of LDS column 8 xc, row y, plane z of the staged region
// (rows past the window repeat its last row).
__device__ inline int64_t stage_elem(const MfParams &p, const BGeo &g, int z, int y, int xc) {
    return ((int64_t)(g.wz0 + z) * p.ny + (g.wy0 + min(y, g.ey - 1))) * p.nx + g.wx0 - g.px +
           8 * xc;
}

// The 16 bytes (8 voxels) of one staged chunk through registers: a 16-byte
// load where it lies inside the volume, else clamped words (the volume's
// last voxels) or, for odd row lengths, voxel by voxel clamped into the
// window's row.
__device__ inline u32x4 load_chunk(const MfParams &p, const BGeo &g, int64_t e, int xc) {
    const int64_t vol_end = (int64_t)p.nx * p.ny * p.nz - 1;
    if ((p.nx & 1) == 0 && e + 7 <= vol_end) return *reinterpret_cast<const u32x4 *>(p.flt + e);
    uint32_t t[4];
    if ((p.nx & 1) == 0) {
        const int64_t last_pair = (vol_end - 1) & ~(int64_t)1;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            t[j] = *reinterpret_cast<const uint32_t *>(p.flt + min(e + 2 * j, last_pair));
    } else {
        const uint16_t *r = p.flt + (e - 8 * xc);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int x0 = min(8 * xc + 2 * j, g.ex - 1), x1 = min(8 * xc + 2 * j + 1, g.ex - 1);
            t[j] = (uint32_t)r[x0] | ((uint32_t)r[x1] << 16);
        }
    }
    u32x4 v;
    __builtin_memcpy(&v, t, 16);
    return v;
}

// One unrolled block of B sweep steps t0 .. t0 + B - 1 (t0 a multiple of B):
// MODE 0 is the first block (plane s of the block only reaches displacement
// planes tau = t - s >= 0), MODE 1 a full block, MODE 2 the last one (B - 1
// steps, tau = t - s < tz).  The accumulator of tau is slot tau mod B; after
// step t, plane tau = t - B + 1 is complete and `rank` takes it.
template <int B, int NQ, int MODE, typename LoadA, typename Rank>
__device__ __attribute__((always_inline)) inline void sweep_block(
    int t0, float4v (&acc)[B], const half8 (&bop)[B][NQ], half8 (&aop)[NQ], LoadA load_a,
    Rank rank) {
    constexpr int STEPS = MODE == 2 ? B - 1 : B;
#pragma unroll
    for (int u = 0; u < STEPS; ++u) {
        const int t = t0 + u;
        // consecutive products feed different accumulators, and the plane
        // completed by this step (block plane B - 1) is fed first in each
        // chunk, so its sums are ready when the ranking reads them
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int k = 0; k < B; ++k) {
                const int s = B - 1 - k;
                if (MODE == 0 && s > u) continue;
                if (MODE == 2 && s <= u) continue;
                const int slot = (u - s + B) % B;
                acc[slot] =
                    __builtin_amdgcn_mfma_f32_16x16x32_f16(aop[q], bop[s][q], acc[slot], 0, 0, 0);
            }
        // the next plane's operand replaces this one (its reads are issued
        // behind the products above and complete while the ranking runs)
        load_a(t + 1, aop);
        const int fs = (u + 1) % B;
        if (MODE != 0 || u == B - 1) rank(acc[fs], t - (B - 1));
        acc[fs] = float4v{0.0f, 0.0f, 0.0f, 0.0f};
    }
}

// Toeplitz B operands of this lane for every block plane and K chunk, from
// the zero-bordered table of T - c.
template <int B>
__device__ __attribute__((always_inline)) inline void build_bop(
    const _Float16 *tt, int lane, half8 (&bop)[B][KGeo<B>::NQ]) {
    using G = KGeo<B>;
    const int grp = lane >> 4, oa = lane & 3, ob = (lane >> 2) & 3;  // column: offset (oa, ob)
#pragma unroll
    for (int q = 0; q < G::NQ; ++q) {
        const int g = 4 * q + grp;
        const bool real = g < G::NG;
        const int gx = real ? g % G::GX : 0, gy = real ? g / G::GX : 0;
#pragma unroll
        for (int s = 0; s < B; ++s) {
            const _Float16 *tr = tt + (s * G::TYW + 2 * gy - ob + OFF) * G::TXW + 4 * gx - oa + OFF;
            const half4u lo = *reinterpret_cast<const half4u *>(tr);
            const half4u hi = *reinterpret_cast<const half4u *>(tr + G::TXW);
            const half8 v = half8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
            bop[s][q] = real ? v : half8{};
        }
    }
}

// This wavefront's tiles of the block's search over the centred window
// `win` (row pitch rp, plane pitch pl halves): keeps the lane's best (key,
// shift index).  key = (N C - S_T S_F) * rsqrt(N varF), with S_T = sum (T -
// c_T) and S_F = sum (F - c_F) = s + N (2048 - c_F) (the table's s sums
// F - 2048): S_T S_F = S_T s + S_T N (2048 - c_F), both terms in FP32 from
// exact integers (relative error 2^-24 of terms at most |S_T| N 2048).
template <int B, int NW, bool SURF>
__device__ __attribute__((always_inline)) inline void sweep_tiles(
    const MfParams &p, const BGeo &g, int64_t blk, const _Float16 *win, int rp, int pl,
    const half8 (&bop)[B][KGeo<B>::NQ], long long sTc, float inv_vt, int cf, int wave, int lane,
    float &bk, int &bi) {
    using G = KGeo<B>;
    constexpr int N = B * B * B, NQ = G::NQ;
    const Tiling &tl = g.tl;
    const int n16 = lane & 15, grp = lane >> 4;
    const int oa = n16 & 3, ob = n16 >> 2;
    const float fN = (float)N, fST = (float)sTc;
    const float fshift = (float)(sTc * (long long)N * (2048 - cf));
    const int side = 2 * p.w + 1, side2 = side * side;
    const int plane_rec = p.oy * p.ox;
    for (int tile = wave; tile < tl.ntiles; tile += NW) {
        // the lane's A row (base of row n16)
        int aoff[NQ], aph;
        {
            const int r = 16 * tile + n16, rr = r < tl.nrows ? r : 0;
            const int xy = rr % tl.nxy, ph = rr / tl.nxy;
            const int bx = 4 * (xy % tl.nbx), by = 4 * (xy / tl.nbx);
            aph = ph * tl.tz;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int gg = 4 * q + grp < G::NG ? 4 * q + grp : 0;
                aoff[q] = (by + 2 * (gg / G::GX)) * rp + bx + 4 * (gg % G::GX);
            }
        }
        // the lane's four output rows: displacement (odx, ody) relative to the
        // valid range's corner, plane offset oph; records at orec + dz planes
        // ranking of plane tau: valid while tau < lim (lim = -1 for rows
        // outside the valid range), shift index oidx + tau side^2; records
        // of plane min(tau + oph, dzn - 1) at rcur, which advances by a plane
        // while tau < lim3 = dzn - 1 - oph
        int rcur[4], lim[4], lim3[4], oidx[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * tile + 4 * grp + i;
            bool orow = r < tl.nrows;
            const int rr = orow ? r : 0;
            const int xy = rr % tl.nxy, ph = rr / tl.nxy;
            const int odx = 4 * (xy % tl.nbx) + oa - g.px;
            const int ody = 4 * (xy / tl.nbx) + ob;
            const int oph = ph * tl.tz;
            orow = orow && odx >= 0 && odx < g.dxn && ody < g.dyn;
            rcur[i] = (g.wz0 * p.oy + (g.wy0 + min(ody, g.dyn - 1))) * p.ox +
                      (g.wx0 + min(max(odx, 0), g.dxn - 1)) + min(oph, g.dzn - 1) * plane_rec;
            lim[i] = orow ? g.dzn - oph : -1;
            lim3[i] = g.dzn - 1 - oph;
            oidx[i] = (g.loz + oph + p.w) * side2 + (g.loy + ody + p.w) * side +
                      (g.lox + odx + p.w);
        }
        float4v acc[B];
#pragma unroll
        for (int k = 0; k < B; ++k) acc[k] = float4v{0.0f, 0.0f, 0.0f, 0.0f};
        // A operand of plane t + phase (clamped: planes past the window feed
        // only displacements that are masked out)
        auto load_a = [&](int t, half8 (&aop)[NQ]) {
            const int pz = min(t + aph, g.ez - 1);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const _Float16 *ap = win + pz * pl + aoff[q];
                const half4 lo = *reinterpret_cast<const half4 *>(ap);
                const half4 hi = *reinterpret_cast<const half4 *>(ap + rp);
                aop[q] = half8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
            }
        };
        // statistics records of the four output rows, loaded one displacement
        // plane ahead of their ranking (clamped into the valid range, so every
        // load is in bounds; invalid ones are masked)
        StatU16 rec0[4];
        auto fetch = [&](int tau, StatU16 (&rec)[4]) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                rec[i] = p.stats[rcur[i]];
                rcur[i] += tau < lim3[i] ? plane_rec : 0;
            }
        };
        // best key of each output row in this tile and its plane (byte i of
        // rtp; 0xff: none; planes < 255, see mf_plan).  Along a row the shift
        // index grows with tau, so a strict comparison keeps the smallest
        // index among equal keys; rows are merged with the full rule after
        // the tile.
        float rk[4];
        uint32_t rtp = 0xffffffffu;
#pragma unroll
        for (int i = 0; i < 4; ++i) rk[i] = -INFINITY;
        // ranking of displacement plane tau, then the records of tau + 1
        auto rank = [&](const float4v &c4, int tau) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float sts = __builtin_fmaf(fST, (float)rec0[i].s, fshift);
                const float cov = __builtin_fmaf(fN, c4[i], -sts);
                const float key = cov * rec0[i].r;
                const bool take = (tau < lim[i]) & (key > rk[i]);
                rk[i] = take ? key : rk[i];
                rtp = take ? (rtp & ~(0xffu << (8 * i))) | ((uint32_t)tau << (8 * i)) : rtp;
                if constexpr (SURF)  // NCC = key / sqrt(N varT)
                    if (tau < lim[i]) p.surface[blk * side2 * side + oidx[i] + tau * side2] =
                        key * inv_vt;
            }
            fetch(tau + 1, rec0);
        };
        fetch(0, rec0);
        half8 aop[NQ];
        load_a(0, aop);
        sweep_block<B, NQ, 0>(0, acc, bop, aop, load_a, rank);
        for (int t0 = B; t0 < tl.tz; t0 += B) sweep_block<B, NQ, 1>(t0, acc, bop, aop, load_a, rank);
        sweep_block<B, NQ, 2>(tl.tz, acc, bop, aop, load_a, rank);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rt = (rtp >> (8 * i)) & 0xff;
            if (rt != 0xff) keep_best(bk, bi, rk[i], oidx[i] + rt * side2);
        }
    }
}

// Workgroup argmax of the lanes' (key, index), then the exact NCC at the
// winner from the staged integers (F - c_F in the window, T - c_T in the
// table; the NCC does not depend on either constant), written by thread 0.  Every
// thread of the workgroup calls it; it ends with a barrier.
template <int B, int NW>
__device__ __attribute__((always_inline)) inline void finish_block(
    const MfParams &p, const BGeo &g, int64_t blk, const _Float16 *win, int rp, int pl,
    const _Float16 *tt, long long st, long long stt, int c, float bk, int bi, MfSmall &sm,
    int tid) {  // c: the block's constant c_T
    using G = KGeo<B>;
    constexpr int N = B * B * B, NT = 64 * NW;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int off = 32; off > 0; off >>= 1) {
        const float ok = __shfl_xor(bk, off);
        const int oi = __shfl_xor(bi, off);
        keep_best(bk, bi, ok, oi);
    }
    if (lane == 0) {
        sm.key[wave] = bk;
        sm.idx[wave] = bi;
    }
    __syncthreads();
    bk = sm.key[0];
    bi = sm.idx[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) keep_best(bk, bi, sm.key[i], sm.idx[i]);
    if (bi == INT_MAX) {  // no finite key (cannot happen for 12-bit data)
        if (tid == 0) put(p, blk, 0, 0, 0, NAN);
        __syncthreads();
        return;
    }
    const int side = 2 * p.w + 1;
    const int ddx = bi % side - p.w, ddy = (bi / side) % side - p.w, ddz = bi / (side * side) - p.w;
    const int rx = ddx - g.lox + g.px, ry = ddy - g.loy, rz = ddz - g.loz;
    long long sf = 0, sff = 0, stf = 0;
    for (int o = tid; o < N; o += NT) {
        const int oz = o / (B * B), oy = (o / B) % B, ox = o % B;
        const long long f = (long long)(float)win[(rz + oz) * pl + (ry + oy) * rp + rx + ox];
        const long long tv = (long long)(float)tt[(oz * G::TYW + oy + OFF) * G::TXW + ox + OFF];
        sf += f;
        sff += f * f;
        stf += tv * f;
    }
    for (int off = 32; off > 0; off >>= 1) {
        sf += __shfl_xor(sf, off);
        sff += __shfl_xor(sff, off);
        stf += __shfl_xor(stf, off);
    }
    __syncthreads();  // sm reused
    if (lane == 0) {
        sm.red[wave * 4] = sf;
        sm.red[wave * 4 + 1] = sff;
        sm.red[wave * 4 + 2] = stf;
    }
    __syncthreads();
    if (tid == 0) {
        sf = sff = stf = 0;
        for (int i = 0; i < NW; ++i) {
            sf += sm.red[i * 4];
            sff += sm.red[i * 4 + 1];
            stf += sm.red[i * 4 + 2];
        }
        const long long sTc = st - (long long)N * c;                       // sum (T - c)
        const long long tc2 = stt - 2ll * c * st + (long long)N * c * c;  // sum (T - c)^2
        const long long vt = (long long)N * tc2 - sTc * sTc;
        const long long vf = (long long)N * sff - sf * sf;
        const long long cv = (long long)N * stf - sTc * sf;
        const double v = (vt > 0 && vf > 0) ? (double)cv / sqrt((double)vt * (double)vf) : 0.0;
        put(p, blk, ddx, ddy, ddz, (float)v);
    }
    __syncthreads();
}

// Workgroup reduction of the block sums and the value ranges (block: tmin,
// tmax; window: vmin, vmax); every thread returns the totals.
template <int NW>
__device__ inline void reduce_block(long long &st, long long &stt, int &tmin, int &tmax,
                                    int &vmin, int &vmax, MfSmall &sm, int tid) {
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int off = 32; off > 0; off >>= 1) {
        st += __shfl_xor(st, off);
        stt += __shfl_xor(stt, off);
        tmin = min(tmin, __shfl_xor(tmin, off));
        tmax = max(tmax, __shfl_xor(tmax, off));
        vmin = min(vmin, __shfl_xor(vmin, off));
        vmax = max(vmax, __shfl_xor(vmax, off));
    }
    if (lane == 0) {
        sm.red[wave * 4] = st;
        sm.red[wave * 4 + 1] = stt;
        sm.mm[wave * 4] = tmin;
        sm.mm[wave * 4 + 1] = tmax;
        sm.mm[wave * 4 + 2] = vmin;
        sm.mm[wave * 4 + 3] = vmax;
    }
    __syncthreads();
    st = 0;
    stt = 0;
    tmin = vmin = 4095;
    tmax = vmax = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        st += sm.red[i * 4];
        stt += sm.red[i * 4 + 1];
        tmin = min(tmin, sm.mm[i * 4]);
        tmax = max(tmax, sm.mm[i * 4 + 1]);
        vmin = min(vmin, sm.mm[i * 4 + 2]);
        vmax = max(vmax, sm.mm[i * 4 + 3]);
    }
}

// A centre: the block's rounded mean, clamped so every |v - c| <= 2048 over
// the values of range [vmin, vmax] (12-bit values: the interval is never
// empty).
__device__ inline int centre(long long st, int n, int vmin, int vmax) {
    return min(max((int)llrint((double)st / (double)n), vmax - 2048), vmin + 2048);
}

// 16 bytes of raw 12-bit voxels -> fp16 (v - c), exact for |v - c| <= 2048.
__device__ inline u32x4 centre_chunk(u32x4 v, i16x2 c2) {
    i16x2 d[4];
    half2v h[4];
    __builtin_memcpy(d, &v, 16);
#pragma unroll
    for (int j = 0; j < 4; ++j) h[j] = __builtin_convertvector(d[j] - c2, half2v);
    __builtin_memcpy(&v, h, 16);
    return v;
}

// ------------------------------------------------------------------ kernel
// One 256-thread workgroup per selected block.  Two wavefronts per SIMD up
// to 7^3 blocks; the 9^3 block's B operands (180 registers) take the whole
// register file of one.
constexpr int PB_NW = 4;

template <int B, bool SURF>
__global__ __launch_bounds__(64 * PB_NW, B <= 7 ? 2 : 1) void k_match_mfma(MfParams p) {
    using G = KGeo<B>;
    constexpr int H = (B - 1) / 2, N = B * B * B, NQ = G::NQ, NT = 64 * PB_NW;
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ MfSmall sm;
    _Float16 *tt = reinterpret_cast<_Float16 *>(lds);  // [B][TYW][TXW]
    _Float16 *win = reinterpret_cast<_Float16 *>(lds + G::TT_BYTES);

    const int64_t blk = p.first + xcd_order(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const BGeo g = block_geo<B>(p, blk, PB_NW);
    if (!g.inside) {
        if (tid == 0) put(p, blk, 0, 0, 0, NAN);
        return;
    }
    const int rp = p.rp, pl = p.pl;
    const int nchunk = g.ez * g.pyb * g.cpr;

    // ---- pass 1: window as raw 12-bit values, block sums, value range.  The
    // block's voxels (at most 3 per thread for edges up to 9) are loaded with
    // the first round of window rows and kept in registers for pass 2.
    for (int i = tid; i < G::TT_HALVES; i += NT) tt[i] = (_Float16)0.0f;
    constexpr int TPT = (N + NT - 1) / NT;  // block voxels per thread
    int tv[TPT];
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        const int o = min(tid + k * NT, N - 1);
        const int oz = o / (B * B), oy = (o / B) % B, ox = o % B;
        tv[k] = p.ref[((int64_t)(g.cz - H + oz) * p.ny + (g.cy - H + oy)) * p.nx + (g.cx - H + ox)];
    }
    // The range that clamps the window's centre covers every staged voxel: the
    // window and the few neighbouring voxels its padded rows pick up.
    u16x2 mn2 = {4095, 4095}, mx2 = {0, 0};
    {
        // chunk coordinates advance by NT chunks per step (no divisions)
        const int sx = NT % g.cpr, sr = NT / g.cpr;
        int xc = tid % g.cpr, y = tid / g.cpr, z = 0;
        while (y >= g.pyb) {
            y -= g.pyb;
            ++z;
        }
        constexpr int UNR = 8;
        for (int c0 = tid; c0 < nchunk; c0 += NT * UNR) {
            u32x4 w[UNR];
            int off[UNR];
            bool live[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                live[u] = c0 + u * NT < nchunk;
                const int zz = live[u] ? z : 0;
                off[u] = zz * pl + y * rp + 8 * xc;
                w[u] = load_chunk(p, g, stage_elem(p, g, zz, y, xc), xc);
                xc += sx;
                y += sr;
                if (xc >= g.cpr) {
                    xc -= g.cpr;
                    ++y;
                }
                while (y >= g.pyb) {
                    y -= g.pyb;
                    ++z;
                }
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
                if (!live[u]) continue;
                u16x2 h[4];
                __builtin_memcpy(h, &w[u], 16);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    mn2 = __builtin_elementwise_min(mn2, h[j]);
                    mx2 = __builtin_elementwise_max(mx2, h[j]);
                }
                *reinterpret_cast<u32x4 *>(win + off[u]) = w[u];
            }
        }
    }
    int vmin = min((int)mn2[0], (int)mn2[1]), vmax = max((int)mx2[0], (int)mx2[1]);
    int tmin = 4095, tmax = 0;
    long long st = 0, stt = 0;
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        if (tid + k * NT >= N) continue;
        st += tv[k];
        stt += (long long)tv[k] * tv[k];
        tmin = min(tmin, tv[k]);
        tmax = max(tmax, tv[k]);
    }
    reduce_block<PB_NW>(st, stt, tmin, tmax, vmin, vmax, sm, tid);
    if ((long long)N * stt - st * st == 0) {  // flat block: every NCC is 0
        if (tid == 0) put(p, blk, g.lox, g.loy, g.loz, 0.0f);
        return;
    }
    const int c = centre(st, N, tmin, tmax);    // c_T
    const int cf = centre(st, N, vmin, vmax);  // c_F

    // ---- pass 2: centre the staged planes in place (whole planes, padding
    // included: those halves are never read) on c_F, and the bordered table
    // of T - c_T
    {
        const i16x2 c2 = {(short)cf, (short)cf};
        const int nq = g.ez * pl / 8;  // pl is a multiple of 8 halves
        for (int i = tid; i < nq; i += NT) {
            u32x4 *a = reinterpret_cast<u32x4 *>(win + 8 * i);
            *a = centre_chunk(*a, c2);
        }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        const int o = tid + k * NT;
        if (o >= N) continue;
        const int oz = o / (B * B), oy = (o / B) % B, ox = o % B;
        tt[(oz * G::TYW + oy + OFF) * G::TXW + ox + OFF] = (_Float16)(float)(tv[k] - c);
    }
    __syncthreads();

    half8 bop[B][NQ];
    build_bop<B>(tt, lane, bop);
    float bk = -INFINITY;
    int bi = INT_MAX;
    const long long sTc = st - (long long)N * c;
    float inv_vt = 0.0f;
    if constexpr (SURF) {  // 1 / sqrt(N sum (T - c)^2 - (sum (T - c))^2), exact integers
        const long long tc2 = stt - 2ll * c * st + (long long)N * c * c;
        inv_vt = (float)(1.0 / sqrt((double)((long long)N * tc2 - sTc * sTc)));
    }
    sweep_tiles<B, PB_NW, SURF>(p, g, blk, win, rp, pl, bop, sTc, inv_vt, cf, wave, lane, bk, bi);
    finish_block<B, PB_NW>(p, g, blk, win, rp, pl, tt, st, stt, c, bk, bi, sm, tid);
}

// ------------------------------------------------------------------- host
typedef void (*mf_kernel_t)(MfParams);

struct MfVariant {
    int b;
    mf_kernel_t fn, surf;
    int tt_bytes;
};

#define MFV(B) {B, k_match_mfma<B, false>, k_match_mfma<B, true>, KGeo<B>::TT_BYTES}
const MfVariant kMfVariants[] = {MFV(3), MFV(5), MFV(7), MFV(9)};
#undef MFV

const MfVariant *mf_variant(int b) {
    for (const MfVariant &v : kMfVariants)
        if (v.b == b) return &v;
    return nullptr;
}

// LDS sizes for the unclipped window of (b, w): rows padded so that rows
// four apart (the bases' y step) start on different banks.
struct MfPlan {
    int rp, pl;  // row and plane pitch (halves)
    size_t lds;
};

bool mf_plan(int b, int w, size_t limit, MfPlan *out) {
    const MfVariant *v = mf_variant(b);
    if (!v) return false;
    const int d = 2 * w + 1;
    const int nbx = (d + 1 + 3) / 4, nby = (d + 3) / 4;  // x: one column of parity shift
    const int gx = (b + 6) / 4, gyp = (b + 4) / 2;
    int rp = (4 * (nbx - 1) + 4 * gx + 7) / 8 * 8;  // whole 8-column chunks
    while (((rp * 8) % 256) < 48 || ((rp * 8) % 256) > 208) rp += 8;
    const int py = 4 * (nby - 1) + 2 * gyp;
    int pl = py * rp;
    if (((pl * 2) % 256) == 0) pl += 8;
    const int planes = d + b - 1;
    if (planes >= 255) return false;  // the ranking keeps plane numbers in bytes
    const size_t lds = (size_t)v->tt_bytes + (size_t)planes * pl * 2;
    if (lds + sizeof(MfSmall) > limit) return false;
    out->rp = rp;
    out->pl = pl;
    out->lds = lds;
    return true;
}

}  // namespace

bool mfma_supported(nrr_dtype dtype, int32_t block, int32_t window) {
    if (dtype != NRR_U16) return false;
    MfPlan pl;
    return mf_plan(block, window, device_lds_limit(), &pl);
}

bool mfma_fits(const MatchArgs &a) {
    // record indices are 32-bit
    return (int64_t)a.ox * a.oy * (a.nz - a.block + 1) < (1ll << 31);
}

hipError_t launch_match_mfma(const MatchArgs &a, hipStream_t stream, float *surface) {
    MfPlan pl;
    if (!mf_plan(a.block, a.window, device_lds_limit(), &pl) || !mfma_fits(a))
        return hipErrorInvalidValue;
    const MfVariant *v = mf_variant(a.block);
    MfParams p;
    p.ref = static_cast<const uint16_t *>(a.ref);
    p.flt = static_cast<const uint16_t *>(a.flt);
    p.nx = a.nx;
    p.ny = a.ny;
    p.nz = a.nz;
    p.centers = a.centers;
    p.first = 0;
    p.w = a.window;
    p.stats = static_cast<const StatU16 *>(a.stats);
    p.ox = a.ox;
    p.oy = a.oy;
    p.rp = pl.rp;
    p.pl = pl.pl;
    p.disp = a.disp;
    p.ncc = a.ncc;
    p.conf = a.conf;
    p.surface = surface;
    const mf_kernel_t fn = surface ? v->surf : v->fn;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds);
    if (e != hipSuccess) return e;
    const int64_t chunk = 1ll << 30;
    for (int64_t first = 0; first < a.n; first += chunk) {
        p.first = first;
        const int64_t cnt = a.n - first < chunk ? a.n - first : chunk;
        hipLaunchKernelGGL(fn, dim3((unsigned)cnt), dim3(64 * PB_NW), pl.lds, stream, p);
    }
    return hipGetLastError();
}

}  // namespace nrr
