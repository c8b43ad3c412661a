// Exhaustive NCC search with per-axis block edges and half windows.
//
// The paper's parameter list has a half block size and a half search window
// per anatomical axis (the "Deep Learning Model Architecture" section), so a
// block is bx x by x bz and the displacement set [-wx, wx] x [-wy, wy] x
// [-wz, wz].  The cubic search has its own tuned kernels; these are the
// general kernels for any such shape (edges and half windows up to 15).
//
// One workgroup of 256 threads per block (XCD-aware order, so that blocks
// with overlapping windows share an L2).  The moving volume's window region
// is staged in LDS, a run of `cz` displacement planes at a time, by rows
// with the lanes along x.  A thread owns RX consecutive x displacements of
// one (dy, dz) and accumulates the cross term X(d) over the block with an
// 8-wide unrolled inner product on 16-byte LDS reads; the tile's statistics
// records are fetched before the products.  The workgroup's argmax (largest
// key, smallest shift index on ties) is then rescored exactly, in two FP64
// passes over the block, for the reported NCC.
//
//   FMA (the default): T' = T - mean(T) in LDS as
//     float, F - mean(T) staged as float, X = sum T' F (T' sums to zero, so
//     X is the covariance term); key = X / sqrt(N sum F^2 - (sum F)^2).
//   DOT2 (12-bit data, on request): T'' = T - 2048 and F'' = F - 2048 as int16, two
//     block rows (y, y+1) packed per 32-bit word, so one v_dot2 does two
//     multiply-adds and each staged word serves two rows; X'' = sum T'' F''
//     exact in int32 per z plane (at most 15 * 8 * 2 * 2048^2 < 2^31) and in
//     FP64 across planes; key = (N X'' - sum T'' sum F'') / sqrt(...), the
//     sums of F'' from the statistics table.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "nrr_internal.h"

namespace nrr {
namespace {

constexpr int NT = 256;
constexpr int TU = 8;   // T row padding and inner-product unroll
constexpr int SU = 16;  // window rows staged per thread per step

// LDS pitch of a staged window row of `fp` words: an odd number of 16-byte
// groups, so that rows two apart do not land on the same banks.
__host__ __device__ inline int row_pitch(int fp) { return (fp / 4) % 2 == 0 ? fp + 4 : fp; }

typedef short short2v __attribute__((ext_vector_type(2)));

template <typename K>
__device__ inline void better(K &bk, int &bi, K k, int i) {
    if (k > bk || (k == bk && i < bi)) {
        bk = k;
        bi = i;
    }
}

// Workgroup index -> block index: the hardware deals workgroups to the 8
// XCDs round-robin, so blocks k*n/8 .. (k+1)*n/8 go to XCD k in order and
// neighbouring blocks (overlapping windows) share that XCD's L2.
__device__ inline int64_t xcd_order(int64_t wg, int64_t n) {
    const int64_t q = n / 8, r = n % 8, k = wg % 8, j = wg / 8;
    return k * q + (k < r ? k : r) + j;
}

// Sum of v over the workgroup (every thread gets it).
__device__ inline double wg_sum(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();  // red is reused across calls
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    return s;
}

// Per-block geometry: block half sizes, centre, valid displacement ranges.
struct AGeom {
    int bx, by, bz, hx, hy, hz, cx, cy, cz;
    int lox, loy, loz, ndx, ndy, ndz;
    int64_t sy, sz, rbase;
    int nb;
    bool inside;
};

__device__ inline AGeom aniso_geom(const AnisoArgs &p, int64_t blk) {
    AGeom g;
    g.bx = p.b[0], g.by = p.b[1], g.bz = p.b[2];
    g.hx = (g.bx - 1) / 2, g.hy = (g.by - 1) / 2, g.hz = (g.bz - 1) / 2;
    g.cx = p.centers[3 * blk], g.cy = p.centers[3 * blk + 1], g.cz = p.centers[3 * blk + 2];
    g.inside = g.cx - g.hx >= 0 && g.cy - g.hy >= 0 && g.cz - g.hz >= 0 &&
               g.cx + g.hx <= p.nx - 1 && g.cy + g.hy <= p.ny - 1 && g.cz + g.hz <= p.nz - 1;
    // displacements that keep the block inside the volume
    g.lox = max(-p.w[0], g.hx - g.cx);
    g.loy = max(-p.w[1], g.hy - g.cy);
    g.loz = max(-p.w[2], g.hz - g.cz);
    g.ndx = min(p.w[0], p.nx - 1 - g.hx - g.cx) - g.lox + 1;
    g.ndy = min(p.w[1], p.ny - 1 - g.hy - g.cy) - g.loy + 1;
    g.ndz = min(p.w[2], p.nz - 1 - g.hz - g.cz) - g.loz + 1;
    g.sy = p.nx;
    g.sz = (int64_t)p.nx * p.ny;
    g.rbase = (g.cz - g.hz) * g.sz + (int64_t)(g.cy - g.hy) * g.sy + (g.cx - g.hx);
    g.nb = g.bx * g.by * g.bz;
    return g;
}

__device__ inline void write_outside(const AnisoArgs &p, int64_t blk) {
    p.disp[3 * blk] = p.disp[3 * blk + 1] = p.disp[3 * blk + 2] = 0;
    p.ncc[blk] = NAN;
    p.conf[blk] = 0.0f;
}

// Workgroup argmax of (key, shift index), then the winner's NCC in two FP64
// passes over the block (mt = the ref block's mean); thread 0 writes.
template <typename Vox, typename Key>
__device__ inline void aniso_finish(const AnisoArgs &p, const AGeom &g, int64_t blk, Key bk, int bi,
                                    double mt, Key *s_key, int *s_idx, double *red) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int off = 32; off > 0; off >>= 1) {
        const Key ok = __shfl_xor(bk, off);
        const int oi = __shfl_xor(bi, off);
        better(bk, bi, ok, oi);
    }
    if ((tid & 63) == 0) {
        s_key[tid >> 6] = bk;
        s_idx[tid >> 6] = bi;
    }
    __syncthreads();
    bk = s_key[0];
    bi = s_idx[0];
    for (int w = 1; w < nt / 64; ++w) better(bk, bi, s_key[w], s_idx[w]);
    const int sxn = 2 * p.w[0] + 1, syn = 2 * p.w[1] + 1;
    const int dx = bi % sxn - p.w[0], dy = (bi / sxn) % syn - p.w[1], dz = bi / (sxn * syn) - p.w[2];

    const Vox *ref = static_cast<const Vox *>(p.ref);
    const Vox *flt = static_cast<const Vox *>(p.flt);
    const int64_t fbase = g.rbase + dz * g.sz + (int64_t)dy * g.sy + dx;
    double sf = 0.0;
    for (int o = tid; o < g.nb; o += nt) {
        const int x = o % g.bx, y = (o / g.bx) % g.by, z = o / (g.bx * g.by);
        sf += (double)flt[fbase + z * g.sz + (int64_t)y * g.sy + x];
    }
    const double mf = wg_sum(sf, red) / g.nb;
    double a = 0.0, b = 0.0, x2 = 0.0;
    for (int o = tid; o < g.nb; o += nt) {
        const int x = o % g.bx, y = (o / g.bx) % g.by, z = o / (g.bx * g.by);
        const int64_t off = z * g.sz + (int64_t)y * g.sy + x;
        const double tv = (double)ref[g.rbase + off] - mt, fv = (double)flt[fbase + off] - mf;
        a += tv * tv;
        b += fv * fv;
        x2 += tv * fv;
    }
    a = wg_sum(a, red);
    b = wg_sum(b, red);
    x2 = wg_sum(x2, red);
    if (tid == 0) {
        const double ab = a * b;
        const double v = ab > 0.0 ? x2 / sqrt(ab) : 0.0;
        p.disp[3 * blk] = dx;
        p.disp[3 * blk + 1] = dy;
        p.disp[3 * blk + 2] = dz;
        p.ncc[blk] = (float)v;
        p.conf[blk] = v > 0.0 ? (float)v : 0.0f;
    }
}

template <typename Vox>
struct Rec;
template <>
struct Rec<uint16_t> {
    using Key = float;
    __device__ static float r(const void *st, int64_t o) {
        return static_cast<const StatU16 *>(st)[o].r;
    }
};
template <>
struct Rec<float> {
    using Key = double;
    __device__ static double r(const void *st, int64_t o) {
        return static_cast<const StatF32 *>(st)[o].r;
    }
};

// FMA form (any voxel type).
template <typename Vox, int RX>
__global__ __launch_bounds__(NT) void k_match_aniso(AnisoArgs p) {
    using Key = typename Rec<Vox>::Key;
    extern __shared__ __align__(16) float lds[];
    __shared__ double red[NT / 64];
    __shared__ Key s_key[NT / 64];
    __shared__ int s_idx[NT / 64];
    const int64_t blk = xcd_order(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x, nt = blockDim.x;
    const Vox *ref = static_cast<const Vox *>(p.ref);
    const Vox *flt = static_cast<const Vox *>(p.flt);
    const AGeom g = aniso_geom(p, blk);
    if (!g.inside) {  // uniform: the whole workgroup leaves
        if (tid == 0) write_outside(p, blk);
        return;
    }
    const int bx = g.bx, by = g.by, bz = g.bz;

    // T' = T - mean(T) in LDS, rows padded to TP with zeros
    const int TP = (bx + TU - 1) / TU * TU;
    float *T = lds;
    double st = 0.0;
    for (int o = tid; o < g.nb; o += nt) {
        const int x = o % bx, y = (o / bx) % by, z = o / (bx * by);
        st += (double)ref[g.rbase + z * g.sz + (int64_t)y * g.sy + x];
    }
    const double mt = wg_sum(st, red) / g.nb;
    for (int e = tid; e < bz * by * TP; e += nt) {
        const int x = e % TP, r = e / TP, y = r % by, z = r / by;
        T[e] = x < bx ? (float)((double)ref[g.rbase + z * g.sz + (int64_t)y * g.sy + x] - mt)
                      : 0.0f;
    }
    const float cf = (float)mt;  // level taken off F (T' sums to zero)

    const int ntx = (g.ndx + RX - 1) / RX;
    const int FP = ntx * RX + TP;  // F row width read (<= 64): the widest tile's reads stay inside
    const int FS = row_pitch(FP);
    const int EY = g.ndy + by - 1, EX = g.ndx + bx - 1;
    float *F = T + bz * by * TP;
    const int wx0 = g.cx - g.hx + g.lox, wy0 = g.cy - g.hy + g.loy, wz0 = g.cz - g.hz + g.loz;
    const int lane = tid & 63, nw = nt >> 6;
    const int rpw = FP <= 32 ? 2 : 1;  // F rows staged per wavefront step
    const int sub = rpw == 2 ? lane >> 5 : 0, xl = rpw == 2 ? lane & 31 : lane;
    Key bk = -INFINITY;
    int bi = INT_MAX;
    for (int z0 = 0; z0 < g.ndz; z0 += p.cz) {
        const int czn = min(p.cz, g.ndz - z0), nrow = (czn + bz - 1) * EY;
        __syncthreads();  // T written / previous run's readers done
        // lanes along x (coalesced rows of flt), zero outside the window
        // region; SU rows per thread in flight before their LDS stores
        const int rstep = nw * rpw;  // <= 8 rows: one wrap of y at most per step
        for (int r0 = (tid >> 6) * rpw + sub; r0 < nrow; r0 += SU * rstep) {
            float v[SU];
            int z = r0 / EY, y = r0 - z * EY;  // (row, plane) of r, advanced per k
#pragma unroll
            for (int k = 0; k < SU; ++k) {
                const int r = r0 + k * rstep;
                v[k] = r < nrow && xl < EX
                           ? (float)flt[(wz0 + z0 + z) * g.sz + (int64_t)(wy0 + y) * g.sy + wx0 +
                                        xl] -
                                 cf
                           : 0.0f;
                y += rstep;
                while (y >= EY) {
                    y -= EY;
                    ++z;
                }
            }
#pragma unroll
            for (int k = 0; k < SU; ++k) {
                const int r = r0 + k * rstep;
                if (r < nrow && xl < FP) F[r * FS + xl] = v[k];
            }
        }
        __syncthreads();
        const int ntile = ntx * g.ndy * czn;
        for (int t = tid; t < ntile; t += nt) {
            const int tx = t % ntx, ty = (t / ntx) % g.ndy, tz = t / (ntx * g.ndy);
            const int dz = g.loz + z0 + tz, dy = g.loy + ty;
            // the tile's ranking records, fetched before the products hide their latency
            const int64_t orow =
                ((int64_t)(g.cz - g.hz + dz) * p.oy + (g.cy - g.hy + dy)) * p.ox + g.cx - g.hx +
                g.lox;
            Key rv[RX];
#pragma unroll
            for (int j = 0; j < RX; ++j)
                rv[j] = tx * RX + j < g.ndx ? Rec<Vox>::r(p.stats, orow + tx * RX + j) : (Key)0;
            float acc[RX];
#pragma unroll
            for (int j = 0; j < RX; ++j) acc[j] = 0.0f;
            for (int z = 0; z < bz; ++z)
                for (int y = 0; y < by; ++y) {
                    const float4 *fr = reinterpret_cast<const float4 *>(
                        F + ((tz + z) * EY + (ty + y)) * FS + tx * RX);
                    const float4 *tr = reinterpret_cast<const float4 *>(T + (z * by + y) * TP);
                    for (int c = 0; c < TP / TU; ++c) {
                        // 16-byte LDS reads: pitches and tile offsets are multiples of 4
                        float f[TU + RX];
#pragma unroll
                        for (int q = 0; q < (TU + RX) / 4; ++q) {
                            const float4 v = fr[c * TU / 4 + q];
                            f[4 * q] = v.x;
                            f[4 * q + 1] = v.y;
                            f[4 * q + 2] = v.z;
                            f[4 * q + 3] = v.w;
                        }
                        const float4 ta = tr[c * TU / 4], tb = tr[c * TU / 4 + 1];
                        const float tv[TU] = {ta.x, ta.y, ta.z, ta.w, tb.x, tb.y, tb.z, tb.w};
#pragma unroll
                        for (int xx = 0; xx < TU; ++xx)
#pragma unroll
                            for (int j = 0; j < RX; ++j) acc[j] = fmaf(tv[xx], f[xx + j], acc[j]);
                    }
                }
            const int irow = ((dz + p.w[2]) * (2 * p.w[1] + 1) + (dy + p.w[1])) * (2 * p.w[0] + 1) +
                             p.w[0];
#pragma unroll
            for (int j = 0; j < RX; ++j) {
                const int ix = tx * RX + j;
                if (ix < g.ndx) {
                    Key k = (Key)acc[j] * rv[j];
                    if (k != k) k = -INFINITY;  // overflowed sums rank last, never unranked
                    better(bk, bi, k, irow + g.lox + ix);
                }
            }
        }
    }
    aniso_finish<Vox, Key>(p, g, blk, bk, bi, mt, s_key, s_idx, red);
}

__device__ inline uint32_t pack2(int lo, int hi) {
    return (uint32_t)(uint16_t)(int16_t)lo | (uint32_t)(uint16_t)(int16_t)hi << 16;
}

// DOT2 form (12-bit data): rows y and y+1 packed per word.
template <int RX>
__global__ __launch_bounds__(NT) void k_match_aniso_dot2(AnisoArgs p) {
    extern __shared__ __align__(16) uint32_t ldsw[];
    __shared__ double red[NT / 64];
    __shared__ double s_key[NT / 64];
    __shared__ int s_idx[NT / 64];
    const int64_t blk = xcd_order(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x, nt = blockDim.x;
    const uint16_t *ref = static_cast<const uint16_t *>(p.ref);
    const uint16_t *flt = static_cast<const uint16_t *>(p.flt);
    const StatU16 *stats = static_cast<const StatU16 *>(p.stats);
    const AGeom g = aniso_geom(p, blk);
    if (!g.inside) {  // uniform: the whole workgroup leaves
        if (tid == 0) write_outside(p, blk);
        return;
    }
    const int bx = g.bx, by = g.by, bz = g.bz;
    const int PY = (by + 1) / 2;  // row pairs of the block (the last one half zero)

    // T'' pair words in LDS [bz][PY][TP], rows padded with zeros; exact sum of T''
    const int TP = (bx + TU - 1) / TU * TU;
    uint32_t *T = ldsw;
    double st = 0.0;
    for (int o = tid; o < g.nb; o += nt) {
        const int x = o % bx, y = (o / bx) % by, z = o / (bx * by);
        st += (double)ref[g.rbase + z * g.sz + (int64_t)y * g.sy + x];
    }
    const double ssum = wg_sum(st, red);  // integer-valued, exact
    const double mt = ssum / g.nb;
    const double sT = ssum - 2048.0 * g.nb;
    for (int e = tid; e < bz * PY * TP; e += nt) {
        const int x = e % TP, r = e / TP, yp = r % PY, z = r / PY;
        const int64_t o = g.rbase + z * g.sz + (int64_t)(2 * yp) * g.sy + x;
        const int lo = x < bx ? (int)ref[o] - 2048 : 0;
        const int hi = x < bx && 2 * yp + 1 < by ? (int)ref[o + g.sy] - 2048 : 0;
        T[e] = pack2(lo, hi);
    }

    const int ntx = (g.ndx + RX - 1) / RX;
    const int FP = ntx * RX + TP;  // F row pitch in words (<= 64)
    const int EY = g.ndy + by - 1, EX = g.ndx + bx - 1;
    uint32_t *F = T + bz * PY * TP;
    const int wx0 = g.cx - g.hx + g.lox, wy0 = g.cy - g.hy + g.loy, wz0 = g.cz - g.hz + g.loz;
    const int lane = tid & 63, nw = nt >> 6;
    const int rpw = FP <= 32 ? 2 : 1;
    const int sub = rpw == 2 ? lane >> 5 : 0, xl = rpw == 2 ? lane & 31 : lane;
    double bk = -INFINITY;
    int bi = INT_MAX;
    for (int z0 = 0; z0 < g.ndz; z0 += p.cz) {
        const int czn = min(p.cz, g.ndz - z0), nrow = (czn + bz - 1) * EY;
        __syncthreads();  // T written / previous run's readers done
        // word (z, u, x) = F''(z, u, x) | F''(z, u + 1, x) << 16 (upper 0 on the last row)
        const int rstep = nw * rpw;
        for (int r0 = (tid >> 6) * rpw + sub; r0 < nrow; r0 += (SU / 2) * rstep) {
            uint32_t v[SU / 2];
#pragma unroll
            for (int k = 0; k < SU / 2; ++k) {
                const int r = r0 + k * rstep, y = r % EY, z = r / EY;
                const bool in = r < nrow && xl < EX;
                const int64_t o = (wz0 + z0 + z) * g.sz + (int64_t)(wy0 + y) * g.sy + wx0 + xl;
                const int lo = in ? (int)flt[o] - 2048 : 0;
                const int hi = in && y + 1 < EY ? (int)flt[o + g.sy] - 2048 : 0;
                v[k] = pack2(lo, hi);
            }
#pragma unroll
            for (int k = 0; k < SU / 2; ++k) {
                const int r = r0 + k * rstep;
                if (r < nrow && xl < FP) F[r * FP + xl] = v[k];
            }
        }
        __syncthreads();
        const int ntile = ntx * g.ndy * czn;
        for (int t = tid; t < ntile; t += nt) {
            const int tx = t % ntx, ty = (t / ntx) % g.ndy, tz = t / (ntx * g.ndy);
            const int dz = g.loz + z0 + tz, dy = g.loy + ty;
            const int64_t orow =
                ((int64_t)(g.cz - g.hz + dz) * p.oy + (g.cy - g.hy + dy)) * p.ox + g.cx - g.hx +
                g.lox;
            int rs[RX];
            float rr[RX];
#pragma unroll
            for (int j = 0; j < RX; ++j) {
                const bool ok = tx * RX + j < g.ndx;
                const StatU16 rec = ok ? stats[orow + tx * RX + j] : StatU16{0, 0.0f};
                rs[j] = rec.s;
                rr[j] = rec.r;
            }
            double dacc[RX];
#pragma unroll
            for (int j = 0; j < RX; ++j) dacc[j] = 0.0;
            for (int z = 0; z < bz; ++z) {
                int acc[RX];  // exact: one plane is at most 15 * 8 two-term products
#pragma unroll
                for (int j = 0; j < RX; ++j) acc[j] = 0;
                for (int yp = 0; yp < PY; ++yp) {
                    const uint4 *fr = reinterpret_cast<const uint4 *>(
                        F + ((tz + z) * EY + (ty + 2 * yp)) * FP + tx * RX);
                    const uint4 *tr = reinterpret_cast<const uint4 *>(T + (z * PY + yp) * TP);
                    for (int c = 0; c < TP / TU; ++c) {
                        uint32_t f[TU + RX];
#pragma unroll
                        for (int q = 0; q < (TU + RX) / 4; ++q) {
                            const uint4 v = fr[c * TU / 4 + q];
                            f[4 * q] = v.x;
                            f[4 * q + 1] = v.y;
                            f[4 * q + 2] = v.z;
                            f[4 * q + 3] = v.w;
                        }
                        const uint4 ta = tr[c * TU / 4], tb = tr[c * TU / 4 + 1];
                        const uint32_t tv[TU] = {ta.x, ta.y, ta.z, ta.w, tb.x, tb.y, tb.z, tb.w};
#pragma unroll
                        for (int xx = 0; xx < TU; ++xx)
#pragma unroll
                            for (int j = 0; j < RX; ++j)
                                acc[j] = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2v, f[xx + j]),
                                                                __builtin_bit_cast(short2v, tv[xx]),
                                                                acc[j], false);
                    }
                }
#pragma unroll
                for (int j = 0; j < RX; ++j) dacc[j] += (double)acc[j];
            }
            const int irow = ((dz + p.w[2]) * (2 * p.w[1] + 1) + (dy + p.w[1])) * (2 * p.w[0] + 1) +
                             p.w[0];
#pragma unroll
            for (int j = 0; j < RX; ++j) {
                const int ix = tx * RX + j;
                if (ix < g.ndx) {
                    // N * covariance (exact in FP64) times 1/sqrt(N var F)
                    const double k = ((double)g.nb * dacc[j] - sT * (double)rs[j]) * (double)rr[j];
                    better(bk, bi, k, irow + g.lox + ix);
                }
            }
        }
    }
    aniso_finish<uint16_t, double>(p, g, blk, bk, bi, mt, s_key, s_idx, red);
}

// Compiled register tiles: RX consecutive x displacements per thread.
struct AnisoTile {
    int rx;
    void (*u16_dot2)(AnisoArgs);
    void (*u16_fma)(AnisoArgs);
    void (*f32)(AnisoArgs);
};
const AnisoTile kTiles[] = {
    {8, k_match_aniso_dot2<8>, k_match_aniso<uint16_t, 8>, k_match_aniso<float, 8>},
    {4, k_match_aniso_dot2<4>, k_match_aniso<uint16_t, 4>, k_match_aniso<float, 4>}};

struct AnisoPlan {
    const AnisoTile *tile;
    int cz;
    size_t lds;
};

// LDS bytes of one workgroup for a z-run of cz displacement planes (the
// float layout; the pair layout of DOT2 needs no more).
size_t aniso_lds(const int32_t b[3], const int32_t w[3], int rx, int cz) {
    const int tp = (b[0] + TU - 1) / TU * TU;
    const int ntx = (2 * w[0] + 1 + rx - 1) / rx;
    const size_t fp = row_pitch(ntx * rx + tp), ey = 2 * w[1] + 1 + b[1] - 1;
    return 4 * ((size_t)b[2] * b[1] * tp + (size_t)(cz + b[2] - 1) * ey * fp);
}

// Largest z-run that fits `budget` bytes of LDS (0: not even one plane).
int aniso_cz(const int32_t b[3], const int32_t w[3], int rx, size_t budget) {
    int cz = 2 * w[2] + 1;
    while (cz > 0 && aniso_lds(b, w, rx, cz) > budget) --cz;
    return cz;
}

// RX = 8 (more products per LDS read) unless the x displacements leave
// more than a quarter more idle tile slots than RX = 4 does.  The z-run is
// the longest that lets six workgroups share a CU's LDS (the kernel is
// latency-bound: more resident blocks beat fewer re-staged planes; on the
// MRI pair with 7x7x3 blocks and 32-word rows 5 planes ran 0.535 ms, the
// whole window of 9 0.569 ms), else two, else one.  NRR_ANISO_TILE=rx and NRR_ANISO_CZ=n force
// the tile and cap the run (for timing sweeps).
bool aniso_plan(const int32_t b[3], const int32_t w[3], AnisoPlan *out) {
    const size_t lim = device_lds_limit();
    const int n = 2 * w[0] + 1;
    int rx = (n + 7) / 8 * 8 * 4 <= (n + 3) / 4 * 4 * 5 ? 8 : 4;
    const char *et = getenv("NRR_ANISO_TILE");
    if (et && *et) rx = atoi(et) == 4 ? 4 : 8;
    const int tp = (b[0] + TU - 1) / TU * TU;
    if ((n + rx - 1) / rx * rx + tp > 64) rx = 4;  // one F row per wavefront step
    if ((n + rx - 1) / rx * rx + tp > 64) return false;
    int cz = aniso_cz(b, w, rx, lim / 6);
    if (cz < 2) cz = aniso_cz(b, w, rx, lim / 2);
    if (cz < 2) cz = aniso_cz(b, w, rx, lim);
    if (cz < 1) return false;
    const char *ec = getenv("NRR_ANISO_CZ");
    if (ec && *ec) cz = max(1, min(cz, atoi(ec)));
    *out = {rx == 8 ? &kTiles[0] : &kTiles[1], cz, aniso_lds(b, w, rx, cz)};
    return true;
}

}  // namespace

const char *aniso_unsupported_reason(const int32_t block[3], const int32_t window[3]) {
    for (int a = 0; a < 3; ++a) {
        if (block[a] > 15) return "block edge above 15 is not built";
        if (window[a] > 15) return "half window above 15 is not built";
    }
    AnisoPlan pl;
    if (!aniso_plan(block, window, &pl)) return "window region does not fit in LDS";
    return nullptr;
}

// 12-bit data take the FMA form too: the DOT2 form halves the LDS reads per
// product but measured slower (0.73 vs 0.57 ms on the MRI pair: its MAC rate
// per instruction is barely above v_fmac's on gfx950, and its staging reads
// two rows per word).  NRR_ANISO_ARITH=dot2 selects it.
hipError_t launch_match_aniso(nrr_dtype dtype, const AnisoArgs &a0, hipStream_t stream) {
    if (a0.n <= 0) return hipSuccess;
    AnisoArgs a = a0;
    AnisoPlan pl;
    if (!aniso_plan(a.b, a.w, &pl)) return hipErrorInvalidValue;
    a.cz = pl.cz;
    void (*fn)(AnisoArgs) = pl.tile->f32;
    if (dtype == NRR_U16) {
        const char *e = getenv("NRR_ANISO_ARITH");
        fn = e && e[0] == 'd' ? pl.tile->u16_dot2 : pl.tile->u16_fma;
    }
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3((unsigned)a.n), dim3(NT), pl.lds, stream, a);
    return hipGetLastError();
}

}  // namespace nrr
