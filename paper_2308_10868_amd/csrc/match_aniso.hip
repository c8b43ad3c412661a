// Exhaustive NCC search with per-axis block edges and half windows.
//
// The paper's parameter list has a half block size and a half search window
// per anatomical axis (the "Deep Learning Model Architecture" section), so a
// block is bx x by x bz and the displacement set [-wx, wx] x [-wy, wy] x
// [-wz, wz].  The cubic search has its own tuned kernels; this is the
// general kernel for any such shape (edges and half windows up to 15).
//
// One workgroup of 256 threads per block (XCD-aware order, so that blocks
// with overlapping windows share an L2).  The reference block T is centred
// in FP64 and kept in LDS as float, its rows padded with zeros to a
// multiple of 8; the moving volume's window region is staged in LDS, a run
// of `cz` displacement planes at a time, by rows with the lanes along x.  A
// thread owns RX consecutive x displacements of one (dy, dz) and
// accumulates X(d) = sum T'(v) F(v + d) with an 8-wide unrolled inner
// product on 16-byte LDS reads (each staged F value feeds up to RX
// products).  As T' sums to zero, X(d) is the cross term of the
// correlation, so X(d) times the displaced block's 1/sqrt(N sum F^2 -
// (sum F)^2) from the statistics table (fetched before the products) ranks
// the displacements like the NCC.  The workgroup's argmax (largest key,
// smallest shift index on ties) is then rescored exactly, in two FP64
// passes over the block, for the reported NCC.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "nrr_internal.h"

namespace nrr {
namespace {

constexpr int NT = 256;
constexpr int TU = 8;  // T row padding and inner-product unroll
constexpr int SU = 16;  // window rows staged per thread per step

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

template <typename Vox, int RX, int RY>
__global__ __launch_bounds__(NT) void k_match_aniso(AnisoArgs p) {
    using Key = typename Rec<Vox>::Key;
    extern __shared__ __align__(16) float lds[];
    __shared__ double red[NT / 64];
    __shared__ Key s_key[NT / 64];
    __shared__ int s_idx[NT / 64];
    const int64_t blk = xcd_order(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x, nt = blockDim.x;  // 128, 192 or 256
    const Vox *ref = static_cast<const Vox *>(p.ref);
    const Vox *flt = static_cast<const Vox *>(p.flt);
    const int bx = p.b[0], by = p.b[1], bz = p.b[2];
    const int wx = p.w[0], wy = p.w[1], wz = p.w[2];
    const int hx = (bx - 1) / 2, hy = (by - 1) / 2, hz = (bz - 1) / 2;
    const int cx = p.centers[3 * blk], cy = p.centers[3 * blk + 1], cz = p.centers[3 * blk + 2];
    if (cx - hx < 0 || cy - hy < 0 || cz - hz < 0 || cx + hx > p.nx - 1 || cy + hy > p.ny - 1 ||
        cz + hz > p.nz - 1) {
        if (tid == 0) {
            p.disp[3 * blk] = p.disp[3 * blk + 1] = p.disp[3 * blk + 2] = 0;
            p.ncc[blk] = NAN;
            p.conf[blk] = 0.0f;
        }
        return;
    }
    // displacements that keep the block inside the volume
    const int lox = max(-wx, hx - cx), loy = max(-wy, hy - cy), loz = max(-wz, hz - cz);
    const int ndx = min(wx, p.nx - 1 - hx - cx) - lox + 1;
    const int ndy = min(wy, p.ny - 1 - hy - cy) - loy + 1;
    const int ndz = min(wz, p.nz - 1 - hz - cz) - loz + 1;
    const int64_t sy = p.nx, sz = (int64_t)p.nx * p.ny;
    const int64_t rbase = (cz - hz) * sz + (int64_t)(cy - hy) * sy + (cx - hx);
    const int nb = bx * by * bz;

    // T' = T - mean(T) in LDS, rows padded to TP with zeros
    const int TP = (bx + TU - 1) / TU * TU;
    float *T = lds;
    double st = 0.0;
    for (int o = tid; o < nb; o += nt) {
        const int x = o % bx, y = (o / bx) % by, z = o / (bx * by);
        st += (double)ref[rbase + z * sz + (int64_t)y * sy + x];
    }
    const double mt = wg_sum(st, red) / nb;
    for (int e = tid; e < bz * by * TP; e += nt) {
        const int x = e % TP, r = e / TP, y = r % by, z = r / by;
        T[e] = x < bx ? (float)((double)ref[rbase + z * sz + (int64_t)y * sy + x] - mt) : 0.0f;
    }
    const float cf = (float)mt;  // level taken off F (T' sums to zero)

    const int ntx = (ndx + RX - 1) / RX;
    const int FP = ntx * RX + TP;  // F row pitch (<= 64): the widest tile's reads stay inside
    const int EY = ndy + by - 1, EX = ndx + bx - 1;
    const int EYa = (ndy + RY - 1) / RY * RY + by - 1;  // rows staged (zero past EY)
    float *F = T + bz * by * TP;
    const int wx0 = cx - hx + lox, wy0 = cy - hy + loy, wz0 = cz - hz + loz;
    const int lane = tid & 63, nw = nt >> 6;
    const int rpw = FP <= 32 ? 2 : 1;  // F rows staged per wavefront step
    const int sub = rpw == 2 ? lane >> 5 : 0, xl = rpw == 2 ? lane & 31 : lane;
    Key bk = -INFINITY;
    int bi = INT_MAX;
    for (int z0 = 0; z0 < ndz; z0 += p.cz) {
        const int czn = min(p.cz, ndz - z0), nrow = (czn + bz - 1) * EYa;
        __syncthreads();  // T written / previous run's readers done
        // lanes along x (coalesced rows of flt), zero outside the window
        // region; SU rows per thread in flight before their LDS stores
        const int rstep = nw * rpw;
        for (int r0 = (tid >> 6) * rpw + sub; r0 < nrow; r0 += SU * rstep) {
            float v[SU];
#pragma unroll
            for (int k = 0; k < SU; ++k) {
                const int r = r0 + k * rstep, y = r % EYa, z = r / EYa;
                v[k] = r < nrow && y < EY && xl < EX
                           ? (float)flt[(wz0 + z0 + z) * sz + (int64_t)(wy0 + y) * sy + wx0 + xl] -
                                 cf
                           : 0.0f;
            }
#pragma unroll
            for (int k = 0; k < SU; ++k) {
                const int r = r0 + k * rstep;
                if (r < nrow && xl < FP) F[r * FP + xl] = v[k];
            }
        }
        __syncthreads();
        const int nty = (ndy + RY - 1) / RY, ntile = ntx * nty * czn;
        for (int t = tid; t < ntile; t += nt) {
            const int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
            const int dz = loz + z0 + tz;
            // the tile's ranking records, fetched before the products hide their latency
            Key rv[RY][RX];
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                const int iy = ty * RY + r;
                const int64_t orow =
                    ((int64_t)(cz - hz + dz) * p.oy + (cy - hy + loy + iy)) * p.ox + cx - hx + lox;
#pragma unroll
                for (int j = 0; j < RX; ++j)
                    rv[r][j] = iy < ndy && tx * RX + j < ndx
                                   ? Rec<Vox>::r(p.stats, orow + tx * RX + j) : (Key)0;
            }
            float acc[RY][RX];
#pragma unroll
            for (int r = 0; r < RY; ++r)
#pragma unroll
                for (int j = 0; j < RX; ++j) acc[r][j] = 0.0f;
            // products of T row y with F row u = y + r (relative to the tile's
            // first row) for output row r: each F row chunk loaded once serves
            // every r with a valid y
            for (int z = 0; z < bz; ++z) {
                const float4 *fz = reinterpret_cast<const float4 *>(
                    F + ((tz + z) * EYa + ty * RY) * FP + tx * RX);
                const float4 *tz4 = reinterpret_cast<const float4 *>(T + z * by * TP);
                for (int u = 0; u < by + RY - 1; ++u) {
                    const bool all = u >= RY - 1 && u < by;  // every r has a block row
                    for (int c = 0; c < TP / TU; ++c) {
                        float f[TU + RX];
#pragma unroll
                        for (int q = 0; q < (TU + RX) / 4; ++q) {
                            const float4 v = fz[(u * FP + c * TU) / 4 + q];
                            f[4 * q] = v.x;
                            f[4 * q + 1] = v.y;
                            f[4 * q + 2] = v.z;
                            f[4 * q + 3] = v.w;
                        }
#pragma unroll
                        for (int r = 0; r < RY; ++r) {
                            const int y = u - r;
                            if (!all && (y < 0 || y >= by)) continue;
                            const float4 ta = tz4[(y * TP + c * TU) / 4];
                            const float4 tb = tz4[(y * TP + c * TU) / 4 + 1];
                            const float tv[TU] = {ta.x, ta.y, ta.z, ta.w, tb.x, tb.y, tb.z, tb.w};
#pragma unroll
                            for (int xx = 0; xx < TU; ++xx)
#pragma unroll
                                for (int j = 0; j < RX; ++j)
                                    acc[r][j] = fmaf(tv[xx], f[xx + j], acc[r][j]);
                        }
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                const int iy = ty * RY + r;
                const int irow = ((dz + wz) * (2 * wy + 1) + (loy + iy + wy)) * (2 * wx + 1) + wx;
#pragma unroll
                for (int j = 0; j < RX; ++j) {
                    const int ix = tx * RX + j;
                    if (iy < ndy && ix < ndx) {
                        Key k = (Key)acc[r][j] * rv[r][j];
                        if (k != k) k = -INFINITY;  // overflowed sums rank last, never unranked
                        better(bk, bi, k, irow + lox + ix);
                    }
                }
            }
        }
    }
    // workgroup argmax
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
    const int sxn = 2 * wx + 1, syn = 2 * wy + 1;
    const int dx = bi % sxn - wx, dy = (bi / sxn) % syn - wy, dz = bi / (sxn * syn) - wz;

    // exact NCC of the winner: two FP64 passes over the block
    const int64_t fbase = rbase + dz * sz + (int64_t)dy * sy + dx;
    double sf = 0.0;
    for (int o = tid; o < nb; o += nt) {
        const int x = o % bx, y = (o / bx) % by, z = o / (bx * by);
        sf += (double)flt[fbase + z * sz + (int64_t)y * sy + x];
    }
    const double mf = wg_sum(sf, red) / nb;
    double a = 0.0, b = 0.0, x2 = 0.0;
    for (int o = tid; o < nb; o += nt) {
        const int x = o % bx, y = (o / bx) % by, z = o / (bx * by);
        const int64_t off = z * sz + (int64_t)y * sy + x;
        const double tv = (double)ref[rbase + off] - mt, fv = (double)flt[fbase + off] - mf;
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

// Compiled register tiles: RX consecutive x displacements per thread.
struct AnisoTile {
    int rx, ry;
    void (*u16)(AnisoArgs);
    void (*f32)(AnisoArgs);
};
#define NRR_ANISO_TILE(X, Y) {X, Y, k_match_aniso<uint16_t, X, Y>, k_match_aniso<float, X, Y>}
// (RY > 1 reuses each staged F row for RY output rows but measured slower on
// gfx950 for the blocks tried, so only RY = 1 is built.)
const AnisoTile kTiles[] = {NRR_ANISO_TILE(8, 1), NRR_ANISO_TILE(4, 1)};
#undef NRR_ANISO_TILE

struct AnisoPlan {
    const AnisoTile *tile;
    int cz;
    size_t lds;
};

// LDS bytes of one workgroup for a z-run of cz displacement planes.
size_t aniso_lds(const int32_t b[3], const int32_t w[3], int rx, int ry, int cz) {
    const int tp = (b[0] + TU - 1) / TU * TU;
    const int ntx = (2 * w[0] + 1 + rx - 1) / rx;
    const size_t fp = (size_t)ntx * rx + tp, ey = (2 * w[1] + 1 + ry - 1) / ry * ry + b[1] - 1;
    return 4 * ((size_t)b[2] * b[1] * tp + (size_t)(cz + b[2] - 1) * ey * fp);
}

// Largest z-run that fits `budget` bytes of LDS (0: not even one plane).
int aniso_cz(const int32_t b[3], const int32_t w[3], int rx, int ry, size_t budget) {
    int cz = 2 * w[2] + 1;
    while (cz > 0 && aniso_lds(b, w, rx, ry, cz) > budget) --cz;
    return cz;
}

// RX = 8 (more products per LDS read) unless the x displacements leave
// more than a quarter more idle tile slots than RX = 4 does; the z-run is
// the longest that lets two workgroups share a CU's LDS, else one.
// NRR_ANISO_TILE=rx forces the tile (for timing sweeps).
bool aniso_plan(const int32_t b[3], const int32_t w[3], AnisoPlan *out) {
    const size_t lim = device_lds_limit();
    const int n = 2 * w[0] + 1;
    int rx = (n + 7) / 8 * 8 * 4 <= (n + 3) / 4 * 4 * 5 ? 8 : 4, ry = 1;
    if (const char *e = getenv("NRR_ANISO_TILE")) sscanf(e, "%d,%d", &rx, &ry);
    const int tp = (b[0] + TU - 1) / TU * TU;
    if ((n + rx - 1) / rx * rx + tp > 64) rx = 4, ry = 1;  // one F row per wavefront step
    if ((n + rx - 1) / rx * rx + tp > 64) return false;
    const AnisoTile *tile = nullptr;
    for (const AnisoTile &t : kTiles)
        if (t.rx == rx && t.ry == ry) tile = &t;
    if (!tile) return false;
    int cz = aniso_cz(b, w, rx, ry, lim / 2);
    if (cz < 2) cz = aniso_cz(b, w, rx, ry, lim);
    if (cz < 1) return false;
    *out = {tile, cz, aniso_lds(b, w, rx, ry, cz)};
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

hipError_t launch_match_aniso(nrr_dtype dtype, const AnisoArgs &a0, hipStream_t stream) {
    if (a0.n <= 0) return hipSuccess;
    AnisoArgs a = a0;
    AnisoPlan pl;
    if (!aniso_plan(a.b, a.w, &pl)) return hipErrorInvalidValue;
    a.cz = pl.cz;
    void (*fn)(AnisoArgs) = dtype == NRR_U16 ? pl.tile->u16 : pl.tile->f32;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3((unsigned)a.n), dim3(NT), pl.lds, stream, a);
    return hipGetLastError();
}

}  // namespace nrr
