// Exhaustive NCC block matching on gfx950.
//
// The paper's GPU algorithm (GPU section) maps one image block to one thread
// block, spreads the loop over the candidate displacements of the search
// window across the threads, and then takes the maximum similarity and its
// displacement.  This kernel keeps that outer mapping (one workgroup per
// selected block) and re-designs the inner part for CDNA:
//
//  * the block's search window of `flt` is staged in LDS, a run of CZ
//    displacement planes at a time (z-chunks, so any window size fits), and
//    the pre-operative block T is staged beside it; every staged voxel is
//    then reused by all displacements that touch it;
//  * each thread owns an RX x RY tile of (dx, dy) displacements at one dz and
//    keeps RX*RY accumulators in registers; a window row read from LDS is
//    reused by every (tile displacement, block column) pair that needs it;
//    LDS is read as single aligned dwords (4 bytes per staged element);
//  * two arithmetic forms of the cross term sum_o T(o) F(o+d):
//      DOT2 (12-bit data, exact): T' = T-2048 and F' = F-2048 as int16
//        pairs of planes (z, z+1), multiplied and accumulated exactly in int32
//        by v_dot2_i32_i16; the block's planes are grouped so no int32 partial
//        sum can overflow (|T'|, |F'| <= 2048);
//      FMA (any data): T^ = T - mean(T) in FP32 against F - c (c = the
//        block mean, rounded to an integer for 12-bit data) with v_fmac_f32,
//        summed in FP32 per block plane, then across planes (FP64 for 12-bit
//        data);
//  * the window statistics (sum F and 1/sqrt of its spread) come from a
//    per-voxel table computed once per call (stats.hip), so the epilogue per
//    displacement is a handful of operations;
//  * displacements are ranked by key = cov * rsqrt(varF), proportional to the
//    NCC (the block's own spread is a constant factor); the argmax keeps the
//    smallest shift index among equal keys and is reduced across the
//    workgroup with wavefront shuffles;
//  * the NCC reported for the winning displacement is recomputed exactly
//    (integer sums for 12-bit data, two-pass FP64 for float data) from the
//    volumes, so it does not inherit the ranking arithmetic's rounding.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "nrr_internal.h"

namespace nrr {
namespace {

typedef short short2v __attribute__((ext_vector_type(2)));
// LDS dword read one at a time: the volatile qualifier keeps the compiler from
// merging neighbouring window reads into wider, misaligned LDS accesses, and
// the LDS address space keeps them ds_read_b32 with immediate offsets.
typedef __attribute__((address_space(3))) const volatile uint32_t lds_word;

constexpr int MAX_B = 15;  // largest block edge served
constexpr int ZPAD = 1;    // padding dwords after each staged window plane
enum Arith { DOT2 = 0, FMA = 1 };

struct Params {
    const void *ref;
    const void *flt;
    int nx, ny, nz;
    const int32_t *centers;
    int64_t n;
    int64_t first;  // first block of this launch
    int w;
    int cz;  // displacement planes per z-chunk
    const void *stats;  // StatU16 / StatF32 records over block origins
    const uint32_t *pv;  // plane-pair volume of flt (12-bit data)
    int ox, oy;
    int32_t *disp;
    float *ncc;
    float *conf;
    float *surface;  // optional ranking NCC per displacement (diagnostic instantiations)
};

// Workgroup index -> block index such that consecutive blocks (overlapping
// windows) land on the same XCD, which round-robins workgroups by index.
__device__ inline int64_t xcd_block(int64_t wg, int64_t n) {
    const int64_t q = n / 8, r = n % 8, k = wg % 8, j = wg / 8;
    return k * q + (k < r ? k : r) + j;
}

// Per-block search geometry: valid displacement range per axis (displaced
// block fully inside the volume) and the window origin in `flt`.
struct Geom {
    int cx, cy, cz;
    int lox, loy, loz;
    int dx, dy, dz;     // number of valid displacements per axis
    int wx0, wy0, wz0;  // window origin = c - h + lo
    bool inside;
};

__device__ inline Geom make_geom(const Params &p, int64_t blk, int h) {
    Geom g;
    g.cx = p.centers[3 * blk];
    g.cy = p.centers[3 * blk + 1];
    g.cz = p.centers[3 * blk + 2];
    g.inside = g.cx - h >= 0 && g.cy - h >= 0 && g.cz - h >= 0 && g.cx + h <= p.nx - 1 &&
               g.cy + h <= p.ny - 1 && g.cz + h <= p.nz - 1;
    g.lox = max(-p.w, h - g.cx);
    g.loy = max(-p.w, h - g.cy);
    g.loz = max(-p.w, h - g.cz);
    g.dx = min(p.w, p.nx - 1 - h - g.cx) - g.lox + 1;
    g.dy = min(p.w, p.ny - 1 - h - g.cy) - g.loy + 1;
    g.dz = min(p.w, p.nz - 1 - h - g.cz) - g.loz + 1;
    g.wx0 = g.cx - h + g.lox;
    g.wy0 = g.cy - h + g.loy;
    g.wz0 = g.cz - h + g.loz;
    return g;
}

template <typename K>
__device__ inline void better(K &bk, int &bi, K k, int i) {
    if (k > bk || (k == bk && i < bi)) {
        bk = k;
        bi = i;
    }
}

// Workgroup argmax of (key, shift index): largest key, smallest index on ties.
template <int NT, typename K>
__device__ inline void wg_argmax(K &key, int &idx, K *s_key, int *s_idx) {
    for (int off = 32; off > 0; off >>= 1) {
        K ok = __shfl_xor(key, off);
        int oi = __shfl_xor(idx, off);
        better(key, idx, ok, oi);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_key[w] = key;
        s_idx[w] = idx;
    }
    __syncthreads();
    key = s_key[0];
    idx = s_idx[0];
    for (int i = 1; i < NT / 64; ++i) better(key, idx, s_key[i], s_idx[i]);
    __syncthreads();
}

template <int NT, typename T, int NV>
__device__ inline void wg_sum(T (&v)[NV], T *s_red) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) s_red[w * NV + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        T s = 0;
        for (int i = 0; i < NT / 64; ++i) s += s_red[i * NV + k];
        v[k] = s;
    }
    __syncthreads();
}

__device__ inline void write_result(const Params &p, int64_t blk, int dx, int dy, int dz,
                                    float v) {
    p.disp[3 * blk] = dx;
    p.disp[3 * blk + 1] = dy;
    p.disp[3 * blk + 2] = dz;
    p.ncc[blk] = v;
    p.conf[blk] = v > 0.0f ? v : 0.0f;
}

// Stage planes [z0, z0 + pz) of the window into LDS as 4-byte elements at
// z*plane + y*pitch + x (plane >= py*pitch); element (z, y, x) = make(a, b, nb)
// where a = src(z0+z, y0+y, x0+x) and, with PAIR, b = the same voxel of the
// next plane (nb = false and b = 0 past plane `ez`), for y < ey and x < ex;
// 0 elsewhere (tile padding).  Each lane moves chunks of 4 consecutive x;
// UNR chunks per lane are loaded before any is written so several global
// loads are in flight, and the chunk coordinates advance incrementally (no
// integer division in the loop).
template <int NT, bool PAIR, int UNR, typename Src, typename Make>
__device__ inline void stage_planes(const Src *__restrict__ src, int nx, int ny, int x0, int y0,
                                    int z0, int ex, int ey, int ez, uint32_t *__restrict__ dst,
                                    int pitch, int plane, int py, int pz, Make make) {
    const int cpr = (pitch + 3) >> 2;  // chunks per row
    const int total = pz * py * cpr;
    const int drow = NT / cpr, dxc = NT - drow * cpr;
    int row = (int)threadIdx.x / cpr;
    int xc = (int)threadIdx.x - row * cpr;
    int z = row / py, y = row - z * py;
    for (int c0 = 0; c0 < total; c0 += NT * UNR) {
        Src a[UNR][4], b[UNR][4];
        int base[UNR], xs[UNR];
        bool rin[UNR], nin[UNR], live[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            live[u] = c0 + u * NT + (int)threadIdx.x < total;
            xs[u] = 4 * xc;
            base[u] = z * plane + y * pitch + 4 * xc;
            rin[u] = live[u] && y < ey && z < ez;
            nin[u] = PAIR && rin[u] && z + 1 < ez;
            const Src *s = src + ((int64_t)(z0 + z) * ny + (y0 + y)) * nx + (x0 + 4 * xc);
            const Src *s1 = s + (int64_t)ny * nx;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bool in = 4 * xc + e < ex;
                a[u][e] = (rin[u] && in) ? s[e] : Src(0);
                b[u][e] = (PAIR && nin[u] && in) ? s1[e] : Src(0);
            }
            xc += dxc;
            y += drow;
            if (xc >= cpr) {
                xc -= cpr;
                ++y;
            }
            while (y >= py) {
                y -= py;
                ++z;
            }
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            if (!live[u]) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int x = xs[u] + e;
                if (x < pitch) {
                    const bool in = rin[u] && x < ex;
                    dst[base[u] + e] = in ? make(a[u][e], b[u][e], nin[u]) : 0u;
                }
            }
        }
    }
}

// Stage planes [z0, z0 + pz) of the window from the plane-pair volume as
// plain copies into LDS at z*plane + y*pitch + x, with `pitch` and `plane`
// multiples of CW words.  Each lane moves whole CW-word row chunks (one
// global and one LDS access each); rows at or past `ey` re-read row ey-1 and
// columns past the window's own width read whatever follows in the volume
// row (the pair volume carries slack at its end), so no load needs a
// predicate.  Those extra words only feed displacements that are masked out.
template <int CW>
struct Chunk {
    typedef uint32_t type __attribute__((ext_vector_type(CW), aligned(4)));
};
constexpr int CW = 4;  // row chunk width of the DOT2 window (16-byte copies)

template <int NT, int UNR>
__device__ inline void stage_rows(const uint32_t *__restrict__ src, int nx, int ny, int x0, int y0,
                                  int z0, int ey, uint32_t *__restrict__ dst, int pitch,
                                  int plane, int py, int pz) {
    using V = typename Chunk<CW>::type;
    const int cpr = pitch / CW;  // chunks per row
    const int total = pz * py * cpr;
    const int drow = NT / cpr, dxc = NT - drow * cpr;
    int row = (int)threadIdx.x / cpr;
    int xc = (int)threadIdx.x - row * cpr;
    int z = row / py, y = row - z * py;
    for (int c0 = 0; c0 < total; c0 += NT * UNR) {
        V v[UNR];
        int off[UNR];
        bool live[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            live[u] = c0 + u * NT + (int)threadIdx.x < total;
            const int zz = live[u] ? z : 0, yy = min(y, ey - 1);
            const uint32_t *s = src + ((int64_t)(z0 + zz) * ny + (y0 + yy)) * nx + (x0 + CW * xc);
            v[u] = *reinterpret_cast<const V *>(s);
            off[u] = z * plane + y * pitch + CW * xc;
            xc += dxc;
            y += drow;
            if (xc >= cpr) {
                xc -= cpr;
                ++y;
            }
            while (y >= py) {
                y -= py;
                ++z;
            }
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u)
            if (live[u]) *reinterpret_cast<V *>(dst + off[u]) = v[u];
    }
}

// The same row-chunk staging for float volumes, storing F - c: a chunk that
// would run past the end of a volume row (the window's right edge at the
// volume border) reads its elements one by one, clamped into the row (the
// extra values only feed masked displacements).
template <int NT, int UNR>
__device__ inline void stage_rows_f32(const float *__restrict__ src, int nx, int ny, int x0, int y0,
                                      int z0, int ey, uint32_t *__restrict__ dst, int pitch,
                                      int plane, int py, int pz, float c) {
    using V = typename Chunk<CW>::type;
    const int cpr = pitch / CW;
    const int total = pz * py * cpr;
    const int drow = NT / cpr, dxc = NT - drow * cpr;
    int row = (int)threadIdx.x / cpr;
    int xc = (int)threadIdx.x - row * cpr;
    int z = row / py, y = row - z * py;
    for (int c0 = 0; c0 < total; c0 += NT * UNR) {
        float v[UNR][CW];
        int off[UNR];
        bool live[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            live[u] = c0 + u * NT + (int)threadIdx.x < total;
            const int zz = live[u] ? z : 0, yy = min(y, ey - 1), xs = x0 + CW * xc;
            const float *r = src + ((int64_t)(z0 + zz) * ny + (y0 + yy)) * nx;
            if (xs + CW <= nx) {
                const V w = *reinterpret_cast<const V *>(r + xs);
#pragma unroll
                for (int e = 0; e < CW; ++e) v[u][e] = __uint_as_float(w[e]);
            } else {
#pragma unroll
                for (int e = 0; e < CW; ++e) v[u][e] = r[min(xs + e, nx - 1)];
            }
            off[u] = z * plane + y * pitch + CW * xc;
            xc += dxc;
            y += drow;
            if (xc >= cpr) {
                xc -= cpr;
                ++y;
            }
            while (y >= py) {
                y -= py;
                ++z;
            }
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u)
            if (live[u]) {
                // word writes: rows start at any word (odd plane stride)
#pragma unroll
                for (int e = 0; e < CW; ++e) dst[off[u] + e] = __float_as_uint(v[u][e] - c);
            }
    }
}

// Exact int32 grouping for DOT2: a plane contributes at most B*B*2048*2048.
template <int B>
struct Groups {
    static constexpr int P = (B + 1) / 2;  // plane pairs of the block
    static constexpr long long PLANE_MAX = (long long)B * B * 2048 * 2048;
    static constexpr int GPAIRS = (int)(2147483647LL / PLANE_MAX) / 2;  // pairs per group
    static constexpr int NG = (P + GPAIRS - 1) / GPAIRS;
    static_assert(GPAIRS >= 1, "block edge too large for exact int32 groups");
};

// DOT2 cross terms X(d) = sum_o T'(o) F'(o + d) of an RX x RY tile of
// displacements at one dz: `tp` is the block's pair table [P][B][BP], `base`
// the tile's first window row and column, and the window plane of pair m is
// in ring slot (slot + 2m) mod R.  Exact: int32 groups of plane pairs that
// cannot overflow, combined in FP64 when a block needs more than one.
template <int B, int RX, int RY, typename XT>
__device__ __attribute__((always_inline)) inline void dot2_cross(
    const uint32_t *tp, const uint32_t *base, int slot, int R, int plane, int pitch,
    XT (&xacc)[RX][RY]) {
    constexpr int P = Groups<B>::P, GP = Groups<B>::GPAIRS, NG = Groups<B>::NG;
    constexpr int BP = (B + 3) & ~3;
    int acc[RX][RY], acc0[RX][RY];
    double dacc[NG > 2 ? RX : 1][NG > 2 ? RY : 1];
#pragma unroll
    for (int i = 0; i < RX; ++i)
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            acc[i][j] = 0;
            acc0[i][j] = 0;
            if constexpr (NG > 2) dacc[i][j] = 0.0;
        }
    for (int m = 0; m < P; ++m) {
        int tq[B][B];
        const uint32_t *tpm = tp + m * B * BP;
#pragma unroll
        for (int oy = 0; oy < B; ++oy)
#pragma unroll
            for (int ox = 0; ox < B; ++ox)  // uniform: kept in scalar registers
                tq[oy][ox] = __builtin_amdgcn_readfirstlane((int)tpm[oy * BP + ox]);
        const lds_word *wm = (const lds_word *)(base + slot * plane);
        slot += 2;
        if (slot >= R) slot -= R;
        // rows are software-pipelined: row yw+1 is read while row yw
        // is multiplied
        int fr[2][RX + B - 1];
#pragma unroll
        for (int xw = 0; xw < RX + B - 1; ++xw) fr[0][xw] = (int)wm[xw];
#pragma unroll
        for (int yw = 0; yw < RY + B - 1; ++yw) {
            if (yw + 1 < RY + B - 1) {
#pragma unroll
                for (int xw = 0; xw < RX + B - 1; ++xw)
                    fr[(yw + 1) & 1][xw] = (int)wm[(yw + 1) * pitch + xw];
            }
            const int *f = fr[yw & 1];
#pragma unroll
            for (int j = 0; j < RY; ++j) {
                const int oy = yw - j;
                if (oy < 0 || oy >= B) continue;
#pragma unroll
                for (int i = 0; i < RX; ++i)
#pragma unroll
                    for (int ox = 0; ox < B; ++ox)
                        acc[i][j] = __builtin_amdgcn_sdot2(
                            __builtin_bit_cast(short2v, f[i + ox]),
                            __builtin_bit_cast(short2v, tq[oy][ox]), acc[i][j],
                            false);
            }
        }
        if constexpr (NG == 2) {
            if (m == GP - 1) {
#pragma unroll
                for (int i = 0; i < RX; ++i)
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        acc0[i][j] = acc[i][j];
                        acc[i][j] = 0;
                    }
            }
        } else if constexpr (NG > 2) {
            if ((m + 1) % GP == 0) {
#pragma unroll
                for (int i = 0; i < RX; ++i)
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        dacc[i][j] += (double)acc[i][j];
                        acc[i][j] = 0;
                    }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < RX; ++i)
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            if constexpr (NG == 1)
                xacc[i][j] = acc[i][j];
            else if constexpr (NG == 2)
                xacc[i][j] = (double)acc0[i][j] + (double)acc[i][j];
            else
                xacc[i][j] = dacc[i][j] + (double)acc[i][j];
        }
}

// Ranking of a tile: key = N*cov * rsqrt(N*varF), proportional to the NCC for
// the block at hand; keeps the largest key and, among equal keys, the
// smallest shift index (irow + j*side + i).  Displacements past the valid
// extents (nvx, nvy) are masked without a branch.  For 12-bit data the staged
// F sums are offset by `fshift` from the table's.
template <bool U16, bool SHIFT, int RX, int RY, typename Rec, typename XT, typename KeyT,
          bool SURF = false>
__device__ __attribute__((always_inline)) inline void rank_tile(
    const Rec (&rec)[RX][RY], const XT (&xacc)[RX][RY], double dN, double tsum, double fshift,
    float c, int nvx, int nvy, int irow, int side, KeyT &tk, int &ti, float *surf = nullptr,
    double inv_vt = 0.0) {
#pragma unroll
    for (int j = 0; j < RY; ++j)
#pragma unroll
        for (int i = 0; i < RX; ++i) {  // increasing shift index
            const bool valid = i < nvx && j < nvy;
            KeyT key;
            if constexpr (U16) {
                const double cov =
                    __builtin_fma(dN, (double)xacc[i][j],
                                  -tsum * (SHIFT ? (double)rec[i][j].s + fshift : (double)rec[i][j].s));
                key = (float)cov * rec[i][j].r;
            } else {
                const double cov = dN * (double)xacc[i][j] - tsum * (rec[i][j].s - dN * (double)c);
                key = cov * rec[i][j].r;
            }
            const bool take = valid && key > tk;  // ties keep the smaller index
            tk = take ? key : tk;
            ti = take ? irow + j * side + i : ti;
            if constexpr (SURF)  // NCC = key / sqrt(N varT)
                if (valid) surf[irow + j * side + i] = (float)((double)key * inv_vt);
        }
}

// Workgroup scratch of the reductions (any NT <= 1024).
struct Small {
    double key[16];
    int idx[16];
    long long red[16 * 5];
    double redd[16 * 3];
};

// Search of one block `blk` (its window staged in `lds`); the body shared by
// the per-block kernel and the batched kernel.  Every thread of the NT-wide
// workgroup calls it; it ends with all LDS reads done by the thread itself,
// so a caller that reuses LDS for another block synchronises first.
template <typename Vox, int ARITH, int B, int RX, int RY, int NT, bool PF, bool SURF = false>
__device__ __attribute__((always_inline)) inline void match_one(const Params &p, int64_t blk,
                                                                unsigned char *lds, Small &sm) {
    constexpr bool U16 = sizeof(Vox) == 2;
    static_assert(ARITH == FMA || U16, "DOT2 needs 12-bit data");
    constexpr int H = (B - 1) / 2, N = B * B * B, BP = (B + 3) & ~3;
    constexpr int P = Groups<B>::P, GP = Groups<B>::GPAIRS, NG = Groups<B>::NG;
    constexpr int TPL = ARITH == DOT2 ? P : B;  // block planes (pairs) in the T table
    constexpr int TP_WORDS = TPL * B * BP;
    using KeyT = typename std::conditional<U16, float, double>::type;
    uint32_t *tp = reinterpret_cast<uint32_t *>(lds);                  // [TPL][B][BP]
    uint32_t *win = reinterpret_cast<uint32_t *>(lds + TP_WORDS * 4);  // [cz+B-1][PY][PX]
    KeyT *s_key = reinterpret_cast<KeyT *>(sm.key);
    int *s_idx = sm.idx;
    long long *s_red = sm.red;
    double *s_redd = sm.redd;
    static_assert(NT <= 1024, "reduction scratch is sized for 16 wavefronts");

    const Geom g = make_geom(p, blk, H);
    const int tid = threadIdx.x;
    if (!g.inside) {
        if (tid == 0) write_result(p, blk, 0, 0, 0, NAN);
        return;
    }
    const Vox *ref = static_cast<const Vox *>(p.ref);
    const Vox *flt = static_cast<const Vox *>(p.flt);
    const int txn = (g.dx + RX - 1) / RX, tyn = (g.dy + RY - 1) / RY;
    const int PX = txn * RX + B - 1, PY = tyn * RY + B - 1;
    // LDS row pitch: DOT2 and float windows are staged in whole CW-word chunks
    constexpr bool ROWS = ARITH == DOT2 || !U16;
    const int pitch = ROWS ? (PX + CW - 1) / CW * CW : PX;
    const int ex = g.dx + B - 1, ey = g.dy + B - 1;
    auto tval = [&](int o) {
        const int oz = o / (B * B), oy = (o / B) % B, ox = o % B;
        return ref[((int64_t)(g.cz - H + oz) * p.ny + (g.cy - H + oy)) * p.nx + (g.cx - H + ox)];
    };

    // ---- block statistics and the staged T table
    // Plane stride: lanes of a wavefront take consecutive dz, so the stride
    // spreads their reads over the LDS banks: odd (one pad dword) for the
    // element-staged and the float windows, 4 x odd for the 12-bit
    // chunk-staged windows (whole 16-byte chunks: 16 consecutive planes still
    // hit distinct banks).
    // (float windows: an odd plane stride in words, since their products
    // read single words with consecutive lanes on consecutive dz planes; a
    // stride of 4 x odd words put 64 lanes on 8 banks)
    const int plane = ROWS ? (U16 ? PY * pitch + (((PY * pitch / CW) & 1) ? 0 : CW)
                                  : PY * pitch + 1)
                           : PY * pitch + ZPAD;
    auto stage_chunk = [&](int zc0, int ezc, float c) {
        if constexpr (ARITH == DOT2)  // plain copies of the precomputed pair words
            stage_rows<NT, 8>(p.pv, p.nx, p.ny, g.wx0, g.wy0, g.wz0 + zc0, ey, win, pitch,
                                  plane, PY, ezc);
        else if constexpr (!U16)
            stage_rows_f32<NT, 4>(reinterpret_cast<const float *>(flt), p.nx, p.ny, g.wx0, g.wy0,
                                  g.wz0 + zc0, ey, win, pitch, plane, PY, ezc, c);
        else
            stage_planes<NT, false, 4>(
                flt, p.nx, p.ny, g.wx0, g.wy0, g.wz0 + zc0, ex, ey, ezc, win, PX, plane, PY, ezc,
                [c](Vox a, Vox, bool) { return __float_as_uint((float)a - c); });
    };
    long long st[2] = {0, 0};  // 12-bit: exact sums of T and T^2
    double tmean;
    double vtn = 0.0;  // N sum T^2 - (sum T)^2 of the T actually used (surface output)
    long long sT = 0;   // DOT2: sum (T - 2048)
    double sTc = 0.0;   // FMA: sum of the centred float T^ actually used
    float c = 0.0f;     // FMA: F is staged as F - c
    if constexpr (ARITH == DOT2) {
        // one pass: each T voxel is read once, into its plane-pair word, and
        // counted into the exact sums; the first window chunk's loads are
        // issued before the reduction's barrier so both latencies overlap
        for (int i = tid; i < TP_WORDS; i += NT) {
            const int pl = i / (B * BP), oy = (i / BP) % B, ox = i % BP;
            uint32_t w = 0;
            if (ox < B) {
                const int z0 = 2 * pl, z1 = 2 * pl + 1;
                const int lo = (int)tval((z0 * B + oy) * B + ox);
                const int hi = z1 < B ? (int)tval((z1 * B + oy) * B + ox) : 2048;
                st[0] += lo + (z1 < B ? hi : 0);
                st[1] += (long long)lo * lo + (z1 < B ? (long long)hi * hi : 0);
                w = (uint32_t)(uint16_t)(lo - 2048) | ((uint32_t)(uint16_t)(hi - 2048) << 16);
            }
            tp[i] = w;
        }
        stage_chunk(0, min(p.cz, g.dz) + B - 1, 0.0f);
        wg_sum<NT, long long, 2>(st, s_red);  // its barrier also publishes tp and the window
        if ((long long)N * st[1] - st[0] * st[0] == 0) {  // flat block: all NCC are 0
            if (tid == 0) write_result(p, blk, g.lox, g.loy, g.loz, 0.0f);
            return;
        }
        tmean = (double)st[0] / (double)N;
        sT = st[0] - 2048ll * N;
        vtn = (double)((long long)N * st[1] - st[0] * st[0]);
    } else {
        double sd[1] = {0.0};
        for (int o = tid; o < N; o += NT) {
            const Vox v = tval(o);
            if constexpr (U16) {
                st[0] += v;
                st[1] += (long long)v * v;
            }
            sd[0] += (double)v;
        }
        wg_sum<NT, double, 1>(sd, s_redd);
        tmean = sd[0] / (double)N;
        if constexpr (U16) wg_sum<NT, long long, 2>(st, s_red);
        // 12-bit data keep c an integer (exact floats)
        c = U16 ? (float)llrint(tmean) : (float)tmean;
        double ctr[2] = {0.0, 0.0};  // sum T^, sum T^^2 of the float values used
        for (int i = tid; i < TP_WORDS; i += NT) {
            const int pl = i / (B * BP), oy = (i / BP) % B, ox = i % BP;
            uint32_t w = 0;
            if (ox < B) {
                const float v = (float)((double)tval((pl * B + oy) * B + ox) - tmean);
                ctr[0] += (double)v;
                ctr[1] += (double)v * (double)v;
                w = __float_as_uint(v);
            }
            tp[i] = w;
        }
        stage_chunk(0, min(p.cz, g.dz) + B - 1, c);
        wg_sum<NT, double, 2>(ctr, s_redd);  // barrier publishes tp and the window
        sTc = ctr[0];
        vtn = (double)N * ctr[1] - ctr[0] * ctr[0];
        if (!(ctr[1] > 0.0)) {  // flat block
            if (tid == 0) write_result(p, blk, g.lox, g.loy, g.loz, 0.0f);
            return;
        }
    }

    // ---- exhaustive search, one z-chunk of displacement planes at a time
    const double dN = (double)N;
    const int side = 2 * p.w + 1;
    KeyT bk = -INFINITY;
    int bi = INT_MAX;
    // DOT2 keeps the staged planes in a ring of R plane slots (window plane q
    // in slot q mod R), so a later chunk stages only the planes it adds
    const int R = min(p.cz, g.dz) + B - 1;
    int staged = R;  // window planes [0, staged) staged so far (chunk 0 above)
    for (int zc0 = 0; zc0 < g.dz; zc0 += p.cz) {
        const int czn = min(p.cz, g.dz - zc0);  // displacement planes in this chunk
        const int ezc = czn + B - 1;            // window planes in this chunk
        if (zc0 > 0) {                          // the first chunk was staged above
            __syncthreads();                    // previous chunk fully consumed
            if constexpr (ARITH == DOT2) {
                // new planes [staged, zc0 + ezc) replace planes below zc0
                for (int q = staged; q < zc0 + ezc;) {
                    const int slot = q % R, n = min(zc0 + ezc - q, R - slot);
                    stage_rows<NT, 8>(p.pv, p.nx, p.ny, g.wx0, g.wy0, g.wz0 + q, ey,
                                          win + slot * plane, pitch, plane, PY, n);
                    q += n;
                }
                staged = zc0 + ezc;
            } else {
                stage_chunk(zc0, ezc, c);
            }
            __syncthreads();
        }
        const int ntiles = txn * tyn * czn;
        for (int t = tid; t < ntiles; t += NT) {
            // consecutive lanes take consecutive dz (then x, then y tiles): with
            // the plane padding this spreads a wavefront's reads over the banks
            const int dzl = t % czn, tx = (t / czn) % txn, ty = t / (czn * txn);
            const int dz = zc0 + dzl;
            const uint32_t *base =
                win + (ARITH == DOT2 ? 0 : dzl * plane) + ty * RY * pitch + tx * RX;
            // the tile's table records: all loaded at once (coordinates clamped
            // into the valid range, so every load is in bounds), either before
            // the multiply loop (PF: their latency hides behind it) or after
            using Rec = typename std::conditional<U16, StatU16, StatF32>::type;
            const Rec *table = static_cast<const Rec *>(p.stats);
            Rec rec[RX][RY];
            // records of displacements past the valid range read neighbouring
            // origins (or the table's slack past its end); they are masked out
            const Rec *rb = table + ((int64_t)(g.wz0 + dz) * p.oy + (g.wy0 + ty * RY)) * p.ox +
                            (g.wx0 + tx * RX);
            auto load_recs = [&]() {
#pragma unroll
                for (int j = 0; j < RY; ++j)
#pragma unroll
                    for (int i = 0; i < RX; ++i) rec[i][j] = rb[j * p.ox + i];
            };
            if constexpr (PF) load_recs();
            // cross term of each displacement of the tile, kept in the narrowest
            // exact type (converted to FP64 per displacement in the ranking)
            // FMA (B >= 5): FP32 sums of one block plane at a time, carried
            // across planes in FP64 for 12-bit data and in a second FP32 sum
            // for float data, so no running sum takes more than B^2 roundings
            // at its own size: where a window's local level lies far from the
            // block's (F - c large, varF small) a whole-block FP32 sum ranks
            // with about 4x the error
            constexpr bool FLUSH = ARITH == FMA && B >= 5;
            using XT = typename std::conditional<
                ARITH == DOT2, typename std::conditional<NG == 1, int, double>::type,
                typename std::conditional<FLUSH && U16, double, float>::type>::type;
            XT xacc[RX][RY];
            if constexpr (ARITH == DOT2) {
                dot2_cross<B, RX, RY>(tp, base, (zc0 + dzl) % R, R, plane, pitch, xacc);
            } else {
                float acc[RX][RY];
#pragma unroll
                for (int i = 0; i < RX; ++i)
#pragma unroll
                    for (int j = 0; j < RY; ++j) {
                        acc[i][j] = 0.0f;
                        xacc[i][j] = 0;
                    }
                for (int oz = 0; oz < B; ++oz) {
                    float tq[B][B];
                    const uint32_t *tpz = tp + oz * B * BP;
#pragma unroll
                    for (int oy = 0; oy < B; ++oy)
#pragma unroll
                        for (int ox = 0; ox < B; ++ox)
                            tq[oy][ox] = __uint_as_float(tpz[oy * BP + ox]);
                    const lds_word *wz = (const lds_word *)(base + oz * plane);
                    float fr[2][RX + B - 1];
#pragma unroll
                    for (int xw = 0; xw < RX + B - 1; ++xw) fr[0][xw] = __uint_as_float(wz[xw]);
#pragma unroll
                    for (int yw = 0; yw < RY + B - 1; ++yw) {
                        if (yw + 1 < RY + B - 1) {
#pragma unroll
                            for (int xw = 0; xw < RX + B - 1; ++xw)
                                fr[(yw + 1) & 1][xw] = __uint_as_float(wz[(yw + 1) * pitch + xw]);
                        }
                        const float *f = fr[yw & 1];
#pragma unroll
                        for (int j = 0; j < RY; ++j) {
                            const int oy = yw - j;
                            if (oy < 0 || oy >= B) continue;
#pragma unroll
                            for (int i = 0; i < RX; ++i)
#pragma unroll
                                for (int ox = 0; ox < B; ++ox)
                                    acc[i][j] = __builtin_fmaf(f[i + ox], tq[oy][ox], acc[i][j]);
                        }
                    }
                    if constexpr (FLUSH) {
#pragma unroll
                        for (int i = 0; i < RX; ++i)
#pragma unroll
                            for (int j = 0; j < RY; ++j) {
                                xacc[i][j] += (XT)acc[i][j];
                                acc[i][j] = 0.0f;
                            }
                    }
                }
                if constexpr (!FLUSH) {
#pragma unroll
                    for (int i = 0; i < RX; ++i)
#pragma unroll
                        for (int j = 0; j < RY; ++j) xacc[i][j] = acc[i][j];
                }
            }
            // ---- rank the tile's displacements: key = N*cov * rsqrt(N*varF);
            // invalid displacements are masked, no branch per displacement
            if constexpr (!PF) load_recs();
            const int irow = ((g.loz + dz + p.w) * side + (g.loy + ty * RY + p.w)) * side +
                             (g.lox + tx * RX + p.w);
            // sum of the staged F: DOT2 F-2048 (= the table's s), FMA F-c
            const double fshift = ARITH == DOT2 ? 0.0 : dN * (2048.0 - (double)c);
            const double tsum = ARITH == DOT2 ? (double)sT : sTc;  // sum of the staged T
            KeyT tk = -INFINITY;
            int ti = INT_MAX;
            if constexpr (SURF)
                rank_tile<U16, ARITH != DOT2, RX, RY, Rec, XT, KeyT, true>(
                    rec, xacc, dN, tsum, fshift, c, g.dx - tx * RX, g.dy - ty * RY, irow, side, tk,
                    ti, p.surface + blk * side * side * side, 1.0 / sqrt(vtn));
            else
                rank_tile<U16, ARITH != DOT2>(rec, xacc, dN, tsum, fshift, c, g.dx - tx * RX,
                                              g.dy - ty * RY, irow, side, tk, ti);
            better(bk, bi, tk, ti);
        }
    }
    wg_argmax<NT>(bk, bi, s_key, s_idx);
    if (bi == INT_MAX) {  // every key NaN (non-finite input): report, never index
        if (tid == 0) write_result(p, blk, 0, 0, 0, NAN);
        return;
    }

    // ---- exact NCC at the winning displacement, from the volumes
    const int ddx = bi % side - p.w, ddy = (bi / side) % side - p.w, ddz = bi / (side * side) - p.w;
    auto fval = [&](int o) {
        const int oz = o / (B * B), oy = (o / B) % B, ox = o % B;
        return flt[((int64_t)(g.cz - H + ddz + oz) * p.ny + (g.cy - H + ddy + oy)) * p.nx +
                   (g.cx - H + ddx + ox)];
    };
    if constexpr (U16) {
        // the exact sums of T and T^2 are already known (st); F and TF here.
        // Sums of shifted values (F - 2048, T - 2048) give the same covariance
        // and spreads as the raw values, and st is shift-free.
        long long sums[3] = {0, 0, 0};  // F, F^2, TF
        long long tS = st[0];             // sum of T in the same offset frame
        if constexpr (ARITH == DOT2) {
            // pair words of the winning window: from the LDS ring when its planes
            // are still staged, else from the plane-pair volume; the block's own
            // words are in the T table.  Values are int16, offset by -2048.
            tS = st[0] - 2048ll * N;
            const int zr = ddz - g.loz, yr = ddy - g.loy, xr = ddx - g.lox;
            const bool in_lds = zr >= staged - R;
            for (int i = tid; i < P * B * B; i += NT) {
                const int m = i / (B * B), oy = (i / B) % B, ox = i % B;
                const uint32_t tw = tp[(m * B + oy) * BP + ox];
                const int q = zr + 2 * m;
                const uint32_t fw =
                    in_lds ? win[(q % R) * plane + (yr + oy) * pitch + (xr + ox)]
                           : p.pv[((int64_t)(g.wz0 + q) * p.ny + (g.wy0 + yr + oy)) * p.nx +
                                  (g.wx0 + xr + ox)];
                const long long tlo = (short)(tw & 0xffff), thi = (short)(tw >> 16);
                const long long flo = (short)(fw & 0xffff);
                const long long fhi = 2 * m + 1 < B ? (long long)(short)(fw >> 16) : 0;
                sums[0] += flo + fhi;
                sums[1] += flo * flo + fhi * fhi;
                sums[2] += tlo * flo + thi * fhi;
            }
        } else {
            for (int o = tid; o < N; o += NT) {
                const long long tv = tval(o), fv = fval(o);
                sums[0] += fv;
                sums[1] += fv * fv;
                sums[2] += tv * fv;
            }
        }
        wg_sum<NT, long long, 3>(sums, s_red);
        if (tid == 0) {
            const long long vt = (long long)N * st[1] - st[0] * st[0];
            const long long vf = (long long)N * sums[1] - sums[0] * sums[0];
            const long long cv = (long long)N * sums[2] - tS * sums[0];
            const double v = (vt > 0 && vf > 0) ? (double)cv / sqrt((double)vt * (double)vf) : 0.0;
            write_result(p, blk, ddx, ddy, ddz, (float)v);
        }
    } else {
        double m2[1] = {0.0};
        for (int o = tid; o < N; o += NT) m2[0] += (double)fval(o);
        wg_sum<NT, double, 1>(m2, s_redd);
        const double fmean = m2[0] / (double)N;
        double q[3] = {0.0, 0.0, 0.0};  // A, B, X of the two-pass Pearson form
        for (int o = tid; o < N; o += NT) {
            const double a = (double)tval(o) - tmean, b = (double)fval(o) - fmean;
            q[0] += a * a;
            q[1] += b * b;
            q[2] += a * b;
        }
        wg_sum<NT, double, 3>(q, s_redd);
        if (tid == 0) {
            const double ab = q[0] * q[1];
            const double v = ab > 0.0 ? q[2] / sqrt(ab) : 0.0;
            write_result(p, blk, ddx, ddy, ddz, (float)v);
        }
    }
}


template <typename Vox, int ARITH, int B, int RX, int RY, int NT, bool PF>
__global__ __launch_bounds__(NT) void k_match(Params p) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ Small sm;
    match_one<Vox, ARITH, B, RX, RY, NT, PF>(p, p.first + xcd_block(blockIdx.x, gridDim.x), lds,
                                             sm);
}

// The same search also writing the ranking NCC of every valid displacement
// to p.surface (a diagnostic of the ranking arithmetic's error).
template <typename Vox, int ARITH, int B, int RX, int RY, int NT, bool PF>
__global__ __launch_bounds__(NT) void k_match_surf(Params p) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ Small sm;
    match_one<Vox, ARITH, B, RX, RY, NT, PF, true>(
        p, p.first + xcd_block(blockIdx.x, gridDim.x), lds, sm);
}


// ------------------------------------------------------------ batched search
//
// Many parameter sets (block size, window, selection) over one volume pair in
// one persistent launch: workgroups stride a list of work items (the blocks
// of every set, the most expensive sets first) and switch to the compiled
// shape the set was planned with.  The shapes all run 256 threads.
#define BATCH_F32(X) X(0, 5, 4, 4, 0) X(1, 7, 4, 4, 0) X(2, 9, 4, 4, 0) X(3, 5, 3, 3, 0) \
    X(4, 7, 3, 3, 0) X(5, 9, 3, 3, 0)
#define BATCH_U16(X) X(0, 5, 4, 4, 0) X(1, 7, 3, 7, 1) X(2, 7, 4, 4, 0) X(3, 9, 4, 4, 0) \
    X(4, 9, 5, 5, 0) X(5, 5, 3, 3, 0)

template <typename Vox>
__global__ __launch_bounds__(256) void k_match_batch(const BatchSet *__restrict__ sets, int nsets,
                                                     int64_t nitems) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ Small sm;
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        int s = 0;
        while (s + 1 < nsets && sets[s + 1].first_item <= it) ++s;
        const BatchSet &S = sets[s];
        Params p;
        p.ref = S.a.ref;
        p.flt = S.a.flt;
        p.nx = S.a.nx;
        p.ny = S.a.ny;
        p.nz = S.a.nz;
        p.centers = S.a.centers;
        p.n = S.a.n;
        p.first = 0;
        p.w = S.a.window;
        p.cz = S.cz;
        p.stats = S.a.stats;
        p.pv = S.a.pairs;
        p.ox = S.a.ox;
        p.oy = S.a.oy;
        p.disp = S.a.disp;
        p.ncc = S.a.ncc;
        p.conf = S.a.conf;
        p.surface = nullptr;
        const int64_t blk = it - S.first_item;
        if constexpr (sizeof(Vox) == 4) {
#define CASE_F32(ID, B, RX, RY, PF) \
    case ID: match_one<float, FMA, B, RX, RY, 256, PF>(p, blk, lds, sm); break;
            switch (S.variant) { BATCH_F32(CASE_F32) }
#undef CASE_F32
        } else {
#define CASE_U16(ID, B, RX, RY, PF) \
    case ID: match_one<uint16_t, DOT2, B, RX, RY, 256, PF>(p, blk, lds, sm); break;
            switch (S.variant) { BATCH_U16(CASE_U16) }
#undef CASE_U16
        }
        __syncthreads();  // the next item restages LDS
    }
}

// ------------------------------------------------------------ dispatch

typedef void (*kernel_t)(Params);

struct Variant {
    nrr_dtype dtype;
    int arith, b, rx, ry, nt, pf;
    kernel_t fn;
};

#define V16D(B, RX, RY, NT, PF) \
    {NRR_U16, DOT2, B, RX, RY, NT, PF, k_match<uint16_t, DOT2, B, RX, RY, NT, PF>}
#define V16F(B, RX, RY, NT, PF) \
    {NRR_U16, FMA, B, RX, RY, NT, PF, k_match<uint16_t, FMA, B, RX, RY, NT, PF>}
#define V32F(B, RX, RY, NT, PF) \
    {NRR_F32, FMA, B, RX, RY, NT, PF, k_match<float, FMA, B, RX, RY, NT, PF>}

// Order matters only between equal-cost shapes (the first wins).  The cost
// model counts wavefront rounds, not occupancy, so shapes that lose on
// occupancy are left out rather than modelled: FMA 3x7 tiles at 448 threads
// (b = 7) ran 1.7x slower than at 256 on the 256x256x124 volume (W = 10) and
// 2.5x slower at W = 5.
const Variant kVariants[] = {
    V16D(3, 4, 4, 256, 0),  V16D(5, 4, 4, 256, 0),  V16D(5, 3, 7, 448, 0),
    V16D(7, 3, 7, 256, 1),  V16D(7, 3, 7, 256, 0),  V16D(7, 4, 4, 256, 0),
    V16D(7, 3, 5, 256, 0),  V16D(7, 5, 5, 256, 0),  V16D(9, 4, 4, 256, 0),
    V16D(9, 5, 5, 256, 0),  V16D(11, 3, 3, 256, 0), V16D(13, 3, 3, 256, 0),
    V16D(15, 2, 2, 256, 0), V16F(3, 4, 4, 256, 0),  V16F(5, 4, 4, 256, 0),
    V16F(5, 3, 7, 448, 0),  V16F(7, 4, 4, 256, 0),  V16F(7, 5, 5, 256, 0),
    V16F(7, 3, 7, 256, 0),
    V16F(9, 4, 4, 256, 0),  V16F(9, 5, 5, 256, 0),  V16F(11, 3, 3, 256, 0),
    V16F(13, 3, 3, 256, 0), V16F(15, 2, 2, 256, 0), V32F(3, 4, 4, 256, 0),
    V32F(5, 4, 4, 256, 0),  V32F(7, 4, 4, 256, 0),  V32F(7, 5, 5, 256, 0),
    V32F(7, 3, 7, 256, 0),  V32F(9, 5, 5, 256, 0),
    V32F(9, 4, 4, 256, 0),  V32F(11, 3, 3, 256, 0), V32F(13, 3, 3, 256, 0),
    V32F(15, 2, 2, 256, 0),
};

struct Plan {
    const Variant *v;
    int cz;
    size_t lds;
};

size_t t_table_bytes(const Variant &v) {
    const int bp = (v.b + 3) & ~3;
    const int planes = v.arith == DOT2 ? (v.b + 1) / 2 : v.b;
    return (size_t)planes * v.b * bp * 4;
}

size_t window_plane_bytes(const Variant &v, int w) {
    const int d = 2 * w + 1;
    const int px = (d + v.rx - 1) / v.rx * v.rx + v.b - 1;
    const int py = (d + v.ry - 1) / v.ry * v.ry + v.b - 1;
    if (v.arith == DOT2 || v.dtype == NRR_F32) {  // as the kernel's chunk-staged plane
        const int pl = (px + CW - 1) / CW * CW * py;
        return (size_t)(v.dtype == NRR_F32 ? pl + 1 : pl + (((pl / CW) & 1) ? 0 : CW)) * 4;
    }
    return ((size_t)px * py + ZPAD) * 4;
}

// Wavefront-rounds of one block's search with z-chunks of cz displacement
// planes (the last chunk takes the rest), plus half a round per extra chunk
// for its staging and barriers.  Idle wavefronts of a round skip the tiles.
double chunk_rounds(const Variant &v, int d, int cz) {
    const int per_dz = ((d + v.rx - 1) / v.rx) * ((d + v.ry - 1) / v.ry);
    double r = 0.0;
    for (int z0 = 0; z0 < d; z0 += cz) {
        const int tiles = per_dz * std::min(cz, d - z0);
        r += std::ceil(tiles / 64.0) + (z0 > 0 ? 0.5 : 0.0);
    }
    return r;
}

// z-chunk and LDS size: the whole window if it fits in `target` bytes (two
// workgroups per CU), else the largest balanced chunk of displacement planes
// that still fits in `target`, else the largest that fits in `limit`.
// (Balanced chunks keep the workgroup's LDS small: on the 256x256x124 search,
// 11 + 10 planes with three workgroups per CU beat 12 + 9 with two, although
// the latter packs the tiles into fewer wavefront-rounds.)
bool plan_variant(const Variant &v, int w, size_t limit, size_t target, Plan *out) {
    const int d = 2 * w + 1;
    const size_t fixed = t_table_bytes(v) + 2048;  // + static shared and slack
    const size_t pb = window_plane_bytes(v, w);
    if (fixed + (size_t)v.b * pb > limit) return false;
    int cz = d;
    if (fixed + (size_t)(cz + v.b - 1) * pb > target) {
        const size_t cap = fixed + (size_t)v.b * pb <= target ? target : limit;
        const long fit = (long)((cap - fixed) / pb) - (v.b - 1);
        cz = (int)(fit < d ? fit : d);
        const int nch = (d + cz - 1) / cz;
        cz = (d + nch - 1) / nch;
    }
    out->v = &v;
    out->cz = cz;
    out->lds = t_table_bytes(v) + (size_t)(cz + v.b - 1) * pb;
    return true;
}

// Cost model: padded displacement work over the workgroup's thread rounds.
double plan_cost(const Plan &pl, int w) {
    const Variant &v = *pl.v;
    const int d = 2 * w + 1;
    const double rounds = chunk_rounds(v, d, pl.cz) * 64.0 / v.nt;
    const double planes = v.arith == DOT2 ? (v.b + 1) / 2 : v.b;
    // instructions per tile: multiply-adds (dot2 issues at half the FMA rate)
    const double per = planes * v.rx * v.ry * v.b * v.b * (v.arith == DOT2 ? 2.0 : 1.0) +
                       planes * (v.rx + v.b - 1) * (v.ry + v.b - 1);
    return rounds * v.nt * per;
}

int arith_preference() {
    const char *e = getenv("NRR_ARITH");
    if (!e) return -1;
    if (!strcmp(e, "dot2")) return DOT2;
    if (!strcmp(e, "fma")) return FMA;
    if (!strcmp(e, "mfma")) return kArithMfma;
    return -1;
}

// Measurement overrides: NRR_TILE="rx,ry,nt[,pf]" restricts the shape and
// NRR_CZ=n caps the z-chunk (unknown or infeasible values are ignored).
bool shape_from_env(TileShape *sh) {
    *sh = TileShape{-1, 0, 0, 0, -1, 0};
    if (const char *e = getenv("NRR_TILE")) sscanf(e, "%d,%d,%d,%d", &sh->rx, &sh->ry, &sh->nt, &sh->pf);
    if (const char *e = getenv("NRR_CZ")) sh->cz = atoi(e);
    return sh->rx > 0 || sh->cz > 0;
}

// Shapes chosen by the tuner, per (dtype, block, window), for the process.
struct TunedEntry {
    nrr_dtype dtype;
    int b, w;
    TileShape sh;
};
std::mutex g_tuned_mu;
std::vector<TunedEntry> g_tuned;

bool shape_matches(const Variant &v, const TileShape &sh) {
    if (sh.arith >= 0 && v.arith != sh.arith) return false;
    if (sh.rx > 0 && (v.rx != sh.rx || v.ry != sh.ry || v.nt != sh.nt)) return false;
    if (sh.pf >= 0 && v.pf != sh.pf) return false;
    return true;
}

// Best plan by the cost model among compiled shapes of (dtype, b); `force`
// (when given and feasible) restricts the shape and caps the z-chunk.
bool choose_with(nrr_dtype dtype, int b, int w, size_t limit, int arith, const TileShape *force,
                 Plan *best) {
    for (int pass = force ? 0 : 1; pass < 2; ++pass) {
        bool found = false;
        double bc = 0.0;
        for (const Variant &v : kVariants) {
            if (v.dtype != dtype || v.b != b) continue;
            if (arith >= 0 && v.arith != arith) continue;
            if (pass == 0 && !shape_matches(v, *force)) continue;
            Plan pl;
            if (!plan_variant(v, w, limit, limit / 2, &pl)) continue;
            if (pass == 0 && force->cz > 0 && force->cz < pl.cz) {  // a smaller chunk, as given
                pl.cz = force->cz;
                pl.lds = t_table_bytes(v) + (size_t)(pl.cz + v.b - 1) * window_plane_bytes(v, w);
            }
            const double c = plan_cost(pl, w);
            if (!found || c < bc) {
                *best = pl;
                bc = c;
                found = true;
            }
        }
        if (found) return true;
    }
    return false;
}

// Shape priority: an explicit one (the tuner's trials), the environment
// overrides, the tuned table, then the cost model.  12-bit volumes use the
// exact dot2 form when a shape has it (it measures faster than FMA on every
// shape tried); NRR_ARITH=dot2|fma restricts them to one form.
bool choose(nrr_dtype dtype, int b, int w, size_t limit, const TileShape *force, Plan *best) {
    TileShape sh;
    if (!force && shape_from_env(&sh)) force = &sh;
    if (!force && tuned_shape(dtype, b, w, &sh)) force = &sh;
    int pref = arith_preference();
    if (pref == kArithMfma) pref = -1;  // the matrix-core form does not serve this case
    if (pref < 0 && dtype == NRR_U16 && !(force && force->arith >= 0)) pref = DOT2;
    if (pref >= 0 && choose_with(dtype, b, w, limit, pref, force, best)) return true;
    return choose_with(dtype, b, w, limit, -1, force, best);
}

}  // namespace

size_t device_lds_limit() {
    static int cached_dev = -1;
    static size_t cached = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (dev != cached_dev) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
            v <= 0)
            v = 65536;
        cached = (size_t)v;
        cached_dev = dev;
    }
    return cached;
}

const char *match_unsupported_reason(nrr_dtype dtype, int32_t block, int32_t window) {
    if (block > MAX_B) return "block edge above 15 is not built";
    if (window > 64) return "window above 64 is not supported";
    Plan pl;
    if (!choose(dtype, block, window, device_lds_limit(), nullptr, &pl))
        return "one window plane does not fit in LDS for this block size";
    return nullptr;
}


namespace {
#define ROW_F32(ID, B, RX, RY, PF) {NRR_F32, FMA, B, RX, RY, 256, PF, nullptr},
#define ROW_U16(ID, B, RX, RY, PF) {NRR_U16, DOT2, B, RX, RY, 256, PF, nullptr},
const Variant kBatchF32[] = {BATCH_F32(ROW_F32)};
const Variant kBatchU16[] = {BATCH_U16(ROW_U16)};
#undef ROW_F32
#undef ROW_U16
}  // namespace

bool plan_batch_set(nrr_dtype dtype, int32_t block, int32_t window, int32_t *variant,
                    int32_t *cz, size_t *lds, double *cost_per_block) {
    const Variant *tab = dtype == NRR_F32 ? kBatchF32 : kBatchU16;
    const int nv = dtype == NRR_F32 ? (int)(sizeof(kBatchF32) / sizeof(Variant))
                                    : (int)(sizeof(kBatchU16) / sizeof(Variant));
    const size_t limit = device_lds_limit();
    // a tuned shape for this (dtype, block, window) wins when it is compiled here
    TileShape ts;
    const bool tuned = tuned_shape(dtype, block, window, &ts);
    bool found = false;
    double best = 0.0;
    for (int pass = 0; pass < 2 && !found; ++pass)
        for (int i = 0; i < nv; ++i) {
            const Variant &v = tab[i];
            if (v.b != block) continue;
            if (pass == 0 && (!tuned || !shape_matches(v, ts))) continue;
            Plan pl;
            if (!plan_variant(v, window, limit, limit / 2, &pl)) continue;
            if (pass == 0 && ts.cz > 0 && ts.cz < pl.cz) {
                const int d = 2 * window + 1, nch = (d + ts.cz - 1) / ts.cz;
                pl.cz = (d + nch - 1) / nch;
                pl.lds = t_table_bytes(v) + (size_t)(pl.cz + v.b - 1) * window_plane_bytes(v, window);
            }
            const double c = plan_cost(pl, window);
            if (!found || c < best) {
                best = c;
                *variant = i;
                *cz = pl.cz;
                *lds = pl.lds;
                *cost_per_block = c;
                found = true;
            }
        }
    return found;
}

hipError_t launch_match_batch(nrr_dtype dtype, const BatchSet *sets, int32_t nsets,
                              int64_t nitems, size_t lds, hipStream_t stream) {
    if (nitems <= 0) return hipSuccess;
    const void *fn = dtype == NRR_F32 ? reinterpret_cast<const void *>(k_match_batch<float>)
                                      : reinterpret_cast<const void *>(k_match_batch<uint16_t>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int per_cu = 0, dev = 0, cus = 0;
    e = dtype == NRR_F32
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_match_batch<float>, 256, lds)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_match_batch<uint16_t>, 256,
                                                           lds);
    if (e != hipSuccess) return e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    const int64_t slots = (int64_t)(per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
    const unsigned grid = (unsigned)(nitems < slots ? nitems : slots);
    if (dtype == NRR_F32)
        hipLaunchKernelGGL(k_match_batch<float>, dim3(grid), dim3(256), lds, stream, sets, nsets,
                           nitems);
    else
        hipLaunchKernelGGL(k_match_batch<uint16_t>, dim3(grid), dim3(256), lds, stream, sets,
                           nsets, nitems);
    return hipGetLastError();
}

bool tuned_shape(nrr_dtype dtype, int32_t block, int32_t window, TileShape *sh) {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    for (const TunedEntry &t : g_tuned)
        if (t.dtype == dtype && t.b == block && t.w == window) {
            *sh = t.sh;
            return true;
        }
    return false;
}

void set_tuned_shape(nrr_dtype dtype, int32_t block, int32_t window, const TileShape &sh) {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    for (TunedEntry &t : g_tuned)
        if (t.dtype == dtype && t.b == block && t.w == window) {
            t.sh = sh;
            return;
        }
    g_tuned.push_back(TunedEntry{dtype, block, window, sh});
}

void clear_tuned_shapes() {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    g_tuned.clear();
}

// The matrix-core form serves a launch when it is asked for (shape, then the
// NRR_ARITH override, then the tuned table) or, by default, whenever it can:
// 12-bit data, block edges 3-9, the whole window in LDS.
static bool wants_mfma(nrr_dtype dtype, int32_t block, int32_t window, const TileShape *shape) {
    if (!mfma_supported(dtype, block, window)) return false;
    if (shape) return shape->arith == kArithMfma;
    TileShape sh;
    if (shape_from_env(&sh)) return false;
    const int pref = arith_preference();
    if (pref >= 0) return pref == kArithMfma;
    if (tuned_shape(dtype, block, window, &sh)) return sh.arith == kArithMfma;
    return true;
}

int match_shapes(nrr_dtype dtype, int32_t block, int32_t window, TileShape *out, int cap) {
    const size_t limit = device_lds_limit();
    const int d = 2 * window + 1;
    int n = 0;
    if (mfma_supported(dtype, block, window)) {
        if (n < cap) out[n] = TileShape{kArithMfma, 0, 0, 256, -1, 0};
        ++n;
    }
    for (const Variant &v : kVariants) {
        if (v.dtype != dtype || v.b != block) continue;
        Plan pl;
        if (!plan_variant(v, window, limit, limit / 2, &pl)) continue;
        // the planned z-chunk and the next two finer splits of the window
        int last = 0;
        for (int nch = (d + pl.cz - 1) / pl.cz; nch <= (d + pl.cz - 1) / pl.cz + 2; ++nch) {
            const int cz = (d + nch - 1) / nch;
            if (cz == last || cz < 1) continue;
            last = cz;
            if (n < cap) out[n] = TileShape{v.arith, v.rx, v.ry, v.nt, v.pf, cz};
            ++n;
        }
    }
    return n < cap ? n : cap;
}

bool match_plan(nrr_dtype dtype, const MatchArgs &a, TileShape *out) {
    if (mfma_fits(a) && wants_mfma(dtype, a.block, a.window, nullptr)) {
        *out = TileShape{kArithMfma, 0, 0, 256, -1, 0};
        return true;
    }
    Plan pl;
    if (!choose(dtype, a.block, a.window, device_lds_limit(), nullptr, &pl)) return false;
    *out = TileShape{pl.v->arith, pl.v->rx, pl.v->ry, pl.v->nt, pl.v->pf, pl.cz};
    return true;
}

bool shape_known(nrr_dtype dtype, int32_t block, int32_t window, const TileShape &sh) {
    if (sh.arith == kArithMfma) return mfma_supported(dtype, block, window);
    const size_t limit = device_lds_limit();
    for (const Variant &v : kVariants)
        if (v.dtype == dtype && v.b == block && v.arith == sh.arith && v.rx == sh.rx &&
            v.ry == sh.ry && v.nt == sh.nt && v.pf == sh.pf) {
            Plan pl;
            if (plan_variant(v, window, limit, limit / 2, &pl)) return true;
        }
    const Variant *tab = dtype == NRR_F32 ? kBatchF32 : kBatchU16;
    const int nv = dtype == NRR_F32 ? (int)(sizeof(kBatchF32) / sizeof(Variant))
                                    : (int)(sizeof(kBatchU16) / sizeof(Variant));
    for (int i = 0; i < nv; ++i)
        if (tab[i].b == block && tab[i].arith == sh.arith && tab[i].rx == sh.rx &&
            tab[i].ry == sh.ry && tab[i].nt == sh.nt && tab[i].pf == sh.pf)
            return true;
    return false;
}

bool batch_variant_shape(nrr_dtype dtype, int32_t variant, int32_t cz, TileShape *out) {
    const Variant *tab = dtype == NRR_F32 ? kBatchF32 : kBatchU16;
    const int nv = dtype == NRR_F32 ? (int)(sizeof(kBatchF32) / sizeof(Variant))
                                    : (int)(sizeof(kBatchU16) / sizeof(Variant));
    if (variant < 0 || variant >= nv) return false;
    const Variant &v = tab[variant];
    *out = TileShape{v.arith, v.rx, v.ry, v.nt, v.pf, cz};
    return true;
}

hipError_t launch_match(nrr_dtype dtype, const MatchArgs &a, hipStream_t stream,
                        const TileShape *shape) {
    if (mfma_fits(a) && wants_mfma(dtype, a.block, a.window, shape))
        return launch_match_mfma(a, stream);
    Plan pl;
    if (!choose(dtype, a.block, a.window, device_lds_limit(), shape, &pl))
        return hipErrorInvalidValue;
    const Variant *v = pl.v;
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(v->fn),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds) != hipSuccess)
        return hipGetLastError();
    Params p;
    p.ref = a.ref;
    p.flt = a.flt;
    p.nx = a.nx;
    p.ny = a.ny;
    p.nz = a.nz;
    p.centers = a.centers;
    p.n = a.n;
    p.w = a.window;
    p.cz = pl.cz;
    p.stats = a.stats;
    p.pv = a.pairs;
    p.ox = a.ox;
    p.oy = a.oy;
    p.disp = a.disp;
    p.ncc = a.ncc;
    p.conf = a.conf;
    p.surface = nullptr;
    const int64_t chunk = 1ll << 30;
    for (int64_t first = 0; first < a.n; first += chunk) {
        p.first = first;
        const int64_t cnt = a.n - first < chunk ? a.n - first : chunk;
        hipLaunchKernelGGL(v->fn, dim3((unsigned)cnt), dim3(v->nt), pl.lds, stream, p);
    }
    return hipGetLastError();
}

namespace {
__global__ void k_fill(float *p, int64_t n, float v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
}  // namespace

hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

namespace {
// Surface-writing instantiations: one shape per (dtype, form, block edge).
#define S16D(B, RX, RY, NT, PF) \
    {NRR_U16, DOT2, B, RX, RY, NT, PF, k_match_surf<uint16_t, DOT2, B, RX, RY, NT, PF>}
#define S16F(B, RX, RY, NT, PF) \
    {NRR_U16, FMA, B, RX, RY, NT, PF, k_match_surf<uint16_t, FMA, B, RX, RY, NT, PF>}
#define S32F(B, RX, RY, NT, PF) \
    {NRR_F32, FMA, B, RX, RY, NT, PF, k_match_surf<float, FMA, B, RX, RY, NT, PF>}
const Variant kSurfVariants[] = {
    S16D(3, 4, 4, 256, 0), S16D(5, 4, 4, 256, 0), S16D(7, 3, 7, 256, 1), S16D(9, 5, 5, 256, 0),
    S16D(11, 3, 3, 256, 0), S16D(13, 3, 3, 256, 0), S16D(15, 2, 2, 256, 0),
    S16F(7, 4, 4, 256, 0),  S32F(3, 4, 4, 256, 0),  S32F(5, 4, 4, 256, 0),
    S32F(7, 4, 4, 256, 0),  S32F(9, 5, 5, 256, 0),
};
#undef S16D
#undef S16F
#undef S32F
}  // namespace

hipError_t launch_match_surface(nrr_dtype dtype, int32_t arith, const MatchArgs &a,
                                float *surface, hipStream_t stream) {
    if (arith == kArithMfma) {
        if (!mfma_supported(dtype, a.block, a.window) || !mfma_fits(a))
            return hipErrorNotSupported;
        return launch_match_mfma(a, stream, surface);
    }
    const size_t limit = device_lds_limit();
    for (const Variant &v : kSurfVariants) {
        if (v.dtype != dtype || v.arith != arith || v.b != a.block) continue;
        Plan pl;
        if (!plan_variant(v, a.window, limit, limit / 2, &pl)) continue;
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(v.fn),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)pl.lds) != hipSuccess)
            return hipGetLastError();
        Params p;
        p.ref = a.ref;
        p.flt = a.flt;
        p.nx = a.nx;
        p.ny = a.ny;
        p.nz = a.nz;
        p.centers = a.centers;
        p.n = a.n;
        p.w = a.window;
        p.cz = pl.cz;
        p.stats = a.stats;
        p.pv = a.pairs;
        p.ox = a.ox;
        p.oy = a.oy;
        p.disp = a.disp;
        p.ncc = a.ncc;
        p.conf = a.conf;
        p.surface = surface;
        const int64_t chunk = 1ll << 30;
        for (int64_t first = 0; first < a.n; first += chunk) {
            p.first = first;
            const int64_t cnt = a.n - first < chunk ? a.n - first : chunk;
            hipLaunchKernelGGL(v.fn, dim3((unsigned)cnt), dim3(v.nt), pl.lds, stream, p);
        }
        return hipGetLastError();
    }
    return hipErrorNotSupported;
}

}  // namespace nrr
