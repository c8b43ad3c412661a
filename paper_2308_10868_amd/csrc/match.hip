// Exhaustive NCC block matching on gfx950.
//
// The paper's GPU algorithm (GPU section) maps one image block to one thread
// block and spreads the loop over the candidate displacements of the search
// window across the threads, then takes the maximum similarity and its
// displacement.  This kernel keeps that outer mapping (one workgroup per
// selected block) and re-designs the inner part for CDNA:
//
//  * the block's whole search window of `flt` is staged once in LDS (every
//    voxel is then reused by all displacements that touch it), and the
//    pre-operative block T is staged beside it;
//  * each thread owns an RX x RY tile of (dx, dy) displacements at one dz and
//    keeps RX*RY accumulators in registers; a window row loaded from LDS is
//    reused by every (tile displacement, block column) pair that reads it;
//  * 12-bit data: the cross term sum T'F' (T' = T-2048, F' = F-2048) is
//    accumulated exactly in int32 with v_dot2_i32_i16, two voxels (planes z
//    and z+1) per instruction; the block's planes are grouped so that no
//    int32 partial sum can overflow (|T'|,|F'| <= 2048);
//  * float data: the cross term sum T^(F - c) with T^ = T - mean(T) and
//    c = mean(T) is accumulated in FP32 FMA;
//  * the window statistics (sum F and 1/sqrt of the spread) come from a
//    per-voxel table computed once per call (stats.hip), so the epilogue per
//    displacement is a handful of operations;
//  * displacements are ranked by key = cov * rsqrt(varF), which is
//    proportional to the NCC (the block's own spread is a constant factor);
//    the argmax keeps the smallest shift index among equal keys and is
//    reduced across the workgroup with wavefront shuffles;
//  * the NCC reported for the winning displacement is recomputed exactly
//    (integer sums for 12-bit data, two-pass FP64 for float data) from the
//    volumes, so it does not inherit the ranking arithmetic's rounding.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "nrr_internal.h"

namespace nrr {
namespace {

typedef short short2v __attribute__((ext_vector_type(2)));

constexpr int NT = 256;     // threads per workgroup (4 wavefronts)
constexpr int MAX_B = 15;   // largest block edge served

struct Params {
    const void *ref;
    const void *flt;
    int nx, ny, nz;
    const int32_t *centers;
    int64_t n;
    int64_t first;  // first block of this launch
    int w;
    const void *stat_s;
    const void *stat_r;
    int ox, oy;
    int32_t *disp;
    float *ncc;
    float *conf;
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
template <typename K>
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

template <typename T, int NV>
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

// Stage a box of a volume into LDS rows: row r = z*py + y (z < pz, y < py) of
// `pitch` elements (pitch a multiple of 4).  Element (z, y, x) becomes
// conv(v) for v = src at (z0+z, y0+y, x0+x) when z < ez, y < ey and x < ex,
// and 0 elsewhere (tile padding is never read as a real voxel).  Each lane
// moves chunks of 4 consecutive x; UNR chunks per lane are loaded before any
// is written so several global loads are in flight, and the chunk coordinates
// advance incrementally (no integer division in the loop).
template <typename Src, typename Dst, typename Conv>
__device__ inline void stage_box(const Src *__restrict__ src, int nx, int ny, int x0, int y0,
                                 int z0, int ex, int ey, int ez, Dst *__restrict__ dst, int pitch,
                                 int py, int pz, Conv conv) {
    constexpr int UNR = 8;
    const int cpr = pitch >> 2;
    const int total = pz * py * cpr;
    const int drow = NT / cpr, dxc = NT - drow * cpr;
    int row = (int)threadIdx.x / cpr;
    int xc = (int)threadIdx.x - row * cpr;
    int z = row / py, y = row - z * py;
    for (int c0 = 0; c0 < total; c0 += NT * UNR) {
        Src v[UNR][4];
        int off[UNR], xs[UNR];
        bool rin[UNR], live[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            live[u] = c0 + u * NT + (int)threadIdx.x < total;
            xs[u] = 4 * xc;
            off[u] = (z * py + y) * pitch + 4 * xc;
            rin[u] = live[u] && z < ez && y < ey;
            const Src *s = src + ((int64_t)(z0 + z) * ny + (y0 + y)) * nx + (x0 + 4 * xc);
#pragma unroll
            for (int e = 0; e < 4; ++e) v[u][e] = (rin[u] && 4 * xc + e < ex) ? s[e] : Src(0);
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
            Dst o[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = (rin[u] && xs[u] + e < ex) ? conv(v[u][e]) : Dst(0);
            if constexpr (sizeof(Dst) == 2) {
                uint2 w;
                w.x = (uint32_t)(uint16_t)o[0] | ((uint32_t)(uint16_t)o[1] << 16);
                w.y = (uint32_t)(uint16_t)o[2] | ((uint32_t)(uint16_t)o[3] << 16);
                *reinterpret_cast<uint2 *>(dst + off[u]) = w;
            } else {
                *reinterpret_cast<float4 *>(dst + off[u]) = make_float4(o[0], o[1], o[2], o[3]);
            }
        }
    }
}

// --------------------------------------------------------- 12-bit volumes

// Shape of the staged window for a block: x/y padded to whole tiles, one
// extra z plane for the zero half of the last plane pair when b is odd.
template <int B, int RX, int RY>
struct U16Shape {
    static constexpr int P = (B + 1) / 2;       // plane pairs of the block
    static constexpr int BP = (B + 3) & ~3;     // padded row of T pairs (dwords)
    static constexpr int TP_DWORDS = P * B * BP;
    // exact int32 groups: a plane contributes at most B*B*2048*2048
    static constexpr long long PLANE_MAX = (long long)B * B * 2048 * 2048;
    static constexpr int GPAIRS = (int)(2147483647LL / PLANE_MAX) / 2;  // pairs per group
    static constexpr int NG = (P + GPAIRS - 1) / GPAIRS;
    static_assert(GPAIRS >= 1, "block edge too large for exact int32 groups");
};

template <int B, int RX, int RY>
__global__ __launch_bounds__(NT) void k_match_u16(Params p) {
    using S = U16Shape<B, RX, RY>;
    constexpr int H = (B - 1) / 2, P = S::P, BP = S::BP, N = B * B * B;
    constexpr int GP = S::GPAIRS, NG = S::NG;
    extern __shared__ __align__(16) unsigned char lds[];
    int32_t *tp = reinterpret_cast<int32_t *>(lds);                 // [P][B][BP] pairs
    int16_t *win = reinterpret_cast<int16_t *>(lds + S::TP_DWORDS * 4);  // [PZ][PY][PX]
    __shared__ float s_key[NT / 64];
    __shared__ int s_idx[NT / 64];
    __shared__ long long s_red[(NT / 64) * 5];

    const int64_t blk = p.first + xcd_block(blockIdx.x, gridDim.x);
    const Geom g = make_geom(p, blk, H);
    const int tid = threadIdx.x;
    if (!g.inside) {
        if (tid == 0) write_result(p, blk, 0, 0, 0, NAN);
        return;
    }
    const uint16_t *ref = static_cast<const uint16_t *>(p.ref);
    const uint16_t *flt = static_cast<const uint16_t *>(p.flt);
    const int txn = (g.dx + RX - 1) / RX, tyn = (g.dy + RY - 1) / RY;
    // row pitch rounded to 4 elements (8-byte LDS writes)
    const int PX = (txn * RX + B - 1 + 3) & ~3, PY = tyn * RY + B - 1, PZ = g.dz + B;
    const int ex = g.dx + B - 1, ey = g.dy + B - 1, ez = g.dz + B - 1;  // real window extent

    // ---- stage T' = T - 2048 as (plane 2m, plane 2m+1) pairs, zero padded
    for (int i = tid; i < S::TP_DWORDS; i += NT) tp[i] = 0;
    __syncthreads();
    int16_t *tp16 = reinterpret_cast<int16_t *>(tp);
    long long red[2] = {0, 0};  // sum T', sum T'^2
    for (int o = tid; o < N; o += NT) {
        const int oz = o / (B * B), oy = (o / B) % B, ox = o % B;
        const int v = (int)ref[((int64_t)(g.cz - H + oz) * p.ny + (g.cy - H + oy)) * p.nx +
                               (g.cx - H + ox)] - 2048;
        tp16[2 * (((oz >> 1) * B + oy) * BP + ox) + (oz & 1)] = (int16_t)v;
        red[0] += v;
        red[1] += v * v;
    }
    // ---- stage the window F' = F - 2048 (zero outside the real window)
    stage_box(flt, p.nx, p.ny, g.wx0, g.wy0, g.wz0, ex, ey, ez, win, PX, PY, PZ,
              [](uint16_t v) { return (int16_t)((int)v - 2048); });
    wg_sum<long long, 2>(red, s_red);  // includes the barrier that publishes LDS
    const long long sT = red[0];
    const long long varT = (long long)N * red[1] - sT * sT;
    if (varT == 0) {  // flat block: every NCC is 0, the smallest shift index wins
        if (tid == 0) write_result(p, blk, g.lox, g.loy, g.loz, 0.0f);
        return;
    }

    // ---- exhaustive search over this workgroup's displacement tiles
    const int32_t *stat_s = static_cast<const int32_t *>(p.stat_s);
    const float *stat_r = static_cast<const float *>(p.stat_r);
    const double dN = (double)N, dST = (double)sT;
    const int side = 2 * p.w + 1;
    float bk = -INFINITY;
    int bi = INT_MAX;
    const int ntiles = txn * tyn * g.dz;
    const int plane = PY * PX;
    for (int t = tid; t < ntiles; t += NT) {
        const int tx = t % txn, ty = (t / txn) % tyn, dz = t / (txn * tyn);
        int acc[RX][RY];
        int acc0[RX][RY];
        double dacc[NG > 2 ? RX : 1][NG > 2 ? RY : 1];
#pragma unroll
        for (int i = 0; i < RX; ++i)
#pragma unroll
            for (int j = 0; j < RY; ++j) {
                acc[i][j] = 0;
                acc0[i][j] = 0;
                if constexpr (NG > 2) dacc[i][j] = 0.0;
            }
        const int16_t *base = win + (dz * PY + ty * RY) * PX + tx * RX;
        for (int m = 0; m < P; ++m) {
            int tq[B][B];
            const int32_t *tpm = tp + m * B * BP;
#pragma unroll
            for (int oy = 0; oy < B; ++oy)
#pragma unroll
                for (int ox = 0; ox < B; ++ox) tq[oy][ox] = tpm[oy * BP + ox];
            const int16_t *w0 = base + 2 * m * plane;
            const int16_t *w1 = w0 + plane;
#pragma unroll
            for (int yw = 0; yw < RY + B - 1; ++yw) {
                short2v f[RX + B - 1];
#pragma unroll
                for (int xw = 0; xw < RX + B - 1; ++xw) {
                    f[xw].x = w0[yw * PX + xw];
                    f[xw].y = w1[yw * PX + xw];
                }
#pragma unroll
                for (int j = 0; j < RY; ++j) {
                    const int oy = yw - j;
                    if (oy < 0 || oy >= B) continue;
#pragma unroll
                    for (int i = 0; i < RX; ++i)
#pragma unroll
                        for (int ox = 0; ox < B; ++ox)
                            acc[i][j] = __builtin_amdgcn_sdot2(
                                f[i + ox], __builtin_bit_cast(short2v, tq[oy][ox]), acc[i][j],
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
        // ---- rank this tile's displacements
#pragma unroll
        for (int i = 0; i < RX; ++i)
#pragma unroll
            for (int j = 0; j < RY; ++j) {
                const int xx = tx * RX + i, yy = ty * RY + j;
                if (xx < g.dx && yy < g.dy) {
                    const int64_t o = ((int64_t)(g.wz0 + dz) * p.oy + (g.wy0 + yy)) * p.ox +
                                      (g.wx0 + xx);
                    double x;
                    if constexpr (NG == 1)
                        x = (double)acc[i][j];
                    else if constexpr (NG == 2)
                        x = (double)acc0[i][j] + (double)acc[i][j];
                    else
                        x = dacc[i][j] + (double)acc[i][j];
                    const double cov = __builtin_fma(dN, x, -dST * (double)stat_s[o]);
                    const float key = (float)cov * stat_r[o];
                    const int iota = ((g.loz + dz + p.w) * side + (g.loy + yy + p.w)) * side +
                                     (g.lox + xx + p.w);
                    better(bk, bi, key, iota);
                }
            }
    }
    wg_argmax(bk, bi, s_key, s_idx);
    if (bi == INT_MAX) {  // no finite key (cannot happen for 12-bit input): report, never index
        if (tid == 0) write_result(p, blk, 0, 0, 0, NAN);
        return;
    }

    // ---- exact NCC at the winning displacement (integer sums of raw voxels)
    const int ddx = bi % side - p.w, ddy = (bi / side) % side - p.w, ddz = bi / (side * side) - p.w;
    long long sums[5] = {0, 0, 0, 0, 0};  // T, T^2, F, F^2, TF
    for (int o = tid; o < N; o += NT) {
        const int oz = o / (B * B), oy = (o / B) % B, ox = o % B;
        const long long tv = ref[((int64_t)(g.cz - H + oz) * p.ny + (g.cy - H + oy)) * p.nx +
                                 (g.cx - H + ox)];
        const long long fv = flt[((int64_t)(g.cz - H + ddz + oz) * p.ny + (g.cy - H + ddy + oy)) *
                                     p.nx +
                                 (g.cx - H + ddx + ox)];
        sums[0] += tv;
        sums[1] += tv * tv;
        sums[2] += fv;
        sums[3] += fv * fv;
        sums[4] += tv * fv;
    }
    wg_sum<long long, 5>(sums, s_red);
    if (tid == 0) {
        const long long vt = (long long)N * sums[1] - sums[0] * sums[0];
        const long long vf = (long long)N * sums[3] - sums[2] * sums[2];
        const long long cv = (long long)N * sums[4] - sums[0] * sums[2];
        const double v = (vt > 0 && vf > 0) ? (double)cv / sqrt((double)vt * (double)vf) : 0.0;
        write_result(p, blk, ddx, ddy, ddz, (float)v);
    }
}

// ---------------------------------------------------------- float volumes

template <int B, int RX, int RY>
__global__ __launch_bounds__(NT) void k_match_f32(Params p) {
    constexpr int H = (B - 1) / 2, BP = (B + 3) & ~3, N = B * B * B;
    extern __shared__ __align__(16) unsigned char lds[];
    float *tf = reinterpret_cast<float *>(lds);            // [B][B][BP]
    float *win = reinterpret_cast<float *>(lds + B * B * BP * 4);  // [PZ][PY][PX]
    __shared__ double s_key[NT / 64];
    __shared__ int s_idx[NT / 64];
    __shared__ double s_red[(NT / 64) * 3];

    const int64_t blk = p.first + xcd_block(blockIdx.x, gridDim.x);
    const Geom g = make_geom(p, blk, H);
    const int tid = threadIdx.x;
    if (!g.inside) {
        if (tid == 0) write_result(p, blk, 0, 0, 0, NAN);
        return;
    }
    const float *ref = static_cast<const float *>(p.ref);
    const float *flt = static_cast<const float *>(p.flt);
    const int txn = (g.dx + RX - 1) / RX, tyn = (g.dy + RY - 1) / RY;
    const int PX = (txn * RX + B - 1 + 3) & ~3, PY = tyn * RY + B - 1, PZ = g.dz + B - 1;
    const int ex = g.dx + B - 1, ey = g.dy + B - 1;

    auto tval = [&](int o) {
        const int oz = o / (B * B), oy = (o / B) % B, ox = o % B;
        return (double)ref[((int64_t)(g.cz - H + oz) * p.ny + (g.cy - H + oy)) * p.nx +
                           (g.cx - H + ox)];
    };
    // ---- mean of T, centred T^ (float) and its FP64 sums
    double r1[1] = {0.0};
    for (int o = tid; o < N; o += NT) r1[0] += tval(o);
    wg_sum<double, 1>(r1, s_red);
    const double tmean = r1[0] / (double)N;
    const float c = (float)tmean;
    double r2[2] = {0.0, 0.0};  // sum T^, sum T^^2 of the float values used
    for (int i = tid; i < B * B * BP; i += NT) {
        const int oz = i / (B * BP), oy = (i / BP) % B, ox = i % BP;
        float v = 0.0f;
        if (ox < B) {
            v = (float)(tval((oz * B + oy) * B + ox) - tmean);
            r2[0] += (double)v;
            r2[1] += (double)v * (double)v;
        }
        tf[i] = v;
    }
    stage_box(flt, p.nx, p.ny, g.wx0, g.wy0, g.wz0, ex, ey, PZ, win, PX, PY, PZ,
              [c](float v) { return v - c; });
    wg_sum<double, 2>(r2, s_red);
    const double sT = r2[0];
    if (!(r2[1] > 0.0)) {  // flat block
        if (tid == 0) write_result(p, blk, g.lox, g.loy, g.loz, 0.0f);
        return;
    }

    const double *stat_s = static_cast<const double *>(p.stat_s);
    const double *stat_r = static_cast<const double *>(p.stat_r);
    const double dN = (double)N, nc = dN * (double)c;
    const int side = 2 * p.w + 1;
    double bk = -INFINITY;
    int bi = INT_MAX;
    const int ntiles = txn * tyn * g.dz;
    const int plane = PY * PX;
    for (int t = tid; t < ntiles; t += NT) {
        const int tx = t % txn, ty = (t / txn) % tyn, dz = t / (txn * tyn);
        float acc[RX][RY];
#pragma unroll
        for (int i = 0; i < RX; ++i)
#pragma unroll
            for (int j = 0; j < RY; ++j) acc[i][j] = 0.0f;
        const float *base = win + (dz * PY + ty * RY) * PX + tx * RX;
        for (int oz = 0; oz < B; ++oz) {
            float tq[B][B];
            const float *tz = tf + oz * B * BP;
#pragma unroll
            for (int oy = 0; oy < B; ++oy)
#pragma unroll
                for (int ox = 0; ox < B; ++ox) tq[oy][ox] = tz[oy * BP + ox];
            const float *w0 = base + oz * plane;
#pragma unroll
            for (int yw = 0; yw < RY + B - 1; ++yw) {
                float f[RX + B - 1];
#pragma unroll
                for (int xw = 0; xw < RX + B - 1; ++xw) f[xw] = w0[yw * PX + xw];
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
        }
#pragma unroll
        for (int i = 0; i < RX; ++i)
#pragma unroll
            for (int j = 0; j < RY; ++j) {
                const int xx = tx * RX + i, yy = ty * RY + j;
                if (xx < g.dx && yy < g.dy) {
                    const int64_t o = ((int64_t)(g.wz0 + dz) * p.oy + (g.wy0 + yy)) * p.ox +
                                      (g.wx0 + xx);
                    // cov * N = N * sum T^(F-c) - sum T^ * (sum F - N c)
                    const double cov = dN * (double)acc[i][j] - sT * (stat_s[o] - nc);
                    const double key = cov * stat_r[o];
                    const int iota = ((g.loz + dz + p.w) * side + (g.loy + yy + p.w)) * side +
                                     (g.lox + xx + p.w);
                    better(bk, bi, key, iota);
                }
            }
    }
    wg_argmax(bk, bi, s_key, s_idx);
    if (bi == INT_MAX) {  // every key NaN (non-finite input): report, never index
        if (tid == 0) write_result(p, blk, 0, 0, 0, NAN);
        return;
    }

    // ---- exact two-pass FP64 NCC at the winning displacement
    const int ddx = bi % side - p.w, ddy = (bi / side) % side - p.w, ddz = bi / (side * side) - p.w;
    auto fval = [&](int o) {
        const int oz = o / (B * B), oy = (o / B) % B, ox = o % B;
        return (double)flt[((int64_t)(g.cz - H + ddz + oz) * p.ny + (g.cy - H + ddy + oy)) * p.nx +
                           (g.cx - H + ddx + ox)];
    };
    double m2[1] = {0.0};
    for (int o = tid; o < N; o += NT) m2[0] += fval(o);
    wg_sum<double, 1>(m2, s_red);
    const double fmean = m2[0] / (double)N;
    double q[3] = {0.0, 0.0, 0.0};  // A, B, X
    for (int o = tid; o < N; o += NT) {
        const double a = tval(o) - tmean, b = fval(o) - fmean;
        q[0] += a * a;
        q[1] += b * b;
        q[2] += a * b;
    }
    wg_sum<double, 3>(q, s_red);
    if (tid == 0) {
        const double ab = q[0] * q[1];
        const double v = ab > 0.0 ? q[2] / sqrt(ab) : 0.0;
        write_result(p, blk, ddx, ddy, ddz, (float)v);
    }
}

// ------------------------------------------------------------ dispatch

typedef void (*kernel_t)(Params);

struct Variant {
    nrr_dtype dtype;
    int b, rx, ry;
    kernel_t fn;
};

#define U16V(B, RX, RY) {NRR_U16, B, RX, RY, k_match_u16<B, RX, RY>}
#define F32V(B, RX, RY) {NRR_F32, B, RX, RY, k_match_f32<B, RX, RY>}

const Variant kVariants[] = {
    U16V(3, 4, 4),  U16V(3, 3, 7),  U16V(3, 5, 5),  U16V(5, 4, 4),  U16V(5, 3, 7),
    U16V(5, 5, 5),  U16V(7, 4, 4),  U16V(7, 3, 7),  U16V(7, 5, 5),  U16V(9, 4, 4),
    U16V(9, 3, 7),  U16V(9, 5, 5),  U16V(11, 3, 3), U16V(13, 3, 3), U16V(15, 2, 2),
    F32V(3, 4, 4),  F32V(5, 4, 4),  F32V(7, 4, 4),  F32V(9, 4, 4),  F32V(11, 3, 3),
    F32V(13, 3, 3), F32V(15, 2, 2),
};

size_t lds_bytes(nrr_dtype dtype, int b, int rx, int ry, int w) {
    const int d = 2 * w + 1;
    const int px = ((d + rx - 1) / rx * rx + b - 1 + 3) & ~3, py = (d + ry - 1) / ry * ry + b - 1;
    const int bp = (b + 3) & ~3;
    if (dtype == NRR_U16) {
        const int pz = d + b;
        return (size_t)((b + 1) / 2) * b * bp * 4 + (size_t)pz * py * px * 2;
    }
    const int pz = d + b - 1;
    return (size_t)b * b * bp * 4 + (size_t)pz * py * px * 4;
}

// Cost model for choosing the displacement tile: padded tiles times the
// per-tile instruction count (multiply-adds plus LDS element reads).
double tile_cost(const Variant &v, int w) {
    const int d = 2 * w + 1;
    const double tiles = (double)((d + v.rx - 1) / v.rx) * ((d + v.ry - 1) / v.ry);
    const double per = (double)v.rx * v.ry * v.b * v.b +
                       (v.dtype == NRR_U16 ? 2.0 : 1.0) * (v.rx + v.b - 1) * (v.ry + v.b - 1);
    return tiles * per;
}

const Variant *choose(nrr_dtype dtype, int b, int w, size_t limit) {
    const Variant *best = nullptr;
    double bc = 0.0;
    for (const Variant &v : kVariants) {
        if (v.dtype != dtype || v.b != b) continue;
        if (lds_bytes(dtype, b, v.rx, v.ry, w) + 1024 > limit) continue;
        const double c = tile_cost(v, w);
        if (!best || c < bc) {
            best = &v;
            bc = c;
        }
    }
    return best;
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
    if (!choose(dtype, block, window, device_lds_limit()))
        return "search window does not fit in LDS for this block size";
    return nullptr;
}

hipError_t launch_match(nrr_dtype dtype, const MatchArgs &a, hipStream_t stream) {
    const size_t limit = device_lds_limit();
    const Variant *v = choose(dtype, a.block, a.window, limit);
    if (!v) return hipErrorInvalidValue;
    const size_t lds = lds_bytes(dtype, a.block, v->rx, v->ry, a.window);
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(v->fn),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
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
    p.stat_s = a.stat_s;
    p.stat_r = a.stat_r;
    p.ox = a.ox;
    p.oy = a.oy;
    p.disp = a.disp;
    p.ncc = a.ncc;
    p.conf = a.conf;
    const int64_t chunk = 1ll << 30;
    for (int64_t first = 0; first < a.n; first += chunk) {
        p.first = first;
        const int64_t cnt = a.n - first < chunk ? a.n - first : chunk;
        hipLaunchKernelGGL(v->fn, dim3((unsigned)cnt), dim3(NT), lds, stream, p);
    }
    return hipGetLastError();
}

}  // namespace nrr
