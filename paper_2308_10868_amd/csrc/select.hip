// Variance-ranked block selection on the GPU.
//
// Follows the "Parallel feature selection" paragraph of the paper's HPC
// section: every candidate block's intensity variance is computed, the
// candidates are ranked by it and K = floor(0.5 + N * Fs) are kept.  The
// paper sorts (variance, index) pairs per thread and merges them; here the
// K-th largest key is found by a radix select over 64-bit keys (no sort of
// the N candidates is needed) and the chosen blocks are written in ascending
// grid index by an ordered compaction (counts, a scan, placement by rank:
// inside the one-workgroup select on grids of up to 32,768 candidates, two
// kernels after the multi-workgroup select otherwise).  Ties (equal variance)
// are broken by the lower grid index, so the result is deterministic.
//
// Keys: u16 volumes use the exact integer N*sum(x^2) - (sum x)^2 (= N^2 times
// the variance, < 2^47 for 12-bit data and b <= 15, < 2^54 for any 16-bit
// values); f32 volumes use the FP64 two-pass
// variance summed in z, y, x order without FMA contraction (bit pattern of a
// non-negative double is monotone in its value).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "nrr_internal.h"
#include "stats_cols.h"

namespace nrr {
namespace {

struct SelectState {
    uint64_t kth;     // value of the K-th largest key
    int64_t take_eq;  // how many candidates with key == kth are kept (lowest indices)
};

// One wavefront per candidate block (grids whose candidates do not overlap,
// or whose tile region is too large for the tiled kernel): lanes take the
// block's by*bz rows, sum them exactly in integers and reduce across the
// wavefront.
__global__ __launch_bounds__(256) void k_block_keys_u16(const uint16_t *__restrict__ vol, int nx,
                                                        int ny, BoxGrid G, int64_t n,
                                                        uint64_t *__restrict__ keys) {
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= n) return;  // whole wavefront leaves together
    const int bx = G.b[0], by = G.b[1], bz = G.b[2];
    // candidate coordinates in 32-bit arithmetic (grids hold < 2^31 candidates)
    const int gi = (int)g, gxy = G.g[0] * G.g[1];
    const int iz = gi / gxy, rr = gi - iz * gxy, iy = rr / G.g[0], ix = rr - iy * G.g[0];
    const int64_t x0 = (int64_t)ix * G.s[0], y0 = (int64_t)iy * G.s[1], z0 = (int64_t)iz * G.s[2];
    uint64_t s = 0, q = 0;
    for (int r = lane; r < by * bz; r += 64) {
        const int z = r / by, y = r - z * by;
        const uint16_t *row = vol + ((z0 + z) * ny + (y0 + y)) * (int64_t)nx + x0;
        uint64_t rs = 0, rq = 0;
        for (int x = 0; x < bx; ++x) {
            const uint64_t v = row[x];
            rs += v;
            rq += v * v;
        }
        s += rs;
        q += rq;
    }
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_xor(s, off);
        q += __shfl_xor(q, off);
    }
    if (lane == 0) keys[g] = (uint64_t)bx * by * bz * q - s * s;  // >= 0 by Cauchy-Schwarz
}

// Keys by candidate rows (grids whose candidates do not overlap in x and y):
// a workgroup takes the candidates of one (y, z) grid row whose columns fit
// in 64 voxels.  Lane t owns voxel column x0 + t; the four wavefronts split
// the block's bz planes (every load a contiguous run of 64 voxels, a plane's
// by rows issued together) and each candidate adds its bx columns of the
// four partial sums from LDS.
__global__ __launch_bounds__(256) void k_block_keys_u16_rows(const uint16_t *__restrict__ vol,
                                                             int nx, int ny, BoxGrid G, int cx,
                                                             uint64_t *__restrict__ keys) {
    __shared__ uint32_t col_s[4][64];
    __shared__ uint64_t col_q[4][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int bx = G.b[0], by = G.b[1], bz = G.b[2], sx = G.s[0];
    const int c0 = blockIdx.x * cx, iy = blockIdx.y, iz = blockIdx.z;
    const int ncx = min(cx, G.g[0] - c0);
    const int width = (ncx - 1) * sx + bx;  // <= 64 by the choice of cx
    const int64_t x0 = (int64_t)c0 * sx;
    uint32_t a = 0;  // <= 225 voxels of 16 bits
    uint64_t q = 0;
    // columns in the gaps between candidates (stride above the edge) are skipped
    if (lane < width && lane % sx < bx) {
        const int64_t plane = (int64_t)ny * nx;
        const uint16_t *base =
            vol + ((int64_t)iz * G.s[2] * ny + (int64_t)iy * G.s[1]) * nx + x0 + lane;
        for (int z = w; z < bz; z += 4) {
            const uint16_t *p = base + z * plane;
            uint32_t v[15];  // block edges are at most 15
#pragma unroll
            for (int y = 0; y < 15; ++y) v[y] = y < by ? p[(int64_t)y * nx] : 0u;
#pragma unroll
            for (int y = 0; y < 15; ++y) {
                a += v[y];
                q += (uint64_t)(v[y] * v[y]);  // a square of 16 bits fits 32
            }
        }
    }
    col_s[w][lane] = a;
    col_q[w][lane] = q;
    __syncthreads();
    if (tid < ncx) {
        uint64_t s = 0, qq = 0;
        for (int k = 0; k < bx; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                s += col_s[j][tid * sx + k];
                qq += col_q[j][tid * sx + k];
            }
        const int64_t g = ((int64_t)iz * G.g[1] + iy) * G.g[0] + c0 + tid;
        keys[g] = (uint64_t)bx * by * bz * qq - s * s;
    }
}

// Tiled keys for overlapping candidates (tile regions up to 120 voxels a side): a
// workgroup takes 16 x 16 candidates in x and y at one candidate plane z.
// For each of the block's bz voxel planes it stages the tile's region
// ((15 sx + bx) x (15 sy + by) voxels, rows along x, coalesced) in LDS, forms
// for every region row the sums over each candidate column's bx voxels, and
// each thread adds its candidate's by rows of those.  Every voxel of the
// region is read from L2 once per candidate plane that contains it.
constexpr int KT = 16, KT_MAXR = 120;  // region edge 15 s + b at most 120

__global__ __launch_bounds__(256) void k_block_keys_u16_tiled(const uint16_t *__restrict__ vol,
                                                              int nx, int ny, BoxGrid G,
                                                              uint64_t *__restrict__ keys) {
    // dynamic LDS: the region [RY][RX] (u16, RX even), then the row sums
    // [RY][KT] and sums of squares [RY][KT] (u32); RX, RY of a full tile
    extern __shared__ __align__(16) unsigned char lds_keys[];
    const int RX = ((KT - 1) * G.s[0] + G.b[0] + 1) & ~1, RY = (KT - 1) * G.s[1] + G.b[1];
    uint16_t *reg = reinterpret_cast<uint16_t *>(lds_keys);
    uint32_t *rsum = reinterpret_cast<uint32_t *>(lds_keys + (size_t)RX * RY * 2);
    uint32_t *rsq = rsum + RY * KT;
    const int tid = threadIdx.x;
    const int bx = G.b[0], by = G.b[1], bz = G.b[2];
    const int cx0 = blockIdx.x * KT, cy0 = blockIdx.y * KT, cz = blockIdx.z;
    const int ncx = min(KT, G.g[0] - cx0), ncy = min(KT, G.g[1] - cy0);
    const int rx = (ncx - 1) * G.s[0] + bx, ry = (ncy - 1) * G.s[1] + by;  // region in the volume
    const int64_t x0 = (int64_t)cx0 * G.s[0], y0 = (int64_t)cy0 * G.s[1];
    const int64_t z0 = (int64_t)cz * G.s[2];
    const int i = tid % KT, j = tid / KT;  // this thread's candidate in the tile
    uint64_t s_acc = 0, q_acc = 0;
    for (int pz = 0; pz < bz; ++pz) {
        const uint16_t *pl = vol + ((z0 + pz) * ny + y0) * (int64_t)nx + x0;
        for (int e = tid; e < rx * ry; e += 256) {
            const int r = e / rx, c = e - r * rx;
            reg[r * RX + c] = pl[(int64_t)r * nx + c];
        }
        __syncthreads();
        for (int e = tid; e < ry * ncx; e += 256) {  // row r, candidate column ci
            const int r = e / ncx, ci = e - r * ncx;
            const uint16_t *row = reg + r * RX + ci * G.s[0];
            uint32_t a = 0, b2 = 0;  // bx <= 120 voxels: < 2^32
            for (int k = 0; k < bx; ++k) {
                const uint32_t v = row[k];
                a += v;
                b2 += v * v;
            }
            rsum[r * KT + ci] = a;
            rsq[r * KT + ci] = b2;
        }
        __syncthreads();
        if (i < ncx && j < ncy) {
            for (int k = 0; k < by; ++k) {
                s_acc += rsum[(j * G.s[1] + k) * KT + i];
                q_acc += rsq[(j * G.s[1] + k) * KT + i];
            }
        }
        __syncthreads();  // the region and the row sums are rewritten next plane
    }
    if (i < ncx && j < ncy) {
        const int64_t g = ((int64_t)cz * G.g[1] + cy0 + j) * G.g[0] + cx0 + i;
        keys[g] = (uint64_t)bx * by * bz * q_acc - s_acc * s_acc;
    }
}

// Calls f on every voxel of the BX*by*bz block at base, in z, y, x order.
// A row is BX loads from one address (immediate offsets, straight-line code,
// so the compiler's waits count exactly the loads still needed), and the
// loads of the next three rows are in flight while a row reaches f: a chain
// of dependent additions in f overlaps the memory round trips.  Loads past
// the last row repeat the last row (in bounds, never passed to f).
template <int BX, typename F>
__device__ __forceinline__ void block_rows_in_order(const float *__restrict__ base, int64_t nx,
                                                    int64_t plane, int by, int bz, F &&f) {
    const int rows = by * bz;
    const float *p = base;  // the next row to load
    int y = 0, left = rows - 1;  // rows after the one p points at
    auto load = [&](float(&t)[BX]) {
#pragma unroll
        for (int j = 0; j < BX; ++j) t[j] = p[j];
        if (left > 0) {
            --left;
            if (++y == by) {
                y = 0;
                p += plane - (int64_t)(by - 1) * nx;
            } else {
                p += nx;
            }
        }
    };
    auto use = [&](const float(&t)[BX]) {
#pragma unroll
        for (int j = 0; j < BX; ++j) f(t[j]);
    };
    float t0[BX], t1[BX], t2[BX], t3[BX];  // a ring: row r in t[r % 4]
    load(t0);
    load(t1);
    load(t2);
    for (int r = 0; r < rows; r += 4) {
        load(t3);
        use(t0);
        load(t0);
        if (r + 1 < rows) use(t1);
        load(t1);
        if (r + 2 < rows) use(t2);
        load(t2);
        if (r + 3 < rows) use(t3);
    }
}

// FP64 two-pass variance of the BX*by*bz block at base, summed in z, y, x
// order without contraction; returned as its (monotone) bit pattern.
template <int BX>
__device__ __forceinline__ uint64_t key_f32_rows(const float *__restrict__ base, int64_t nx,
                                                 int64_t plane, int by, int bz) {
#pragma clang fp contract(off)
    const double dn = (double)BX * by * bz;
    double sum = 0.0;
    block_rows_in_order<BX>(base, nx, plane, by, bz, [&](float v) { sum += (double)v; });
    const double mean = sum / dn;
    double ss = 0.0;
    block_rows_in_order<BX>(base, nx, plane, by, bz, [&](float v) {
        const double d = (double)v - mean;
        ss += d * d;
    });
    return (uint64_t)__double_as_longlong(ss / dn);
}

// FP64 two-pass variance of the bx*by*bz block at (x0, y0, z0), summed in
// z, y, x order without contraction; returned as its (monotone) bit pattern.
// Odd row lengths up to 15 take the prefetching row walk, others plain loops
// (the same order, so the same result).
__device__ __forceinline__ uint64_t key_f32(const float *__restrict__ vol, int nx, int ny, int bx,
                                            int by, int bz, int64_t x0, int64_t y0,
                                            int64_t z0) {
#pragma clang fp contract(off)
    const float *base = vol + (z0 * ny + y0) * (int64_t)nx + x0;
    const int64_t plane = (int64_t)ny * nx;
    switch (bx) {
    case 3: return key_f32_rows<3>(base, nx, plane, by, bz);
    case 5: return key_f32_rows<5>(base, nx, plane, by, bz);
    case 7: return key_f32_rows<7>(base, nx, plane, by, bz);
    case 9: return key_f32_rows<9>(base, nx, plane, by, bz);
    case 11: return key_f32_rows<11>(base, nx, plane, by, bz);
    case 13: return key_f32_rows<13>(base, nx, plane, by, bz);
    case 15: return key_f32_rows<15>(base, nx, plane, by, bz);
    default: break;
    }
    const double dn = (double)bx * by * bz;
    double sum = 0.0;
    for (int z = 0; z < bz; ++z)
        for (int y = 0; y < by; ++y) {
            const float *row = base + (int64_t)z * plane + (int64_t)y * nx;
            for (int x = 0; x < bx; ++x) sum += (double)row[x];
        }
    const double mean = sum / dn;
    double ss = 0.0;
    for (int z = 0; z < bz; ++z)
        for (int y = 0; y < by; ++y) {
            const float *row = base + (int64_t)z * plane + (int64_t)y * nx;
            for (int x = 0; x < bx; ++x) {
                const double d = (double)row[x] - mean;
                ss += d * d;
            }
        }
    return (uint64_t)__double_as_longlong(ss / dn);  // var >= +0: bit pattern is monotone
}

// Float keys, one thread per candidate.  64-thread workgroups spread a small
// grid's candidates over many CUs: a wavefront's loads reach one cache line
// per few lanes, so each CU's vector memory path is the bound.
__global__ __launch_bounds__(64) void k_block_keys_f32(const float *__restrict__ vol, int nx,
                                                       int ny, BoxGrid G, int64_t n,
                                                       uint64_t *__restrict__ keys) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int gi = (int)g, gxy = G.g[0] * G.g[1];
    const int iz = gi / gxy, rr = gi - iz * gxy, iy = rr / G.g[0], ix = rr - iy * G.g[0];
    keys[g] = key_f32(vol, nx, ny, G.b[0], G.b[1], G.b[2], (int64_t)ix * G.s[0],
                      (int64_t)iy * G.s[1], (int64_t)iz * G.s[2]);
}

// Count `d` (< 256) into the LDS histogram.  A wavefront whose counted lanes
// all hold the same digit (common in the leading bytes) adds once; otherwise
// every lane adds its own (LDS atomics on distinct bins proceed in parallel).
__device__ inline void hist_add(uint32_t *hist, uint32_t d, bool valid) {
    const uint64_t act = __ballot(valid);
    if (act == 0) return;
    const int leader = __ffsll((unsigned long long)act) - 1;
    const uint32_t dl = __shfl(d, leader);
    const uint64_t same = __ballot(valid && d == dl);
    if (same == act) {
        if ((int)(threadIdx.x & 63) == leader) atomicAdd(&hist[dl], (uint32_t)__popcll(act));
    } else if (valid) {
        atomicAdd(&hist[d], 1u);
    }
}

// Radix select of the K-th largest key, 8 bits per pass from the most
// significant set bit down; one 1024-thread workgroup for grids of at most
// kRadixMultiMin candidates, whose keys it holds in registers (thread t holds
// keys t + 1024 j), so the passes wait on no memory.  A pass counts digits
// into 16 copies of the histogram (copy = lane mod 16: variance keys crowd a
// few bins, and lanes adding to one LDS word serialise), folds them and picks
// the digit that holds the need-th largest key.  Once at most 1024 keys match
// the prefix found so far they are moved to an LDS list, one per thread, and
// the remaining passes read only that.  The first pass is aligned to the
// highest set bit of all keys; the last one may overlap bits already fixed
// (those are equal in every key it counts, so the pick is unchanged).
// K comes from `k`, or from *kd when kd is given (a count made on the device);
// K = 0 selects nothing.  The K-th key and the equal keys kept go to *st when
// st is given.
// The same workgroup then writes the chosen blocks' centres in ascending grid
// index (the ordered compaction, from the registers): per key slot and
// wavefront it counts the keys above and equal to the K-th by ballots, scans
// those counts in index order, and places each kept key by its rank.
constexpr int kThrKeys = (int)(kRadixMultiMin / 1024);  // keys per thread
static_assert(kRadixMultiMin % 1024 == 0, "whole keys per thread");
constexpr int kThrCopies = 16;  // histogram copies (lane mod 16)
constexpr int64_t kSmallSelect = 4096;  // grids up to this size take 4 key slots per thread

// The select's LDS (a struct, so a fused kernel can overlay it with its other
// work's LDS).
struct ThrShared {
    __align__(16) uint32_t hist_c[256 * kThrCopies];  // [digit][copy]
    uint32_t hist[256];
    uint64_t list[1024];
    uint32_t pre[kThrKeys * 16];  // (above | equal << 16) per (slot, wavefront)
    uint64_t s_prefix, s_mask, s_or;
    int64_t s_need;
    uint32_t s_left, s_count;
};

// The select of one 1024-thread workgroup (see above), for at most NK * 1024
// keys (NK key slots per thread).
template <int NK = kThrKeys>
__device__ __attribute__((always_inline)) inline void select_threshold_wg(
    const uint64_t *__restrict__ keys, int64_t n, int64_t k, const int64_t *__restrict__ kd,
    SelectState *__restrict__ st, const BoxGrid &G, int32_t *__restrict__ centers,
    ThrShared &sm) {
    static_assert(NK % 4 == 0 && NK <= kThrKeys, "whole scan entries, within the LDS tables");
    uint32_t *hist_c = sm.hist_c, *hist = sm.hist, *pre = sm.pre;
    uint64_t *list = sm.list;
    uint64_t &s_prefix = sm.s_prefix, &s_mask = sm.s_mask, &s_or = sm.s_or;
    int64_t &s_need = sm.s_need;
    uint32_t &s_left = sm.s_left, &s_count = sm.s_count;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t kk = kd ? *kd : k;  // K
    if (tid == 0) {
        s_prefix = 0;
        s_mask = 0;
        s_need = kk;
        s_or = 0;
        s_count = 0;
    }
    uint64_t kr[NK];  // all loads issued before any is used
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const int64_t i = (int64_t)j * 1024 + tid;
        kr[j] = i < n ? keys[i] : 0;
    }
    __syncthreads();
    uint64_t orv = 0;
#pragma unroll
    for (int j = 0; j < NK; ++j) orv |= kr[j];
    for (int off = 32; off > 0; off >>= 1) orv |= __shfl_xor(orv, off);
    if (lane == 0) atomicOr((unsigned long long *)&s_or, (unsigned long long)orv);
    __syncthreads();
    const int bits = s_or ? 64 - __clzll((long long)s_or) : 1;
    bool in_list = false;  // workgroup-uniform
    uint32_t n_list = 0;
    for (int shift = bits > 8 ? bits - 8 : 0;; shift = shift > 8 ? shift - 8 : 0) {
        const uint64_t prefix = s_prefix, mask = s_mask;
        if (!in_list) {
            uint32_t *hrow = hist_c + (tid & (kThrCopies - 1));
            for (int i = tid; i < 256 * kThrCopies; i += 1024) hist_c[i] = 0;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < NK; ++j)
                if ((int64_t)j * 1024 + tid < n && (kr[j] & mask) == prefix)
                    atomicAdd(&hrow[((kr[j] >> shift) & 0xff) * kThrCopies], 1u);
            __syncthreads();
            if (tid < 256) {
                const uint4 *c = reinterpret_cast<const uint4 *>(hist_c + tid * kThrCopies);
                uint32_t t = 0;
#pragma unroll
                for (int q = 0; q < kThrCopies / 4; ++q) t += c[q].x + c[q].y + c[q].z + c[q].w;
                hist[tid] = t;
            }
        } else {  // at most 1024 keys: one histogram
            if (tid < 256) hist[tid] = 0;
            __syncthreads();
            if (tid < (int)n_list && (list[tid] & mask) == prefix)
                atomicAdd(&hist[(list[tid] >> shift) & 0xff], 1u);
        }
        __syncthreads();
        if (tid < 64) {  // wavefront 0: find the digit holding the need-th largest key
            // (every thread read the previous pass's s_left before this
            // pass's first barrier; the picking lane's store comes later in
            // this wavefront's program order than this one)
            if (tid == 0) s_left = 0xffffffffu;
            // lane l owns bins 255-4l .. 252-4l (descending)
            uint32_t h4[4];
            uint32_t mine = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                h4[j] = hist[255 - 4 * tid - j];
                mine += h4[j];
            }
            // exclusive prefix over lower lanes = count of keys in higher bins
            uint32_t incl = mine;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t o = __shfl_up(incl, off);
                if (tid >= off) incl += o;
            }
            const int64_t need = s_need;
            const int64_t above = (int64_t)(incl - mine);
            if (above < need && need <= (int64_t)incl) {
                int64_t cum = above;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (cum + h4[j] >= need) {
                        const int d = 255 - 4 * tid - j;
                        s_need = need - cum;
                        s_prefix = prefix | ((uint64_t)d << shift);
                        s_mask = mask | (0xffull << shift);
                        s_left = h4[j];  // keys matching the new prefix
                        break;
                    }
                    cum += h4[j];
                }
            }
        }
        __syncthreads();
        if (shift == 0) break;
        if (!in_list && s_need > 0 && s_left <= 1024) {
            // move the keys that still match to the LDS list: one slot
            // range per wavefront (one atomic), then its keys in slot order
            const uint64_t p2 = s_prefix, m2 = s_mask;
            uint32_t mm = 0, wave_total = 0;
#pragma unroll
            for (int j = 0; j < NK; ++j) {
                const bool m = (int64_t)j * 1024 + tid < n && (kr[j] & m2) == p2;
                mm |= (uint32_t)m << j;
                wave_total += (uint32_t)__popcll(__ballot(m));
            }
            uint32_t base = 0;
            if (lane == 0 && wave_total) base = atomicAdd(&s_count, wave_total);
            base = __shfl(base, 0);
#pragma unroll
            for (int j = 0; j < NK; ++j) {
                const bool m = (mm >> j) & 1;
                const uint64_t b = __ballot(m);
                const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
                if (m && base + below < 1024) list[base + below] = kr[j];
                base += (uint32_t)__popcll(b);
            }
            __syncthreads();
            in_list = true;
            n_list = min(s_count, 1024u);
        }
    }
    if (tid == 0 && st) {
        st->kth = s_prefix;
        st->take_eq = s_need;
    }
    // ordered compaction: key 1024 j + tid sits in slot j of wavefront w's
    // lane; index order is (slot, wavefront, lane)
    const uint64_t kth = s_prefix;
    const int64_t take = s_need;  // equal keys kept, lowest indices first
    uint32_t fgt = 0, feq = 0;  // bit j: key j of this thread is above / equal to the K-th
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const bool in = (int64_t)j * 1024 + tid < n;
        const bool gt = in && kr[j] > kth, eq = in && kr[j] == kth;
        fgt |= (uint32_t)gt << j;
        feq |= (uint32_t)eq << j;
        const uint32_t a = (uint32_t)__popcll(__ballot(gt));
        const uint32_t e = (uint32_t)__popcll(__ballot(eq));
        if (lane == 0) pre[j * 16 + w] = a | e << 16;  // each < 2^16 (n <= 2^15)
    }
    __syncthreads();
    if (tid < 64) {  // exclusive scan of the NK * 16 entries, NK / 4 per lane
        constexpr int PL = NK * 16 / 64;
        uint32_t v[PL], sum = 0;
#pragma unroll
        for (int i = 0; i < PL; ++i) {
            v[i] = pre[tid * PL + i];
            sum += v[i];
        }
        uint32_t incl = sum;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(incl, off);
            if (tid >= off) incl += o;
        }
        uint32_t run = incl - sum;
#pragma unroll
        for (int i = 0; i < PL; ++i) {
            pre[tid * PL + i] = run;
            run += v[i];
        }
    }
    __syncthreads();
    // counts, ranks and grid indices below 2^15 + 1: 32-bit arithmetic, and
    // the grid coordinates by a float reciprocal corrected by one step
    const int gxy = G.g[0] * G.g[1], take32 = (int)take, k32 = (int)kk;
    const float inv_gxy = 1.0f / (float)gxy, inv_gx = 1.0f / (float)G.g[0];
    auto div_small = [](int a, int d, float inv) {  // floor(a / d), 0 <= a < 2^24
        int q = (int)((float)a * inv);
        const int r = a - q * d;
        return r < 0 ? q - 1 : (r >= d ? q + 1 : q);
    };
    const int nslots = (int)((n + 1023) / 1024);
#pragma unroll 1
    for (int j = 0; j < nslots; ++j) {  // the flags are bits: no key register is indexed
        const int g = j * 1024 + tid;
        const bool gt = (fgt >> j) & 1, eq = (feq >> j) & 1;
        const uint64_t bg = __ballot(gt), be = __ballot(eq);
        const uint32_t p = pre[j * 16 + w];
        const int gt_before = (int)((p & 0xffff) + __builtin_amdgcn_mbcnt_hi(
            (uint32_t)(bg >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bg, 0u)));
        const int eq_before = (int)((p >> 16) + __builtin_amdgcn_mbcnt_hi(
            (uint32_t)(be >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)be, 0u)));
        const bool keep = gt || (eq && eq_before < take32);
        const int pos = gt_before + min(eq_before, take32);
        if (keep && pos < k32) {
            const int iz = div_small(g, gxy, inv_gxy), rr = g - iz * gxy;
            const int iy = div_small(rr, G.g[0], inv_gx), ix = rr - iy * G.g[0];
            centers[3 * pos + 0] = (int32_t)(ix * G.s[0] + (G.b[0] - 1) / 2);
            centers[3 * pos + 1] = (int32_t)(iy * G.s[1] + (G.b[1] - 1) / 2);
            centers[3 * pos + 2] = (int32_t)(iz * G.s[2] + (G.b[2] - 1) / 2);
        }
    }
}

// NK key slots per thread: grids of at most NK * 1024 candidates.
template <int NK>
__global__ __launch_bounds__(1024) void k_select_threshold(const uint64_t *__restrict__ keys,
                                                           int64_t n, int64_t k,
                                                           const int64_t *__restrict__ kd,
                                                           SelectState *__restrict__ st, BoxGrid G,
                                                           int32_t *__restrict__ centers) {
    __shared__ ThrShared sm;
    select_threshold_wg<NK>(keys, n, k, kd, st, G, centers, sm);
}

// The select and the 12-bit column statistics of a cubic block edge B in one
// launch of 1024-thread workgroups: workgroup 0 is the select (dispatched
// first, it is placed on a free CU before the statistics fill the device);
// every other workgroup runs 16 statistics wavefronts (wavefront id = x-tile
// fastest, then y-tile, then z-run).  No stream fork or join is needed.
union SelectStatsShared {
    ThrShared thr;
    uint2 xch[16][SC_RY][SC_LW];
};

template <int B>
__global__ __launch_bounds__(1024) void k_select_stats(
    const uint64_t *__restrict__ keys, int64_t n, int64_t k, SelectState *__restrict__ st,
    BoxGrid G, int32_t *__restrict__ centers, const uint16_t *__restrict__ flt, int nx, int ny,
    int nz, int ox, int oy, int oz, int zc, int nwx, int nwy, int64_t nwaves,
    StatU16 *__restrict__ out) {
    __shared__ SelectStatsShared sm;
    if (blockIdx.x == 0) {
        select_threshold_wg(keys, n, k, nullptr, st, G, centers, sm.thr);
        return;
    }
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t wid = (int64_t)(blockIdx.x - 1) * 16 + w;
    if (wid >= nwaves) return;  // whole wavefront
    const int xw = (int)(wid % nwx);
    const int64_t r = wid / nwx;
    const int yw = (int)(r % nwy), run = (int)(r / nwy);
    stats_cols_wave<B, B>(flt, nx, ny, nz, B, B, ox, oy, oz, zc, out, xw, yw, run, sm.xch[w]);
}

// Multi-workgroup radix select for large grids: eight passes of one byte,
// most significant first.  Each pass counts the digits of the keys that
// match the prefix found so far into one histogram row per workgroup; one
// workgroup then sums the rows and picks the digit that holds the need-th
// largest key.  Fixed launches, no host round trip.
constexpr int kRadixWG = 256;  // workgroups of a histogram pass
constexpr int kRadixRows = 8;  // histogram rows they add into (spreads the atomics)

struct RadixState {
    uint64_t prefix, mask;
    int64_t need;
};

__global__ __launch_bounds__(256) void k_radix_init(int64_t k, const int64_t *__restrict__ kd,
                                                    RadixState *__restrict__ rs,
                                                    uint32_t *__restrict__ rows) {
    for (int i = threadIdx.x; i < kRadixRows * 256; i += 256) rows[i] = 0;
    if (threadIdx.x != 0) return;
    rs->prefix = 0;
    rs->mask = 0;
    rs->need = kd ? *kd : k;
}

__global__ __launch_bounds__(256) void k_radix_hist(const uint64_t *__restrict__ keys, int64_t n,
                                                    const RadixState *__restrict__ rs, int shift,
                                                    uint32_t *__restrict__ rows) {
    __shared__ uint32_t hist[256];
    const int tid = threadIdx.x;
    hist[tid] = 0;
    __syncthreads();
    const uint64_t prefix = rs->prefix, mask = rs->mask;
    const int64_t step = (int64_t)gridDim.x * 256;
    // uniform trip count per workgroup so the ballots in hist_add converge
    const int64_t iters = (n + step - 1) / step;
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t i = it * step + (int64_t)blockIdx.x * 256 + tid;
        const uint64_t kv = i < n ? keys[i] : 0;
        hist_add(hist, (uint32_t)((kv >> shift) & 0xff), i < n && (kv & mask) == prefix);
    }
    __syncthreads();
    if (hist[tid]) atomicAdd(&rows[(blockIdx.x % kRadixRows) * 256 + tid], hist[tid]);
}

__global__ __launch_bounds__(256) void k_radix_pick(uint32_t *__restrict__ rows, int nrows,
                                                    int shift, RadixState *__restrict__ rs,
                                                    SelectState *__restrict__ st) {
    __shared__ int64_t s_w[4];
    __shared__ uint64_t s_prefix, s_mask;
    __shared__ int64_t s_need;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) {
        s_prefix = rs->prefix;
        s_mask = rs->mask;
        s_need = rs->need;
    }
    const int d = 255 - tid;  // thread t holds digit 255 - t: descending order
    int64_t c = 0;
    for (int r = 0; r < nrows; ++r) {  // read, then cleared for the next pass
        c += rows[r * 256 + d];
        rows[r * 256 + d] = 0;
    }
    // inclusive scan over the 256 threads
    int64_t incl = c;
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
    }
    if (lane == 63) s_w[w] = incl;
    __syncthreads();
    for (int i = 0; i < w; ++i) incl += s_w[i];
    const int64_t need = s_need, above = incl - c;
    __syncthreads();  // every thread has read s_need before it changes
    if (above < need && need <= incl) {  // one thread at most
        s_need = need - above;
        s_prefix |= (uint64_t)d << shift;
        s_mask |= 0xffull << shift;
    }
    __syncthreads();
    if (tid == 0) {
        rs->prefix = s_prefix;
        rs->mask = s_mask;
        rs->need = s_need;
        if (shift == 0) {  // every byte resolved
            st->kth = s_prefix;
            st->take_eq = s_need;
        }
    }
}

// Per tile of kSelectTile candidates: how many keys are > kth and == kth.
__global__ __launch_bounds__(256) void k_tile_counts(const uint64_t *__restrict__ keys, int64_t n,
                                                     const SelectState *__restrict__ st,
                                                     int64_t *__restrict__ tiles) {
    __shared__ int64_t red[2][4];
    const uint64_t kth = st->kth;
    int64_t base = (int64_t)blockIdx.x * kSelectTile;
    int64_t gt = 0, eq = 0;
    for (int i = threadIdx.x; i < kSelectTile; i += blockDim.x) {
        int64_t g = base + i;
        if (g < n) {
            uint64_t key = keys[g];
            gt += key > kth;
            eq += key == kth;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        gt += __shfl_xor(gt, off);
        eq += __shfl_xor(eq, off);
    }
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = gt;
        red[1][w] = eq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        tiles[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        tiles[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

// Ordered compaction: candidate g is kept if key > kth, or key == kth and
// fewer than take_eq equal keys precede it; its output slot is the number of
// kept candidates before it.  Each thread owns kSelectTile/256 consecutive
// candidates of the workgroup's tile.
__global__ __launch_bounds__(256) void k_compact(const uint64_t *__restrict__ keys, int64_t n,
                                                 const SelectState *__restrict__ st,
                                                 const int64_t *__restrict__ tiles, BoxGrid G,
                                                 int64_t k, const int64_t *__restrict__ kd,
                                                 int32_t *__restrict__ centers) {
    constexpr int PER = kSelectTile / 256;
    if (kd) k = *kd;
    __shared__ int64_t s_gt[256], s_eq[256];
    __shared__ int64_t s_base[2];
    const uint64_t kth = st->kth;
    const int64_t take = st->take_eq;
    const int tid = threadIdx.x;
    // exclusive prefix over earlier tiles (strided partial sums, then reduce)
    int64_t pg = 0, pe = 0;
    for (int64_t t = tid; t < blockIdx.x; t += 256) {
        pg += tiles[2 * t];
        pe += tiles[2 * t + 1];
    }
    s_gt[tid] = pg;
    s_eq[tid] = pe;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) {
            s_gt[tid] += s_gt[tid + off];
            s_eq[tid] += s_eq[tid + off];
        }
        __syncthreads();
    }
    if (tid == 0) {
        s_base[0] = s_gt[0];
        s_base[1] = s_eq[0];
    }
    __syncthreads();
    const int64_t base_gt = s_base[0], base_eq = s_base[1];
    __syncthreads();
    // this thread's candidates and local counts
    const int64_t g0 = (int64_t)blockIdx.x * kSelectTile + (int64_t)tid * PER;
    uint64_t kv[PER];
    int64_t lg = 0, le = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        int64_t g = g0 + j;
        kv[j] = g < n ? keys[g] : 0;
        bool ok = g < n;
        lg += ok && kv[j] > kth;
        le += ok && kv[j] == kth;
    }
    // inclusive scan over the workgroup (Hillis-Steele in LDS)
    s_gt[tid] = lg;
    s_eq[tid] = le;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        int64_t a = tid >= off ? s_gt[tid - off] : 0;
        int64_t e = tid >= off ? s_eq[tid - off] : 0;
        __syncthreads();
        s_gt[tid] += a;
        s_eq[tid] += e;
        __syncthreads();
    }
    int64_t gt_before = base_gt + s_gt[tid] - lg;
    int64_t eq_before = base_eq + s_eq[tid] - le;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        int64_t g = g0 + j;
        if (g >= n) break;
        bool is_gt = kv[j] > kth, is_eq = kv[j] == kth;
        bool keep = is_gt || (is_eq && eq_before < take);
        const int64_t pos = gt_before + (eq_before < take ? eq_before : take);
        if (keep && pos < k) {
            const int gi = (int)g, gxy = G.g[0] * G.g[1];
            const int iz = gi / gxy, rr = gi - iz * gxy, iy = rr / G.g[0], ix = rr - iy * G.g[0];
            centers[3 * pos + 0] = (int32_t)(ix * G.s[0] + (G.b[0] - 1) / 2);
            centers[3 * pos + 1] = (int32_t)(iy * G.s[1] + (G.b[1] - 1) / 2);
            centers[3 * pos + 2] = (int32_t)(iz * G.s[2] + (G.b[2] - 1) / 2);
        }
        gt_before += is_gt;
        eq_before += is_eq;
    }
}


// Inclusive scan of one value per thread over a 1024-thread workgroup
// (wavefront shuffles, then the 16 wavefront totals); `tot` gets the sum.
__device__ inline int64_t wg_scan1024_ex(int64_t v, int64_t *s_w, int64_t *tot) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t o = __shfl_up(v, off);
        if (lane >= off) v += o;
    }
    if (lane == 63) s_w[w] = v;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int i = 0; i < 16; ++i) {
        const int64_t x = s_w[i];
        before += i < w ? x : 0;
        all += x;
    }
    __syncthreads();
    *tot = all;
    return v + before;
}

// ------------------------------------------------------- selection variants
//
// Selection with a candidate mask and a connectivity pattern (the region
// restriction and the connectivity patterns of the parallel feature
// selection paragraph): candidates whose centre lies outside the mask take
// no part (N counts the others, K = floor(0.5 + N * F)); in rank order a
// candidate is taken unless one of its 6/18/26 grid neighbours is already
// taken, until K are taken.  That greedy visit equals the first K (in rank
// order) of the whole greedy set, which parallel rounds compute: a block is
// taken once every neighbour ranked above it has been left out, and left out
// as soon as one of them is taken; each round settles at least the best
// block still open, so the rounds end.  One 1024-thread workgroup, the
// candidates' state and "ranked-above" neighbour masks in LDS.
constexpr int kExCand = 24576;

// Neighbour j (0..25) of the 26-neighbourhood, the centre skipped.
__device__ inline void nb_offset(int j, int *dx, int *dy, int *dz) {
    const int i = j < 13 ? j : j + 1;
    *dx = i % 3 - 1;
    *dy = (i / 3) % 3 - 1;
    *dz = i / 9 - 1;
}

__device__ inline bool ranks_above(uint64_t ka, int64_t ia, uint64_t kb, int64_t ib) {
    return ka > kb || (ka == kb && ia < ib);
}

__global__ __launch_bounds__(1024) void k_select_ex(const uint64_t *__restrict__ keys, int64_t n,
                                                    BoxGrid G, int nx, int ny,
                                                    const uint8_t *__restrict__ mask,
                                                    int connectivity, double fraction,
                                                    int32_t *__restrict__ centers,
                                                    int64_t *__restrict__ k_out) {
    __shared__ uint8_t state[kExCand];       // 0 open, 1 taken, 2 left out, 3 outside the mask
    __shared__ uint32_t above[kExCand];      // bit j: neighbour j ranks above
    __shared__ uint32_t hist[2048];
    __shared__ int64_t s_w[16];
    __shared__ int s_changed;
    __shared__ int32_t s_off[26];  // grid-index offset of neighbour j
    __shared__ int8_t s_dir[26][4];  // the pattern's neighbours: j, dx, dy, dz
    __shared__ int s_ndir;
    __shared__ uint64_t s_prefix, s_mask;
    __shared__ int64_t s_need;
    const int tid = threadIdx.x;
    const int gx = G.g[0], gy = G.g[1], gz = G.g[2];
    // neighbours of the pattern: one, up to two, or up to three axis steps
    const int max_steps = connectivity == 6 ? 1 : (connectivity == 18 ? 2 : (connectivity == 26 ? 3 : 0));
    if (tid < 26) {
        int dx, dy, dz;
        nb_offset(tid, &dx, &dy, &dz);
        s_off[tid] = (dz * gy + dy) * gx + dx;
    }
    if (tid == 0) {  // the neighbours the pattern looks at
        int c = 0;
        for (int j = 0; j < 26; ++j) {
            int dx, dy, dz;
            nb_offset(j, &dx, &dy, &dz);
            if ((dx != 0) + (dy != 0) + (dz != 0) > max_steps) continue;
            s_dir[c][0] = (int8_t)j;
            s_dir[c][1] = (int8_t)dx;
            s_dir[c][2] = (int8_t)dy;
            s_dir[c][3] = (int8_t)dz;
            ++c;
        }
        s_ndir = c;
    }
    __syncthreads();
    const int ndir = s_ndir;
    int64_t in_local = 0;
    const int gxy = gx * gy;
    for (int g = tid; g < (int)n; g += 1024) {  // n <= kExCand: 32-bit index arithmetic
        const int iz = g / gxy, r = g - iz * gxy, iy = r / gx, ix = r - iy * gx;
        bool in = true;
        if (mask)
            in = mask[((int64_t)(iz * G.s[2] + (G.b[2] - 1) / 2) * ny +
                       (iy * G.s[1] + (G.b[1] - 1) / 2)) * nx +
                      (ix * G.s[0] + (G.b[0] - 1) / 2)] != 0;
        state[g] = in ? 0 : 3;
        in_local += in;
        uint32_t bits = 0;
        const uint64_t kg = keys[g];
        for (int t = 0; t < ndir; ++t) {
            const int x = ix + s_dir[t][1], y = iy + s_dir[t][2], z = iz + s_dir[t][3];
            if (x < 0 || y < 0 || z < 0 || x >= gx || y >= gy || z >= gz) continue;
            const int q = (z * gy + y) * gx + x;
            if (ranks_above(keys[q], q, kg, g)) bits |= 1u << s_dir[t][0];
        }
        above[g] = bits;
    }
    int64_t n_in;
    (void)wg_scan1024_ex(in_local, s_w, &n_in);
    // the count rule over the candidates inside the mask
    double kd = floor(0.5 + (double)n_in * fraction);
    const int64_t k = kd < 0 ? 0 : (kd > (double)n_in ? n_in : (int64_t)kd);
    __syncthreads();
    // greedy set by rounds (every candidate inside the mask when no pattern)
    for (;;) {
        if (tid == 0) s_changed = 0;
        __syncthreads();
        int changed = 0;
        for (int g = tid; g < (int)n; g += 1024) {  // n <= kExCand
            if (state[g] != 0) continue;
            bool any_taken = false, all_out = true;
            uint32_t bits = above[g];  // only neighbours inside the grid are flagged
            while (bits) {
                const int j = __ffs(bits) - 1;
                bits &= bits - 1;
                const uint8_t sq = state[g + s_off[j]];
                any_taken |= sq == 1;
                all_out &= sq >= 2;
            }
            if (any_taken) {
                state[g] = 2;
                changed = 1;
            } else if (all_out) {
                state[g] = 1;
                changed = 1;
            }
        }
        if (changed) s_changed = 1;
        __syncthreads();
        if (!s_changed) break;
        __syncthreads();
    }
    // the K best of the taken candidates: radix select of the K-th key among them
    int64_t t_local = 0;
    for (int64_t g = tid; g < n; g += 1024) t_local += state[g] == 1;
    int64_t n_taken;
    (void)wg_scan1024_ex(t_local, s_w, &n_taken);
    const int64_t want = k < n_taken ? k : n_taken;
    uint64_t kth = 0;
    int64_t take_eq = 0;
    const bool all = want == n_taken;  // keep every taken candidate
    if (!all) {
        if (tid == 0) {
            s_prefix = 0;
            s_mask = 0;
            s_need = want;
        }
        __syncthreads();
        for (int hi = 63; hi >= 0; hi -= 11) {
            const int shift = hi - 10 > 0 ? hi - 10 : 0, width = hi - shift + 1;
            const uint64_t dmask = (width == 64 ? ~0ull : ((1ull << width) - 1)) << shift;
            for (int i = tid; i < 2048; i += 1024) hist[i] = 0;
            __syncthreads();
            const uint64_t prefix = s_prefix, pm = s_mask;
            for (int64_t g = tid; g < n; g += 1024) {
                const uint64_t kv = keys[g];
                if (state[g] == 1 && (kv & pm) == prefix) atomicAdd(&hist[(kv & dmask) >> shift], 1u);
            }
            __syncthreads();
            const uint32_t a = hist[2047 - 2 * tid], b = hist[2046 - 2 * tid];
            int64_t tot;
            const int64_t incl = wg_scan1024_ex((int64_t)a + b, s_w, &tot);
            const int64_t above_cnt = incl - a - b, need = s_need;
            __syncthreads();
            if (above_cnt < need && need <= incl) {
                const bool first = above_cnt + a >= need;
                const uint64_t d = (uint64_t)(first ? 2047 - 2 * tid : 2046 - 2 * tid);
                s_need = need - (first ? above_cnt : above_cnt + a);
                s_prefix = prefix | (d << shift);
                s_mask = pm | dmask;
            }
            __syncthreads();
        }
        kth = s_prefix;
        take_eq = s_need;
    }
    // ordered compaction: thread t owns candidates [t*per, (t+1)*per)
    const int64_t per = (n + 1023) / 1024;
    const int64_t lo = (int64_t)tid * per < n ? (int64_t)tid * per : n, hi = lo + per < n ? lo + per : n;
    int64_t lg = 0, le = 0;
    for (int64_t g = lo; g < hi; ++g) {
        if (state[g] != 1) continue;
        const uint64_t kv = keys[g];
        lg += all || kv > kth;
        le += !all && kv == kth;
    }
    int64_t tg, te;
    int64_t gt_before = wg_scan1024_ex(lg, s_w, &tg) - lg;
    int64_t eq_before = wg_scan1024_ex(le, s_w, &te) - le;
    for (int64_t g = lo; g < hi; ++g) {
        if (state[g] != 1) continue;
        const uint64_t kv = keys[g];
        const bool is_gt = all || kv > kth, is_eq = !all && kv == kth;
        if (is_gt || (is_eq && eq_before < take_eq)) {
            const int64_t pos = gt_before + (eq_before < take_eq ? eq_before : take_eq);
            const int gi = (int)g, iz = gi / (gx * gy), r = gi - iz * gx * gy, iy = r / gx,
                      ix = r - iy * gx;
            centers[3 * pos + 0] = (int32_t)(ix * G.s[0] + (G.b[0] - 1) / 2);
            centers[3 * pos + 1] = (int32_t)(iy * G.s[1] + (G.b[1] - 1) / 2);
            centers[3 * pos + 2] = (int32_t)(iz * G.s[2] + (G.b[2] - 1) / 2);
        }
        gt_before += is_gt;
        eq_before += is_eq;
    }
    if (tid == 0) *k_out = want;
}

// ---------------------------------------------- selection variants, large grids
//
// The same greedy rank-order set on grids of any size, in rounds.  The state
// of each candidate (0 open, 1 taken, 2 left out, 3 outside the mask) and
// the mask of its pattern neighbours ranked above it live in global memory.
// A round launch gives each workgroup a tile of 8 x 8 x 8 candidates, which
// it iterates in LDS until nothing in the tile changes, reading the states
// of neighbours outside the tile from global memory (a state only ever goes
// from open to final, and a candidate is decided only from final states, so
// reading a neighbour late just delays a decision).  Each launch settles at
// least the best candidate still open, whose ranked-above neighbours are all
// final, so launches repeat until none is open.  The K best taken
// candidates then come from the multi-workgroup radix select, on keys
// remapped so that only taken candidates can be chosen (taken: key + 1, any
// other: 0; the order among taken candidates is unchanged).
constexpr int EXT = 8;  // tile edge (candidates)
enum { EX_N_IN = 0, EX_OPEN = 1, EX_TAKEN = 3, EX_WANT = 4 };  // counters (EX_OPEN: 2 slots)

struct ExDirs {
    int n;
    int8_t j[26], dx[26], dy[26], dz[26];
};

ExDirs ex_dirs(int connectivity) {
    ExDirs d{};
    const int max_steps =
        connectivity == 6 ? 1 : (connectivity == 18 ? 2 : (connectivity == 26 ? 3 : 0));
    for (int j = 0; j < 26; ++j) {
        const int i = j < 13 ? j : j + 1;
        const int dx = i % 3 - 1, dy = (i / 3) % 3 - 1, dz = i / 9 - 1;
        if ((dx != 0) + (dy != 0) + (dz != 0) > max_steps) continue;
        d.j[d.n] = (int8_t)j;
        d.dx[d.n] = (int8_t)dx;
        d.dy[d.n] = (int8_t)dy;
        d.dz[d.n] = (int8_t)dz;
        ++d.n;
    }
    return d;
}

// Adds the workgroup's total of `c` to *dst with one atomic (the per-wavefront
// atomics on one address serialise at L2 across thousands of wavefronts).
// Every thread of the 256-thread workgroup calls it.
__device__ inline void wg_count_add(unsigned long long c, int64_t *dst) {
    __shared__ unsigned long long part[4];
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd((unsigned long long *)dst, t);
    }
}

__global__ __launch_bounds__(256) void k_ex_zero(int64_t *__restrict__ ctr) {
    if (threadIdx.x < 8) ctr[threadIdx.x] = 0;
}

// States, ranked-above masks (bit t: pattern neighbour t), candidates inside
// the mask counted into ctr[EX_N_IN].
__global__ __launch_bounds__(256) void k_ex_init(const uint64_t *__restrict__ keys, BoxGrid G,
                                                 int nx, int ny, const uint8_t *__restrict__ mask,
                                                 ExDirs D, uint8_t *__restrict__ state,
                                                 uint32_t *__restrict__ above,
                                                 int64_t *__restrict__ ctr) {
    const int64_t n = (int64_t)G.g[0] * G.g[1] * G.g[2];
    unsigned long long n_in = 0;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < n; g += (int64_t)gridDim.x * 256) {
        const int64_t gxy = (int64_t)G.g[0] * G.g[1];
        const int iz = (int)(g / gxy), r = (int)(g - iz * gxy), iy = r / G.g[0],
                  ix = r - iy * G.g[0];
        bool in = true;
        if (mask)
            in = mask[((int64_t)(iz * G.s[2] + (G.b[2] - 1) / 2) * ny +
                       (iy * G.s[1] + (G.b[1] - 1) / 2)) * nx +
                      (ix * G.s[0] + (G.b[0] - 1) / 2)] != 0;
        uint32_t bits = 0;
        const uint64_t kg = keys[g];
        for (int t = 0; t < D.n; ++t) {
            const int x = ix + D.dx[t], y = iy + D.dy[t], z = iz + D.dz[t];
            if (x < 0 || y < 0 || z < 0 || x >= G.g[0] || y >= G.g[1] || z >= G.g[2]) continue;
            const int64_t q = ((int64_t)z * G.g[1] + y) * G.g[0] + x;
            if (ranks_above(keys[q], q, kg, g)) bits |= 1u << t;
        }
        state[g] = in ? 0 : 3;
        above[g] = bits;
        n_in += in;
    }
    wg_count_add(n_in, &ctr[EX_N_IN]);
}

// One round launch (see above); a workgroup with open candidates left after
// it sets ctr[EX_OPEN + parity] to 1 (the host only asks whether any are
// left), and the other parity's flag is cleared for the next launch.
__global__ __launch_bounds__(256) void k_ex_round(BoxGrid G, ExDirs D,
                                                  uint8_t *__restrict__ state,
                                                  const uint32_t *__restrict__ above, int parity,
                                                  int64_t *__restrict__ ctr) {
    constexpr int TN = EXT * EXT * EXT, PER = TN / 256;
    __shared__ uint8_t ts[TN];
    __shared__ int s_changed;
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * EXT, y0 = blockIdx.y * EXT, z0 = blockIdx.z * EXT;
    const int gx = G.g[0], gy = G.g[1], gz = G.g[2];
    if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && tid == 0)
        ctr[EX_OPEN + (parity ^ 1)] = 0;
    int64_t gi[PER];
    int lx[PER], ly[PER], lz[PER];
    bool live[PER];
    uint32_t ab[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int e = tid + 256 * p;
        lx[p] = e % EXT;
        ly[p] = (e / EXT) % EXT;
        lz[p] = e / (EXT * EXT);
        const int x = x0 + lx[p], y = y0 + ly[p], z = z0 + lz[p];
        live[p] = x < gx && y < gy && z < gz;
        gi[p] = live[p] ? ((int64_t)z * gy + y) * gx + x : 0;
        ts[e] = live[p] ? state[gi[p]] : 3;
        ab[p] = live[p] ? above[gi[p]] : 0;
    }
    __syncthreads();
    for (;;) {
        if (tid == 0) s_changed = 0;
        __syncthreads();
        int changed = 0;
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int e = tid + 256 * p;
            if (ts[e] != 0) continue;
            bool any_taken = false, all_out = true;
            uint32_t bits = ab[p];
            while (bits) {
                const int t = __ffs(bits) - 1;
                bits &= bits - 1;
                const int ax = lx[p] + D.dx[t], ay = ly[p] + D.dy[t], az = lz[p] + D.dz[t];
                uint8_t sq;
                if (ax >= 0 && ay >= 0 && az >= 0 && ax < EXT && ay < EXT && az < EXT)
                    sq = ts[(az * EXT + ay) * EXT + ax];
                else  // outside the tile (inside the grid: only those are flagged)
                    sq = state[gi[p] + ((int64_t)D.dz[t] * gy + D.dy[t]) * gx + D.dx[t]];
                any_taken |= sq == 1;
                all_out &= sq >= 2;
            }
            if (any_taken || all_out) {
                ts[e] = any_taken ? 2 : 1;
                changed = 1;
            }
        }
        if (changed) s_changed = 1;
        __syncthreads();
        if (!s_changed) break;
        __syncthreads();
    }
    bool open = false;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int e = tid + 256 * p;
        if (live[p]) state[gi[p]] = ts[e];
        open |= live[p] && ts[e] == 0;
    }
    if (__syncthreads_or(open) && tid == 0) ctr[EX_OPEN + parity] = 1;
}

// Keys remapped for the final select (taken: key + 1, other: 0) and the taken
// candidates counted into ctr[EX_TAKEN].
__global__ __launch_bounds__(256) void k_ex_count(uint64_t *__restrict__ keys, int64_t n,
                                                  const uint8_t *__restrict__ state,
                                                  int64_t *__restrict__ ctr) {
    unsigned long long taken = 0;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < n; g += (int64_t)gridDim.x * 256) {
        const bool t = state[g] == 1;
        keys[g] = t ? keys[g] + 1 : 0;
        taken += t;
    }
    wg_count_add(taken, &ctr[EX_TAKEN]);
}

// K from the count rule over the candidates inside the mask, then the number
// kept: min(K, taken).
__global__ void k_ex_want(double fraction, int64_t *__restrict__ ctr, int64_t *__restrict__ k_out) {
    if (threadIdx.x != 0) return;
    const int64_t n_in = ctr[EX_N_IN];
    const double kd = floor(0.5 + (double)n_in * fraction);
    const int64_t k = kd < 0 ? 0 : (kd > (double)n_in ? n_in : (int64_t)kd);
    const int64_t want = k < ctr[EX_TAKEN] ? k : ctr[EX_TAKEN];
    ctr[EX_WANT] = want;
    *k_out = want;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Batched selection for small candidate grids.  The keys of every set's
// candidates are computed first (grid y = set); then one workgroup per set
// selects and writes the centres in ascending grid index.  The keys, the tie
// rule and the select are the plain path's, so the same blocks come out.

// Batched selection keys, 12-bit data: one wavefront per candidate; the sums
// are exact integers, so every lane adds the voxels it loads and the
// wavefront reduces them.  Grid: (candidates / 4, sets).
__global__ __launch_bounds__(256) void k_batch_keys_u16(const uint16_t *__restrict__ vol, int nx,
                                                        int ny,
                                                        const BatchSelectSet *__restrict__ sets) {
    const BatchSelectSet &S = sets[blockIdx.y];
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= S.ncand) return;  // whole wavefront leaves together
    const int b = S.b, nb = b * b * b;
    const int ix = i % S.gx, iy = (i / S.gx) % S.gy, iz = i / (S.gx * S.gy);
    const int64_t x0 = (int64_t)ix * S.stride, y0 = (int64_t)iy * S.stride,
                  z0 = (int64_t)iz * S.stride;
    uint64_t s = 0, q = 0;
    for (int o = lane; o < nb; o += 64) {
        const int z = o / (b * b), y = (o / b) % b, x = o % b;
        const uint64_t v = vol[((z0 + z) * ny + (y0 + y)) * (int64_t)nx + x0 + x];
        s += v;
        q += v * v;
    }
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_xor(s, off);
        q += __shfl_xor(q, off);
    }
    if (lane == 0) S.keys[i] = (uint64_t)nb * q - s * s;
}

// Batched selection keys, float data: one thread per candidate, key_f32 in
// the plain selection's order (so a set's keys equal a plain call's).  Each
// lane's sums are a dependent FP64 chain of its own, so all 64 lanes work;
// neighbouring lanes read neighbouring blocks, a few lanes to a cache line.
// 64-thread workgroups spread a set's few candidates over many CUs, whose
// vector memory paths bound these loads.  Grid: (candidates / 64, sets).
__global__ __launch_bounds__(64) void k_batch_keys_f32(const float *__restrict__ vol, int nx,
                                                       int ny,
                                                       const BatchSelectSet *__restrict__ sets) {
    const BatchSelectSet &S = sets[blockIdx.y];
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i >= S.ncand) return;
    const int ix = i % S.gx, iy = (i / S.gx) % S.gy, iz = i / (S.gx * S.gy);
    S.keys[i] = key_f32(vol, nx, ny, S.b, S.b, S.b, (int64_t)ix * S.stride,
                        (int64_t)iy * S.stride, (int64_t)iz * S.stride);
}

// Per set, the plain path's one-workgroup select (radix passes for the K-th
// key, then the ordered compaction), so a set's centres are a plain call's;
// key slots for the batched grids only (at most kBatchCand candidates).
__global__ __launch_bounds__(1024) void k_select_batch(const BatchSelectSet *__restrict__ sets) {
    __shared__ ThrShared sm;
    const BatchSelectSet &S = sets[blockIdx.x];
    BoxGrid G;
    for (int a = 0; a < 3; ++a) {
        G.b[a] = S.b;
        G.s[a] = S.stride;
    }
    G.g[0] = S.gx;
    G.g[1] = S.gy;
    G.g[2] = S.gz;
    select_threshold_wg<kBatchCand / 1024>(S.keys, S.ncand, S.k, nullptr, nullptr, G, S.centers,
                                           sm);
}

}  // namespace

hipError_t launch_select_batch(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                               const BatchSelectSet *sets, int nsets, int64_t max_cand,
                               hipStream_t stream) {
    static_assert(kBatchCand % 4096 == 0, "whole select scan entries per set");
    if (max_cand > 0 && dtype == NRR_U16)
        hipLaunchKernelGGL(k_batch_keys_u16, dim3((unsigned)((max_cand + 3) / 4), (unsigned)nsets),
                           dim3(256), 0, stream, static_cast<const uint16_t *>(vol), dims[0],
                           dims[1], sets);
    else if (max_cand > 0)
        hipLaunchKernelGGL(k_batch_keys_f32, dim3((unsigned)((max_cand + 63) / 64), (unsigned)nsets),
                           dim3(64), 0, stream, static_cast<const float *>(vol), dims[0], dims[1],
                           sets);
    hipLaunchKernelGGL(k_select_batch, dim3((unsigned)nsets), dim3(1024), 0, stream, sets);
    return hipGetLastError();
}

hipError_t launch_select_ex(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                            int32_t block, int32_t stride, const int32_t grid[3], double fraction,
                            const uint8_t *mask, int32_t connectivity, int32_t *centers,
                            int64_t *k_device, void *workspace, hipStream_t stream) {
    return launch_select_ex(vol, dtype, dims, cubic_grid(block, stride, grid), fraction, mask,
                            connectivity, centers, k_device, workspace, stream);
}

hipError_t launch_select_ex(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                            const BoxGrid &G, double fraction, const uint8_t *mask,
                            int32_t connectivity, int32_t *centers, int64_t *k_device,
                            void *workspace, hipStream_t stream) {
    const int64_t n = (int64_t)G.g[0] * G.g[1] * G.g[2];
    if (n > kSelectExCand)
        return launch_select_ex_large(vol, dtype, dims, G, fraction, mask, connectivity, centers,
                                      k_device, workspace, stream);
    SelectLayout L = select_layout(n);
    uint64_t *keys = reinterpret_cast<uint64_t *>(static_cast<char *>(workspace) + L.keys_off);
    launch_keys(vol, dtype, dims, G, n, keys, stream);
    hipLaunchKernelGGL(k_select_ex, dim3(1), dim3(1024), 0, stream, keys, n, G, dims[0], dims[1],
                       mask, connectivity, fraction, centers, k_device);
    return hipGetLastError();
}

// Large grids: round launches until no candidate is open.  The host reads the
// open count after each launch (a wait on the stream), so this path does not
// return before its selection is done.
hipError_t launch_select_ex_large(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                                  const BoxGrid &G, double fraction, const uint8_t *mask,
                                  int32_t connectivity, int32_t *centers, int64_t *k_device,
                                  void *workspace, hipStream_t stream) {
    const int64_t n = (int64_t)G.g[0] * G.g[1] * G.g[2];
    const SelectLayout L = select_layout(n, true);
    char *ws = static_cast<char *>(workspace);
    uint64_t *keys = reinterpret_cast<uint64_t *>(ws + L.keys_off);
    int64_t *ctr = reinterpret_cast<int64_t *>(ws + L.ex_ctr_off);
    uint8_t *state = reinterpret_cast<uint8_t *>(ws + L.ex_state_off);
    uint32_t *above = reinterpret_cast<uint32_t *>(ws + L.ex_above_off);
    // page-locked slot for the open count, one per host thread
    thread_local int64_t *open_h = nullptr;
    if (!open_h) {
        void *p = nullptr;
        if (hipHostMalloc(&p, 64, hipHostMallocDefault) != hipSuccess) return hipErrorOutOfMemory;
        open_h = static_cast<int64_t *>(p);
    }
    const ExDirs D = ex_dirs(connectivity);
    launch_keys(vol, dtype, dims, G, n, keys, stream);
    hipLaunchKernelGGL(k_ex_zero, dim3(1), dim3(256), 0, stream, ctr);
    // element passes: at most 1024 workgroups (one counter atomic each)
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_ex_init, dim3(blocks), dim3(256), 0, stream, keys, G, dims[0], dims[1],
                       mask, D, state, above, ctr);
    const dim3 tiles((G.g[0] + EXT - 1) / EXT, (G.g[1] + EXT - 1) / EXT, (G.g[2] + EXT - 1) / EXT);
    // each launch settles at least one candidate, so n launches always end it
    for (int64_t round = 0; round < n + 1; ++round) {
        const int parity = (int)(round & 1);
        hipLaunchKernelGGL(k_ex_round, tiles, dim3(256), 0, stream, G, D, state, above, parity,
                           ctr);
        hipError_t e = hipMemcpyAsync(open_h, ctr + EX_OPEN + parity, sizeof(int64_t),
                                      hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        if (*open_h == 0) break;
    }
    hipLaunchKernelGGL(k_ex_count, dim3(blocks), dim3(256), 0, stream, keys, n, state, ctr);
    hipLaunchKernelGGL(k_ex_want, dim3(1), dim3(64), 0, stream, fraction, ctr, k_device);
    select_from_keys(keys, n, G, 0, ctr + EX_WANT, centers, L, ws, stream);
    return hipGetLastError();
}

// Ranking keys of every candidate of the grid G.
void launch_keys(const void *vol, nrr_dtype dtype, const int32_t dims[3], const BoxGrid &G,
                 int64_t n, uint64_t *keys, hipStream_t stream) {
    // overlapping candidates (stride below the edge in x or y) whose tile
    // region fits: the tiled kernel; candidates apart in x and y: by grid
    // rows; otherwise one wavefront per candidate
    const bool overlap = G.s[0] < G.b[0] || G.s[1] < G.b[1];
    const int rx = ((KT - 1) * G.s[0] + G.b[0] + 1) & ~1, ry = (KT - 1) * G.s[1] + G.b[1];
    if (dtype == NRR_U16 && overlap && rx <= KT_MAXR && ry <= KT_MAXR)
        hipLaunchKernelGGL(k_block_keys_u16_tiled,
                           dim3((unsigned)((G.g[0] + KT - 1) / KT), (unsigned)((G.g[1] + KT - 1) / KT),
                                (unsigned)G.g[2]),
                           dim3(256), (size_t)rx * ry * 2 + (size_t)ry * KT * 8, stream,
                           static_cast<const uint16_t *>(vol), dims[0], dims[1], G, keys);
    else if (dtype == NRR_U16 && !overlap && G.g[1] <= 65535 && G.g[2] <= 65535) {
        const int cx = (64 - G.b[0]) / G.s[0] + 1;  // candidates of a row per workgroup
        hipLaunchKernelGGL(k_block_keys_u16_rows,
                           dim3((unsigned)((G.g[0] + cx - 1) / cx), (unsigned)G.g[1],
                                (unsigned)G.g[2]),
                           dim3(256), 0, stream, static_cast<const uint16_t *>(vol), dims[0],
                           dims[1], G, cx, keys);
    } else if (dtype == NRR_U16)
        hipLaunchKernelGGL(k_block_keys_u16, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream,
                           static_cast<const uint16_t *>(vol), dims[0], dims[1], G, n, keys);
    else
        hipLaunchKernelGGL(k_block_keys_f32, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, stream,
                           static_cast<const float *>(vol), dims[0], dims[1], G, n, keys);
}

SelectLayout select_layout(int64_t n_candidates, bool variants) {
    SelectLayout L;
    L.n_tiles = (n_candidates + kSelectTile - 1) / kSelectTile;
    L.keys_off = 0;
    L.state_off = align_up((size_t)n_candidates * sizeof(uint64_t), 256);
    L.tiles_off = L.state_off + 256;
    L.total = L.tiles_off + align_up((size_t)L.n_tiles * 2 * sizeof(int64_t), 256);
    // the multi-workgroup radix select's histogram rows (large grids)
    L.radix_rows_off = 0;
    if (n_candidates > kRadixMultiMin) {
        L.radix_rows_off = L.total;
        L.total += (size_t)kRadixRows * 256 * 4;
    }
    // the selection variants on grids of more than kSelectExCand candidates:
    // a state byte and a ranked-above mask per candidate, four counters
    L.ex_ctr_off = L.total;
    L.ex_state_off = L.ex_ctr_off + 256;
    L.ex_above_off = L.ex_state_off + align_up((size_t)n_candidates, 256);
    if (variants && n_candidates > kSelectExCand)
        L.total = L.ex_above_off + align_up((size_t)n_candidates * 4, 256);
    return L;
}

BoxGrid cubic_grid(int32_t block, int32_t stride, const int32_t grid[3]) {
    BoxGrid G;
    for (int a = 0; a < 3; ++a) {
        G.b[a] = block;
        G.s[a] = stride;
        G.g[a] = grid[a];
    }
    return G;
}

// The K best keys' candidates (key descending, grid index ascending among
// equal keys) as centres in ascending grid index; K = k, or *kd when given.
void select_from_keys(const uint64_t *keys, int64_t n, const BoxGrid &G, int64_t k,
                      const int64_t *kd, int32_t *centers, const SelectLayout &L, char *ws,
                      hipStream_t stream) {
    SelectState *st = reinterpret_cast<SelectState *>(ws + L.state_off);
    int64_t *tiles = reinterpret_cast<int64_t *>(ws + L.tiles_off);
    if (L.radix_rows_off) {  // large grid: multi-workgroup passes
        RadixState *rs = reinterpret_cast<RadixState *>(ws + L.state_off + 64);
        uint32_t *rows = reinterpret_cast<uint32_t *>(ws + L.radix_rows_off);
        hipLaunchKernelGGL(k_radix_init, dim3(1), dim3(256), 0, stream, k, kd, rs, rows);
        for (int shift = 56; shift >= 0; shift -= 8) {
            hipLaunchKernelGGL(k_radix_hist, dim3(kRadixWG), dim3(256), 0, stream, keys, n, rs,
                               shift, rows);
            hipLaunchKernelGGL(k_radix_pick, dim3(1), dim3(256), 0, stream, rows, kRadixRows,
                               shift, rs, st);
        }
        hipLaunchKernelGGL(k_tile_counts, dim3((unsigned)L.n_tiles), dim3(256), 0, stream, keys,
                           n, st, tiles);
        hipLaunchKernelGGL(k_compact, dim3((unsigned)L.n_tiles), dim3(256), 0, stream, keys, n,
                           st, tiles, G, k, kd, centers);
    } else if (n <= kSmallSelect) {  // one workgroup, few key slots (less work per pass)
        hipLaunchKernelGGL(k_select_threshold<kSmallSelect / 1024>, dim3(1), dim3(1024), 0, stream,
                           keys, n, k, kd, st, G, centers);
    } else {  // one workgroup: the K-th key and the compaction
        hipLaunchKernelGGL(k_select_threshold<kThrKeys>, dim3(1), dim3(1024), 0, stream, keys, n,
                           k, kd, st, G, centers);
    }
}

bool select_stats_fusable(nrr_dtype dtype, int64_t n, int64_t k, int32_t block) {
    return dtype == NRR_U16 && k > 0 && n <= kRadixMultiMin && block >= 1 && block <= 9 &&
           (block & 1);
}

hipError_t launch_select_stats(const uint64_t *keys, int64_t n, const BoxGrid &G, int64_t k,
                               int32_t *centers, const SelectLayout &SL, char *sws,
                               const uint16_t *flt, const int32_t dims[3], int32_t block,
                               const StatsLayout &L, void *stats, hipStream_t stream) {
    SelectState *st = reinterpret_cast<SelectState *>(sws + SL.state_off);
    // one workgroup (16 wavefronts) per CU holds the launch: z-runs cut so
    // the statistics fill the CUs beside the select's once, not 1.x rounds
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const ColsGrid cg = cols_grid(L, block, 16 * (int64_t)std::max(ncu - 1, 1));
    const int64_t nwaves = cg.nwx * cg.nwy * cg.runs;
    const dim3 grid((unsigned)(1 + (nwaves + 15) / 16));
    StatU16 *out = static_cast<StatU16 *>(stats);
    switch (block) {
#define NRR_SELECT_STATS(B)                                                                      \
    case B:                                                                                      \
        hipLaunchKernelGGL(k_select_stats<B>, grid, dim3(1024), 0, stream, keys, n, k, st, G,    \
                           centers, flt, dims[0], dims[1], dims[2], L.ox, L.oy, L.oz, cg.zc,     \
                           (int)cg.nwx, (int)cg.nwy, nwaves, out);                               \
        break;
        NRR_SELECT_STATS(1)
        NRR_SELECT_STATS(3)
        NRR_SELECT_STATS(5)
        NRR_SELECT_STATS(7)
        NRR_SELECT_STATS(9)
#undef NRR_SELECT_STATS
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_select(const void *vol, nrr_dtype dtype, const int32_t dims[3],
                         const BoxGrid &G, int64_t k, int32_t *centers, void *workspace,
                         hipStream_t stream) {
    const int64_t n = (int64_t)G.g[0] * G.g[1] * G.g[2];
    SelectLayout L = select_layout(n);
    char *ws = static_cast<char *>(workspace);
    uint64_t *keys = reinterpret_cast<uint64_t *>(ws + L.keys_off);
    launch_keys(vol, dtype, dims, G, n, keys, stream);
    select_from_keys(keys, n, G, k, nullptr, centers, L, ws, stream);
    return hipGetLastError();
}

hipError_t launch_select(const void *vol, nrr_dtype dtype, const int32_t dims[3], int32_t block,
                         int32_t stride, const int32_t grid[3], int64_t k, int32_t *centers,
                         void *workspace, hipStream_t stream) {
    return launch_select(vol, dtype, dims, cubic_grid(block, stride, grid), k, centers, workspace,
                         stream);
}

}  // namespace nrr
