// Per-voxel statistics of every block (bx x by x bz, cubic for the plain
// search) of the intra-operative volume.
//
// The NCC of the paper's similarity equation needs, for each displaced block
// F, its mean and its spread sum (F - Fbar)^2.  Those depend only on the
// block's position, not on which pre-operative block is being matched, so
// they are computed once per call for every possible block origin (a 3-D box
// filter of F and F^2) instead of once per (block, displacement) pair.
//
//   u16: s = sum (F - 2048) exact in int32, q = sum (F - 2048)^2 exact in
//        uint64, r = 1/sqrt(N q - s^2) as float (0 when the block is flat,
//        i.e. N q == s^2 exactly).
//   f32: s = sum F, q = sum F^2 in FP64, r = 1/sqrt(N q - s^2) in FP64;
//        the block counts as flat when N q - s^2 <= 1e-12 * N q (FP64 cannot
//        resolve a smaller relative spread from these sums).
//
// Layout of the outputs: dense [Oz][Oy][Ox] with O = dims - block + 1 (index =
// lowest corner of the block).
//
// 12-bit data, by voxel columns: a wavefront owns 64 consecutive voxel
// columns (x) over the rows of 8 origin rows (y) and slides along a run of
// origin planes.  Each lane keeps, per row, the sums over the block's current
// bz planes of F - 2048 and of its square (exact integers: each step adds the
// plane entering and subtracts the plane leaving, read again), forms the
// by-row sums in registers and the bx-column sums across lanes through LDS.
// Wavefronts share no data, so the kernel has no barrier.  The plane-pair
// volume that the search reads is written by a separate pass.
//
// Float data, by tiles: a workgroup owns a 64 x 4 tile of (x, y) origins and
// a run of zc origin planes; each input plane is staged in LDS (fetched two
// planes ahead) and summed along x (sliding windows over 4-wide segments)
// then along y; the per-plane sums of the last bz planes sit in a small LDS
// ring and the block sums are re-added from it (no rounding drifts along
// the volume).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "nrr_internal.h"
#include "stats_cols.h"

namespace nrr {
namespace {

constexpr int TX = 64, TY = 4, ZC = 32, MAXB = 15, SEG = 4;  // ZC: most origin planes per run
constexpr int PW = TX + MAXB - 1, PH = TY + MAXB - 1;
constexpr int PATCH = PH * PW;
constexpr int PER = (PATCH + 255) / 256;  // patch elements staged per thread

// Workgroup barrier for LDS traffic only.  __syncthreads also orders global
// memory, which on this architecture means waiting for every load in flight
// (loads and stores share one counter), including the planes fetched ahead;
// this kernel's global stores are read by no other thread of the launch.
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Body of the float statistics kernel.  V: staged voxel type, A/AQ: row and
// plane sums of F and F^2, AS/AQQ: block sums, re-added from the ring of the
// last bz plane sums.  Global loads run two planes ahead of the plane being
// summed.
template <typename V, typename A, typename AQ, typename AS, typename AQQ, typename Src,
          typename Conv, typename Emit>
__device__ inline void stats_body(const Src *__restrict__ flt, int nx, int ny, int nz, int bx,
                                  int by, int bz, int ox, int oy, int oz, int zc, int tile_x,
                                  int tile_y, int run, V *patch /*[2][PATCH]*/, A *rs, AQ *rq,
                                  A *ringP, AQ *ringQ, Conv conv, Emit emit) {
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;  // output (tx, ty)
    const int x0 = tile_x * TX, y0 = tile_y * TY, z0 = run * zc;
    const int ph = TY + by - 1, pw = TX + bx - 1;
    const int zend = min(z0 + zc + bz - 1, nz);  // input planes [z0, zend)
    // this thread's patch elements: fixed offsets inside a plane
    int goff[PER];
    bool gok[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = tid + 256 * k, r = e / pw, c = e - r * pw;
        gok[k] = e < ph * pw && x0 + c < nx && y0 + r < ny;
        goff[k] = r * nx + c;
    }
    const int64_t pstride = (int64_t)ny * nx;
    const Src *pbase = flt + (int64_t)y0 * nx + x0;
    // Loads are issued unconditionally (elements outside the volume or past
    // the run read the tile's first voxel of a plane inside the volume) and
    // kept raw; the mask and the conversion are applied when the values go
    // to LDS a plane later, so no wait follows a load in the step it is
    // issued in.
    struct Raw {
        Src v[PER];
        uint32_t ok;  // bit k: element k is inside the volume and the run
    };
    auto fetch = [&](Raw &r, int zi) {
        const Src *pl = pbase + (int64_t)min(zi, nz - 1) * pstride;
        r.ok = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const bool ok = gok[k] && zi < zend;
            r.ok |= (uint32_t)ok << k;
            r.v[k] = pl[ok ? goff[k] : 0];
        }
    };
    auto value = [&](const Raw &r, int k) { return ((r.ok >> k) & 1) ? conv(r.v[k]) : V(0); };
    Raw r1, r2;
    fetch(r1, z0);
#pragma unroll
    for (int k = 0; k < PER; ++k) patch[tid + 256 * k] = value(r1, k);
    fetch(r1, z0 + 1);
    lds_barrier();
    const int nseg = ph * (TX / SEG);
    // one plane step; rn holds plane zi + 1 (fetched a step earlier), rf
    // receives plane zi + 2.  The loop runs two steps per iteration with the
    // buffers' roles swapped, so no register copy waits on a load in flight.
    auto step = [&](int zi, Raw &rn, Raw &rf) {
        const int cur = (zi - z0) & 1;
        const V *pc = patch + cur * PATCH;
        fetch(rf, zi + 2);
        // sums along x: SEG outputs per segment by a sliding window
        for (int sg = tid; sg < nseg; sg += 256) {
            const int r = sg / (TX / SEG), xs = (sg % (TX / SEG)) * SEG;
            const V *row = pc + r * pw + xs;
            A sv = 0;
            AQ qv = 0;
            for (int k = 0; k < bx; ++k) {
                const A v = (A)row[k];
                sv += v;
                qv += (AQ)(v * v);
            }
            rs[r * TX + xs] = sv;
            rq[r * TX + xs] = qv;
#pragma unroll
            for (int u = 1; u < SEG; ++u) {
                const A vin = (A)row[u + bx - 1], vout = (A)row[u - 1];
                sv += vin - vout;
                qv += (AQ)(vin * vin) - (AQ)(vout * vout);
                rs[r * TX + xs + u] = sv;
                rq[r * TX + xs + u] = qv;
            }
        }
        lds_barrier();
        A P = 0;  // then along y
        AQ Q = 0;
        for (int k = 0; k < by; ++k) {
            P += rs[(ty + k) * TX + tx];
            Q += rq[(ty + k) * TX + tx];
        }
        const int slot = (zi - z0) % bz;
        ringP[slot * 256 + tid] = P;
        ringQ[slot * 256 + tid] = Q;
        if (zi - z0 >= bz - 1) {  // the last bz plane sums give the block sums
            const int z = zi - bz + 1, x = x0 + tx, y = y0 + ty;
            if (x < ox && y < oy && z < oz) {
                AS sb = 0;
                AQQ qb = 0;
                for (int k = 0; k < bz; ++k) {
                    sb += (AS)ringP[k * 256 + tid];
                    qb += (AQQ)ringQ[k * 256 + tid];
                }
                emit(((int64_t)z * oy + y) * ox + x, sb, qb);
            }
        }
        V *pn = patch + (cur ^ 1) * PATCH;
#pragma unroll
        for (int k = 0; k < PER; ++k) pn[tid + 256 * k] = value(rn, k);
        lds_barrier();
    };
    for (int zi = z0; zi < zend; zi += 2) {
        step(zi, r1, r2);
        if (zi + 1 < zend) step(zi + 1, r2, r1);
    }
}

// 12-bit statistics by voxel columns (see the top of the file): four
// independent wavefronts per workgroup.
template <int BY, int BC>
__global__ __launch_bounds__(256) void k_stats_u16(const uint16_t *__restrict__ flt, int nx,
                                                   int ny, int nz, int bx_rt, int bz_rt, int ox,
                                                   int oy, int oz, int zc,
                                                   StatU16 *__restrict__ out) {
    __shared__ uint2 xch[4][SC_RY][SC_LW];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    stats_cols_wave<BY, BC>(flt, nx, ny, nz, bx_rt, bz_rt, ox, oy, oz, zc, out, blockIdx.x,
                            blockIdx.y * 4 + w, blockIdx.z, xch[w]);
}

__global__ __launch_bounds__(256) void k_stats_f32(const float *__restrict__ flt, int nx, int ny,
                                                   int nz, int bx, int by, int bz, int ox, int oy,
                                                   int oz, int zc, StatF32 *__restrict__ out) {
    __shared__ float patch[2 * PATCH + 256];
    __shared__ double rs[PH * TX];
    __shared__ double rq[PH * TX];
    extern __shared__ __align__(16) unsigned char dyn_f32[];
    double *ringP = reinterpret_cast<double *>(dyn_f32);
    double *ringQ = reinterpret_cast<double *>(dyn_f32 + (size_t)bz * 256 * 8);
    const double n = (double)bx * by * bz;
    stats_body<float, double, double, double, double>(
        flt, nx, ny, nz, bx, by, bz, ox, oy, oz, zc, blockIdx.x, blockIdx.y, blockIdx.z, patch, rs,
        rq, ringP, ringQ, [](float v) { return v; },
        [&](int64_t o, double S, double QQ) {
            const double nq = n * QQ;
            const double var = nq - S * S;
            StatF32 rec;
            rec.s = S;
            rec.r = var > 1e-12 * nq ? 1.0 / sqrt(var) : 0.0;
            out[o] = rec;
        });
}

// One cubic block edge's share of a several-edge float statistics launch.
struct StatsF32Job {
    int b, ox, oy, oz, zc;
    int tiles_x, tiles_y, z_first;  // its tiles, and its first grid z (its runs follow)
    StatF32 *out;
};
struct StatsF32Jobs {
    StatsF32Job job[kStatsJobs];
    int n;
};

// Float statistics of several block edges over one volume in one launch:
// grid z holds each edge's runs in turn, and a workgroup past its edge's x
// or y tiles leaves at once.  The same body and records as k_stats_f32.
__global__ __launch_bounds__(256) void k_stats_f32_multi(const float *__restrict__ flt, int nx,
                                                         int ny, int nz, StatsF32Jobs J) {
    __shared__ float patch[2 * PATCH + 256];
    __shared__ double rs[PH * TX];
    __shared__ double rq[PH * TX];
    extern __shared__ __align__(16) unsigned char dyn_f32m[];
    StatsF32Job jb = J.job[0];
#pragma unroll
    for (int i = 1; i < kStatsJobs; ++i)  // constant indices: the table stays in kernel arguments
        if (i < J.n && (int)blockIdx.z >= J.job[i].z_first) jb = J.job[i];
    if ((int)blockIdx.x >= jb.tiles_x || (int)blockIdx.y >= jb.tiles_y) return;
    double *ringP = reinterpret_cast<double *>(dyn_f32m);
    double *ringQ = reinterpret_cast<double *>(dyn_f32m + (size_t)jb.b * 256 * 8);
    const double n = (double)jb.b * jb.b * jb.b;
    StatF32 *out = jb.out;
    stats_body<float, double, double, double, double>(
        flt, nx, ny, nz, jb.b, jb.b, jb.b, jb.ox, jb.oy, jb.oz, jb.zc, blockIdx.x, blockIdx.y,
        (int)blockIdx.z - jb.z_first, patch, rs, rq, ringP, ringQ, [](float v) { return v; },
        [&](int64_t o, double S, double QQ) {
            const double nq = n * QQ;
            const double var = nq - S * S;
            StatF32 rec;
            rec.s = S;
            rec.r = var > 1e-12 * nq ? 1.0 / sqrt(var) : 0.0;
            out[o] = rec;
        });
}

// Plane-pair copy of a 12-bit volume: one 4-byte word per voxel holding the
// voxel and the one a plane above, both offset by -2048 into int16 (the next
// plane's half is 0 on the last plane).  Four consecutive voxels per thread.
__global__ __launch_bounds__(256) void k_pair_volume(const uint16_t *__restrict__ flt,
                                                     int64_t nvox, int64_t pstride,
                                                     uint32_t *__restrict__ out) {
    const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (i >= nvox) return;
    auto word = [&](int64_t j) {
        const uint32_t lo = (uint16_t)((int)flt[j] - 2048);
        const uint32_t hi = j + pstride < nvox ? (uint16_t)((int)flt[j + pstride] - 2048) : 0u;
        return lo | hi << 16;
    };
    if (i + 4 <= nvox) {
        uint4 w;
        w.x = word(i);
        w.y = word(i + 1);
        w.z = word(i + 2);
        w.w = word(i + 3);
        *reinterpret_cast<uint4 *>(out + i) = w;
    } else {
        for (int64_t j = i; j < nvox; ++j) out[j] = word(j);
    }
}

// Directional confidence (the FEM update's confidence matrix S, no formula in
// the paper): S = conf * J / trace(J) with J the block's intensity structure
// tensor, sum over its voxels of g g^T, g by central differences of `ref`
// (one-sided on the volume's border planes).  One wavefront per block, FP64
// sums (exact for 12-bit data), S as (xx, yy, zz, xy, xz, yz).
template <typename Vox>
__global__ __launch_bounds__(256) void k_structure_conf(const Vox *__restrict__ ref, int nx, int ny,
                                                        int nz, const int32_t *__restrict__ centers,
                                                        int64_t n, int b,
                                                        const float *__restrict__ conf,
                                                        float *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= n) return;  // whole wavefront leaves together
    const int h = (b - 1) / 2;
    const int cx = centers[3 * k], cy = centers[3 * k + 1], cz = centers[3 * k + 2];
    const bool inside = cx - h >= 0 && cy - h >= 0 && cz - h >= 0 && cx + h < nx && cy + h < ny &&
                        cz + h < nz;
    double j[6] = {0, 0, 0, 0, 0, 0};
    if (inside) {
        const int64_t sy = nx, sz = (int64_t)nx * ny;
        auto at = [&](int x, int y, int z) {
            return (double)ref[(int64_t)z * sz + (int64_t)y * sy + x];
        };
        auto diff = [&](int x, int y, int z, int dx, int dy, int dz, int p, int len) {
            if (len == 1) return 0.0;
            if (p == 0) return at(x + dx, y + dy, z + dz) - at(x, y, z);
            if (p == len - 1) return at(x, y, z) - at(x - dx, y - dy, z - dz);
            return 0.5 * (at(x + dx, y + dy, z + dz) - at(x - dx, y - dy, z - dz));
        };
        const int nb = b * b * b;
        for (int o = lane; o < nb; o += 64) {
            const int x = cx - h + o % b, y = cy - h + (o / b) % b, z = cz - h + o / (b * b);
            const double gx = diff(x, y, z, 1, 0, 0, x, nx);
            const double gy = diff(x, y, z, 0, 1, 0, y, ny);
            const double gz = diff(x, y, z, 0, 0, 1, z, nz);
            j[0] += gx * gx;
            j[1] += gy * gy;
            j[2] += gz * gz;
            j[3] += gx * gy;
            j[4] += gx * gz;
            j[5] += gy * gz;
        }
    }
#pragma unroll
    for (int e = 0; e < 6; ++e)
        for (int off = 32; off > 0; off >>= 1) j[e] += __shfl_xor(j[e], off);
    if (lane < 6) {
        const double tr = j[0] + j[1] + j[2];
        double v = 0.0;
#pragma unroll
        for (int e = 0; e < 6; ++e)
            if (e == lane) v = j[e];
        out[6 * k + lane] = tr > 0.0 ? (float)((double)conf[k] * v / tr) : 0.0f;
    }
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

hipError_t launch_structure_conf(const void *ref, nrr_dtype dtype, const int32_t dims[3],
                                 const int32_t *centers, int64_t n, int32_t block,
                                 const float *conf, float *out, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 3) / 4));
    if (dtype == NRR_U16)
        hipLaunchKernelGGL(k_structure_conf<uint16_t>, grid, dim3(256), 0, stream,
                           static_cast<const uint16_t *>(ref), dims[0], dims[1], dims[2], centers,
                           n, block, conf, out);
    else
        hipLaunchKernelGGL(k_structure_conf<float>, grid, dim3(256), 0, stream,
                           static_cast<const float *>(ref), dims[0], dims[1], dims[2], centers, n,
                           block, conf, out);
    return hipGetLastError();
}

StatsLayout stats_layout(nrr_dtype dtype, const int32_t dims[3], const int32_t block[3],
                         bool pairs) {
    StatsLayout L;
    L.ox = dims[0] - block[0] + 1;
    L.oy = dims[1] - block[1] + 1;
    L.oz = dims[2] - block[2] + 1;
    // slack after the table: the search reads whole tiles of records, up to
    // kTileSlack rows and columns past the last valid origin
    const size_t nvox = (size_t)L.ox * L.oy * L.oz + (size_t)kTileSlack * (L.ox + 1);
    L.total = align_up(nvox * (dtype == NRR_U16 ? sizeof(StatU16) : sizeof(StatF32)), 256);
    L.pair_off = 0;
    if (pairs && dtype == NRR_U16) {  // + slack: staging reads whole 4-word row chunks
        L.pair_off = L.total;
        L.total += align_up(((size_t)dims[0] * dims[1] * dims[2] + 64) * 4, 256);
    }
    return L;
}

StatsLayout stats_layout(nrr_dtype dtype, const int32_t dims[3], int32_t block) {
    const int32_t b3[3] = {block, block, block};
    return stats_layout(dtype, dims, b3, true);
}

namespace {
// Origin planes per float statistics workgroup: ZC, fewer when that leaves
// the device with too few workgroups (small volumes), never below 4; then
// the same number of runs, of balanced lengths (a workgroup's time is its
// run plus bz - 1 planes: 256x256x124 at b = 7 takes 30+30+30+28 instead of
// 32+32+32+22).
int f32_run_planes(const StatsLayout &L) {
    const int64_t per_slab = (int64_t)((L.ox + TX - 1) / TX) * ((L.oy + TY - 1) / TY);
    const int64_t slabs = (512 + per_slab - 1) / per_slab;
    int zc = (int)((L.oz + slabs - 1) / slabs);
    zc = zc < 4 ? 4 : (zc > ZC ? ZC : zc);
    const int runs = (L.oz + zc - 1) / zc;
    return (L.oz + runs - 1) / runs;
}
}  // namespace

hipError_t launch_stats(const void *flt, nrr_dtype dtype, const int32_t dims[3],
                        const int32_t block[3], bool pairs, void *workspace, hipStream_t stream) {
    StatsLayout L = stats_layout(dtype, dims, block, pairs);
    char *ws = static_cast<char *>(workspace);
    const int bx = block[0], by = block[1], bz = block[2];
    if (dtype == NRR_U16) {
        const ColsGrid cg = cols_grid(L, bx);
        const int zc = cg.zc;
        const dim3 grid((unsigned)cg.nwx, (unsigned)((cg.nwy + 3) / 4), (unsigned)cg.runs);
        StatU16 *out = reinterpret_cast<StatU16 *>(ws);
        const uint16_t *f = static_cast<const uint16_t *>(flt);
        switch (by) {
#define NRR_STATS_BY(BY)                                                                         \
    case BY:                                                                                     \
        if (bx == BY && bz == BY)                                                                \
            hipLaunchKernelGGL((k_stats_u16<BY, BY>), grid, dim3(256), 0, stream, f, dims[0],    \
                               dims[1], dims[2], bx, bz, L.ox, L.oy, L.oz, zc, out);             \
        else                                                                                     \
            hipLaunchKernelGGL((k_stats_u16<BY, 0>), grid, dim3(256), 0, stream, f, dims[0],     \
                               dims[1], dims[2], bx, bz, L.ox, L.oy, L.oz, zc, out);             \
        break;
            NRR_STATS_BY(1)
            NRR_STATS_BY(3)
            NRR_STATS_BY(5)
            NRR_STATS_BY(7)
            NRR_STATS_BY(9)
            NRR_STATS_BY(11)
            NRR_STATS_BY(13)
            NRR_STATS_BY(15)
#undef NRR_STATS_BY
        default:
            return hipErrorInvalidValue;  // block edges are odd, 1 .. 15
        }
        if (L.pair_off) {
            const int64_t nvox = (int64_t)dims[0] * dims[1] * dims[2];
            hipLaunchKernelGGL(k_pair_volume, dim3((unsigned)((nvox + 1023) / 1024)), dim3(256), 0,
                               stream, f, nvox, (int64_t)dims[0] * dims[1],
                               reinterpret_cast<uint32_t *>(ws + L.pair_off));
        }
        return hipGetLastError();
    }
    const int zc = f32_run_planes(L);
    dim3 grid((L.ox + TX - 1) / TX, (L.oy + TY - 1) / TY, (L.oz + zc - 1) / zc);
    hipLaunchKernelGGL(k_stats_f32, grid, dim3(256), (size_t)bz * 256 * 16, stream,
                       static_cast<const float *>(flt), dims[0], dims[1], dims[2], bx, by, bz,
                       L.ox, L.oy, L.oz, zc, reinterpret_cast<StatF32 *>(ws));
    return hipGetLastError();
}

// Voxels outside the dtype's contract (12-bit data above 4095, float data
// not finite), counted into *bad.
__global__ __launch_bounds__(256) void k_check_u16(const uint16_t *__restrict__ v, int64_t n,
                                                   unsigned long long *__restrict__ bad) {
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        c += v[i] > 4095;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(bad, c);
}

__global__ __launch_bounds__(256) void k_check_f32(const float *__restrict__ v, int64_t n,
                                                   unsigned long long *__restrict__ bad) {
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        c += !isfinite(v[i]);
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(bad, c);
}

__global__ void k_zero_u64(unsigned long long *p) {
    if (threadIdx.x == 0) *p = 0;
}

hipError_t launch_check_volume(const void *vol, nrr_dtype dtype, int64_t n, int64_t *bad,
                               hipStream_t stream) {
    unsigned long long *b = reinterpret_cast<unsigned long long *>(bad);
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, stream, b);
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    if (n > 0) {
        if (dtype == NRR_U16)
            hipLaunchKernelGGL(k_check_u16, dim3(blocks), dim3(256), 0, stream,
                               static_cast<const uint16_t *>(vol), n, b);
        else
            hipLaunchKernelGGL(k_check_f32, dim3(blocks), dim3(256), 0, stream,
                               static_cast<const float *>(vol), n, b);
    }
    return hipGetLastError();
}

hipError_t launch_pair_volume(const uint16_t *flt, const int32_t dims[3], uint32_t *pairs,
                              hipStream_t stream) {
    const int64_t nvox = (int64_t)dims[0] * dims[1] * dims[2];
    hipLaunchKernelGGL(k_pair_volume, dim3((unsigned)((nvox + 1023) / 1024)), dim3(256), 0, stream,
                       flt, nvox, (int64_t)dims[0] * dims[1], pairs);
    return hipGetLastError();
}

hipError_t launch_stats(const void *flt, nrr_dtype dtype, const int32_t dims[3], int32_t block,
                        void *workspace, hipStream_t stream) {
    const int32_t b3[3] = {block, block, block};
    return launch_stats(flt, dtype, dims, b3, true, workspace, stream);
}

hipError_t launch_stats_f32_multi(const float *flt, const int32_t dims[3], const int32_t *blocks,
                                  void *const *outs, int n, hipStream_t stream) {
    if (n < 1 || n > kStatsJobs) return hipErrorInvalidValue;
    StatsF32Jobs J{};
    J.n = n;
    int gx = 0, gy = 0, gz = 0, maxb = 0;
    for (int i = 0; i < n; ++i) {
        if (blocks[i] < 1 || blocks[i] > MAXB) return hipErrorInvalidValue;
        const int32_t b3[3] = {blocks[i], blocks[i], blocks[i]};
        const StatsLayout L = stats_layout(NRR_F32, dims, b3, false);
        StatsF32Job &j = J.job[i];
        j.b = blocks[i];
        j.ox = L.ox;
        j.oy = L.oy;
        j.oz = L.oz;
        j.zc = f32_run_planes(L);
        j.tiles_x = (L.ox + TX - 1) / TX;
        j.tiles_y = (L.oy + TY - 1) / TY;
        j.z_first = gz;
        gz += (L.oz + j.zc - 1) / j.zc;
        j.out = static_cast<StatF32 *>(outs[i]);
        gx = std::max(gx, j.tiles_x);
        gy = std::max(gy, j.tiles_y);
        maxb = std::max(maxb, (int)blocks[i]);
    }
    hipLaunchKernelGGL(k_stats_f32_multi, dim3((unsigned)gx, (unsigned)gy, (unsigned)gz), dim3(256),
                       (size_t)maxb * 256 * 16, stream, flt, dims[0], dims[1], dims[2], J);
    return hipGetLastError();
}

}  // namespace nrr
