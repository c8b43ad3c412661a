// Per-voxel statistics of every b^3 block of the intra-operative volume.
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
// Layout of the outputs: dense [Oz][Oy][Ox] with O = dims - b + 1 (index =
// lowest corner of the block).  Work decomposition: a workgroup owns a
// 64 x 4 tile of (x, y) origins and a run of ZC origin planes; each input
// plane is staged in LDS, summed along x then y (separable box sums), and the
// per-plane sums of the last b planes are kept in a small LDS ring per thread
// so the z sum is b adds.  The next plane's patch is fetched into registers
// while the current one is summed (double-buffered LDS patch).
#include <hip/hip_runtime.h>

#include "nrr_internal.h"

namespace nrr {
namespace {

constexpr int TX = 64, TY = 4, ZC = 32, MAXB = 15;
constexpr int PW = TX + MAXB - 1, PH = TY + MAXB - 1;
constexpr int PATCH = PH * PW;
constexpr int PER = (PATCH + 255) / 256;  // patch elements staged per thread

// One input plane of the tile's patch: thread-owned elements e = tid + 256*k.
template <typename V, typename Src, typename Conv>
__device__ inline void load_plane(V (&reg)[PER], const Src *__restrict__ flt, int nx, int ny,
                                  int zi, int x0, int y0, int ph, int pw, Conv conv) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = (int)threadIdx.x + 256 * k;
        const int r = e / pw, c = e - r * pw;
        const int x = x0 + c, y = y0 + r;
        reg[k] = (e < ph * pw && x < nx && y < ny) ? conv(flt[((int64_t)zi * ny + y) * nx + x]) : V(0);
    }
}

// Shared body of the two statistics kernels.  V: staged voxel type, A: plane
// sum type, AQ: plane sum-of-squares type, AS/AQQ: block sum types.
template <typename V, typename A, typename AQ, typename AS, typename AQQ, typename Src,
          typename Conv, typename Emit>
__device__ inline void stats_body(const Src *__restrict__ flt, int nx, int ny, int nz, int b,
                                  int ox, int oy, int oz, V *patch /*[2][PATCH]*/, A *xs, AQ *xq,
                                  A *ringP, AQ *ringQ, Conv conv, Emit emit) {
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * ZC;
    const int ph = TY + b - 1, pw = TX + b - 1;
    const int zend = min(z0 + ZC + b - 1, nz);  // input planes [z0, zend)
    V reg[PER];
    load_plane(reg, flt, nx, ny, z0, x0, y0, ph, pw, conv);
#pragma unroll
    for (int k = 0; k < PER; ++k) patch[tid + 256 * k] = reg[k];
    __syncthreads();
    for (int zi = z0; zi < zend; ++zi) {
        const int cur = (zi - z0) & 1;
        const V *pc = patch + cur * PATCH;
        if (zi + 1 < zend) load_plane(reg, flt, nx, ny, zi + 1, x0, y0, ph, pw, conv);
        for (int r = ty; r < ph; r += TY) {  // sums along x of each patch row
            A sv = 0;
            AQ qv = 0;
            for (int k = 0; k < b; ++k) {
                const A v = (A)pc[r * pw + tx + k];
                sv += v;
                qv += (AQ)(v * v);
            }
            xs[r * TX + tx] = sv;
            xq[r * TX + tx] = qv;
        }
        __syncthreads();
        A P = 0;
        AQ Q = 0;
        for (int k = 0; k < b; ++k) {  // then along y
            P += xs[(ty + k) * TX + tx];
            Q += xq[(ty + k) * TX + tx];
        }
        const int slot = (zi - z0) % b;
        ringP[slot * 256 + tid] = P;
        ringQ[slot * 256 + tid] = Q;
        if (zi - z0 >= b - 1) {  // the last b plane sums give the block sums
            const int z = zi - b + 1, x = x0 + tx, y = y0 + ty;
            if (x < ox && y < oy && z < oz) {
                AS S = 0;
                AQQ QQ = 0;
                for (int k = 0; k < b; ++k) {
                    S += (AS)ringP[k * 256 + tid];
                    QQ += (AQQ)ringQ[k * 256 + tid];
                }
                emit(((int64_t)z * oy + y) * ox + x, S, QQ);
            }
        }
        if (zi + 1 < zend) {
            V *pn = patch + (cur ^ 1) * PATCH;
#pragma unroll
            for (int k = 0; k < PER; ++k) pn[tid + 256 * k] = reg[k];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_stats_u16(const uint16_t *__restrict__ flt, int nx,
                                                   int ny, int nz, int b, int ox, int oy, int oz,
                                                   int32_t *__restrict__ s_out,
                                                   float *__restrict__ r_out) {
    __shared__ int32_t patch[2 * PATCH + 256];
    __shared__ int32_t xs[PH * TX];
    __shared__ uint32_t xq[PH * TX];
    // ring of the last b per-plane sums, [b][256] each (dynamic LDS)
    extern __shared__ __align__(16) unsigned char dyn_u16[];
    int32_t *ringP = reinterpret_cast<int32_t *>(dyn_u16);
    uint32_t *ringQ = reinterpret_cast<uint32_t *>(dyn_u16 + (size_t)b * 256 * 4);
    const int64_t n = (int64_t)b * b * b;
    stats_body<int32_t, int32_t, uint32_t, int32_t, uint64_t>(
        flt, nx, ny, nz, b, ox, oy, oz, patch, xs, xq, ringP, ringQ,
        [](uint16_t v) { return (int32_t)v - 2048; },
        [&](int64_t o, int32_t S, uint64_t QQ) {
            const int64_t var = n * (int64_t)QQ - (int64_t)S * S;
            s_out[o] = S;
            r_out[o] = var > 0 ? (float)(1.0 / sqrt((double)var)) : 0.0f;
        });
}

__global__ __launch_bounds__(256) void k_stats_f32(const float *__restrict__ flt, int nx, int ny,
                                                   int nz, int b, int ox, int oy, int oz,
                                                   double *__restrict__ s_out,
                                                   double *__restrict__ r_out) {
    __shared__ float patch[2 * PATCH + 256];
    __shared__ double xs[PH * TX];
    __shared__ double xq[PH * TX];
    extern __shared__ __align__(16) unsigned char dyn_f32[];
    double *ringP = reinterpret_cast<double *>(dyn_f32);
    double *ringQ = reinterpret_cast<double *>(dyn_f32 + (size_t)b * 256 * 8);
    const double n = (double)b * b * b;
    stats_body<float, double, double, double, double>(
        flt, nx, ny, nz, b, ox, oy, oz, patch, xs, xq, ringP, ringQ, [](float v) { return v; },
        [&](int64_t o, double S, double QQ) {
            const double nq = n * QQ;
            const double var = nq - S * S;
            s_out[o] = S;
            r_out[o] = var > 1e-12 * nq ? 1.0 / sqrt(var) : 0.0;
        });
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

StatsLayout stats_layout(nrr_dtype dtype, const int32_t dims[3], int32_t block) {
    StatsLayout L;
    L.ox = dims[0] - block + 1;
    L.oy = dims[1] - block + 1;
    L.oz = dims[2] - block + 1;
    size_t nvox = (size_t)L.ox * L.oy * L.oz;
    size_t es = dtype == NRR_U16 ? sizeof(int32_t) : sizeof(double);
    size_t er = dtype == NRR_U16 ? sizeof(float) : sizeof(double);
    L.s_off = 0;
    L.r_off = align_up(nvox * es, 256);
    L.total = L.r_off + align_up(nvox * er, 256);
    return L;
}

hipError_t launch_stats(const void *flt, nrr_dtype dtype, const int32_t dims[3], int32_t block,
                        void *workspace, hipStream_t stream) {
    StatsLayout L = stats_layout(dtype, dims, block);
    char *ws = static_cast<char *>(workspace);
    dim3 grid((L.ox + TX - 1) / TX, (L.oy + TY - 1) / TY, (L.oz + ZC - 1) / ZC);
    if (dtype == NRR_U16)
        hipLaunchKernelGGL(k_stats_u16, grid, dim3(256), (size_t)block * TX * TY * 8, stream,
                           static_cast<const uint16_t *>(flt), dims[0], dims[1], dims[2], block,
                           L.ox, L.oy, L.oz, reinterpret_cast<int32_t *>(ws + L.s_off),
                           reinterpret_cast<float *>(ws + L.r_off));
    else
        hipLaunchKernelGGL(k_stats_f32, grid, dim3(256), (size_t)block * TX * TY * 16, stream,
                           static_cast<const float *>(flt), dims[0], dims[1], dims[2], block,
                           L.ox, L.oy, L.oz, reinterpret_cast<double *>(ws + L.s_off),
                           reinterpret_cast<double *>(ws + L.r_off));
    return hipGetLastError();
}

}  // namespace nrr
