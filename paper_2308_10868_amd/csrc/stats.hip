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
// so the z sum is b adds.
#include <hip/hip_runtime.h>

#include "nrr_internal.h"

namespace nrr {
namespace {

constexpr int TX = 64, TY = 4, ZC = 16, MAXB = 15;
constexpr int PW = TX + MAXB - 1, PH = TY + MAXB - 1;

__global__ __launch_bounds__(256) void k_stats_u16(const uint16_t *__restrict__ flt, int nx,
                                                   int ny, int nz, int b, int ox, int oy, int oz,
                                                   int32_t *__restrict__ s_out,
                                                   float *__restrict__ r_out) {
    __shared__ int32_t patch[PH][PW];
    __shared__ int32_t xs[PH][TX];
    __shared__ uint32_t xq[PH][TX];
    // ring of the last b per-plane sums, [b][256] each (dynamic LDS)
    extern __shared__ __align__(16) unsigned char dyn_u16[];
    int32_t(*ringP)[TX * TY] = reinterpret_cast<int32_t(*)[TX * TY]>(dyn_u16);
    uint32_t(*ringQ)[TX * TY] = reinterpret_cast<uint32_t(*)[TX * TY]>(dyn_u16 + (size_t)b * TX * TY * 4);
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * ZC;
    const int ph = TY + b - 1, pw = TX + b - 1;
    const int zend = min(z0 + ZC + b - 1, nz);  // input planes [z0, zend)
    const int64_t n = (int64_t)b * b * b;
    for (int zi = z0; zi < zend; ++zi) {
        for (int e = tid; e < ph * pw; e += 256) {
            int r = e / pw, c = e % pw;
            int x = x0 + c, y = y0 + r;
            patch[r][c] = (x < nx && y < ny) ? (int32_t)flt[((int64_t)zi * ny + y) * nx + x] - 2048 : 0;
        }
        __syncthreads();
        for (int r = ty; r < ph; r += TY) {
            int32_t s = 0;
            uint32_t q = 0;
            for (int k = 0; k < b; ++k) {
                int32_t v = patch[r][tx + k];
                s += v;
                q += (uint32_t)(v * v);
            }
            xs[r][tx] = s;
            xq[r][tx] = q;
        }
        __syncthreads();
        int32_t P = 0;
        uint32_t Q = 0;
        for (int k = 0; k < b; ++k) {
            P += xs[ty + k][tx];
            Q += xq[ty + k][tx];
        }
        const int slot = (zi - z0) % b;
        ringP[slot][tid] = P;
        ringQ[slot][tid] = Q;
        if (zi - z0 >= b - 1) {
            const int z = zi - b + 1, x = x0 + tx, y = y0 + ty;
            if (x < ox && y < oy && z < oz) {
                int32_t S = 0;
                uint64_t QQ = 0;
                for (int k = 0; k < b; ++k) {
                    S += ringP[k][tid];
                    QQ += ringQ[k][tid];
                }
                int64_t var = n * (int64_t)QQ - (int64_t)S * S;
                int64_t o = ((int64_t)z * oy + y) * ox + x;
                s_out[o] = S;
                r_out[o] = var > 0 ? (float)(1.0 / sqrt((double)var)) : 0.0f;
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_stats_f32(const float *__restrict__ flt, int nx, int ny,
                                                   int nz, int b, int ox, int oy, int oz,
                                                   double *__restrict__ s_out,
                                                   double *__restrict__ r_out) {
    __shared__ float patch[PH][PW];
    __shared__ double xs[PH][TX];
    __shared__ double xq[PH][TX];
    extern __shared__ __align__(16) unsigned char dyn_f32[];
    double(*ringP)[TX * TY] = reinterpret_cast<double(*)[TX * TY]>(dyn_f32);
    double(*ringQ)[TX * TY] = reinterpret_cast<double(*)[TX * TY]>(dyn_f32 + (size_t)b * TX * TY * 8);
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * ZC;
    const int ph = TY + b - 1, pw = TX + b - 1;
    const int zend = min(z0 + ZC + b - 1, nz);
    const double n = (double)b * b * b;
    for (int zi = z0; zi < zend; ++zi) {
        for (int e = tid; e < ph * pw; e += 256) {
            int r = e / pw, c = e % pw;
            int x = x0 + c, y = y0 + r;
            patch[r][c] = (x < nx && y < ny) ? flt[((int64_t)zi * ny + y) * nx + x] : 0.0f;
        }
        __syncthreads();
        for (int r = ty; r < ph; r += TY) {
            double s = 0.0, q = 0.0;
            for (int k = 0; k < b; ++k) {
                double v = (double)patch[r][tx + k];
                s += v;
                q += v * v;
            }
            xs[r][tx] = s;
            xq[r][tx] = q;
        }
        __syncthreads();
        double P = 0.0, Q = 0.0;
        for (int k = 0; k < b; ++k) {
            P += xs[ty + k][tx];
            Q += xq[ty + k][tx];
        }
        const int slot = (zi - z0) % b;
        ringP[slot][tid] = P;
        ringQ[slot][tid] = Q;
        if (zi - z0 >= b - 1) {
            const int z = zi - b + 1, x = x0 + tx, y = y0 + ty;
            if (x < ox && y < oy && z < oz) {
                double S = 0.0, QQ = 0.0;
                for (int k = 0; k < b; ++k) {
                    S += ringP[k][tid];
                    QQ += ringQ[k][tid];
                }
                double nq = n * QQ;
                double var = nq - S * S;
                int64_t o = ((int64_t)z * oy + y) * ox + x;
                s_out[o] = S;
                r_out[o] = var > 1e-12 * nq ? 1.0 / sqrt(var) : 0.0;
            }
        }
        __syncthreads();
    }
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
