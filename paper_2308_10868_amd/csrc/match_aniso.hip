// Exhaustive NCC search with per-axis block edges and half windows.
//
// The paper's parameter list has a half block size and a half search window
// per anatomical axis (the "Deep Learning Model Architecture" section), so a
// block is bx x by x bz and the displacement set [-wx, wx] x [-wy, wy] x
// [-wz, wz].  The cubic search has its own tuned kernels; this is the
// general kernel for any such shape (edges and half windows up to 15).
//
// One workgroup per block.  The reference block T is centred in FP64 and
// kept in LDS as float, its rows padded with zeros to a multiple of 8; the
// moving volume's window region is staged in LDS a run of `cz` displacement
// planes at a time.  A thread owns RX consecutive x displacements of one
// (dy, dz) and accumulates X(d) = sum T'(v) F(v + d) with an 8-wide
// unrolled inner product (each staged F value feeds up to RX products).  As
// T' sums to zero, X(d) is the cross term of the correlation, so X(d) times
// the displaced block's 1/sqrt(N sum F^2 - (sum F)^2) from the statistics
// table ranks the displacements like the NCC.  The workgroup's argmax
// (largest key, smallest shift index on ties) is then rescored exactly, in
// two FP64 passes over the block, for the reported NCC.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "nrr_internal.h"

namespace nrr {
namespace {

constexpr int NT = 256;
constexpr int TU = 8;  // T row padding and inner-product unroll

template <typename K>
__device__ inline void better(K &bk, int &bi, K k, int i) {
    if (k > bk || (k == bk && i < bi)) {
        bk = k;
        bi = i;
    }
}

// Sum of v over the workgroup (every thread gets it).
__device__ inline double wg_sum(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();  // red is reused across calls
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[w];
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

template <typename Vox, int RX>
__global__ __launch_bounds__(NT) void k_match_aniso(AnisoArgs p) {
    using Key = typename Rec<Vox>::Key;
    extern __shared__ __align__(16) float lds[];
    __shared__ double red[NT / 64];
    __shared__ Key s_key[NT / 64];
    __shared__ int s_idx[NT / 64];
    const int64_t blk = blockIdx.x;
    const int tid = threadIdx.x;
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
    for (int o = tid; o < nb; o += NT) {
        const int x = o % bx, y = (o / bx) % by, z = o / (bx * by);
        st += (double)ref[rbase + z * sz + (int64_t)y * sy + x];
    }
    const double mt = wg_sum(st, red) / nb;
    for (int e = tid; e < bz * by * TP; e += NT) {
        const int x = e % TP, r = e / TP, y = r % by, z = r / by;
        T[e] = x < bx ? (float)((double)ref[rbase + z * sz + (int64_t)y * sy + x] - mt) : 0.0f;
    }
    const float cf = (float)mt;  // level taken off F (T' sums to zero)

    const int ntx = (ndx + RX - 1) / RX;
    const int FP = ntx * RX + TP;  // F row pitch: the widest tile's reads stay inside
    const int EY = ndy + by - 1, EX = ndx + bx - 1;
    float *F = T + bz * by * TP;
    const int wx0 = cx - hx + lox, wy0 = cy - hy + loy, wz0 = cz - hz + loz;
    Key bk = -INFINITY;
    int bi = INT_MAX;
    for (int z0 = 0; z0 < ndz; z0 += p.cz) {
        const int czn = min(p.cz, ndz - z0), EZ = czn + bz - 1;
        __syncthreads();  // T written / previous run's readers done
        for (int e = tid; e < EZ * EY * FP; e += NT) {
            const int x = e % FP, r = e / FP, y = r % EY, z = r / EY;
            F[e] = x < EX ? (float)flt[(wz0 + z0 + z) * sz + (int64_t)(wy0 + y) * sy + wx0 + x] - cf
                          : 0.0f;
        }
        __syncthreads();
        const int ntile = ntx * ndy * czn;
        for (int t = tid; t < ntile; t += NT) {
            const int tx = t % ntx, ty = (t / ntx) % ndy, tz = t / (ntx * ndy);
            float acc[RX];
#pragma unroll
            for (int j = 0; j < RX; ++j) acc[j] = 0.0f;
            for (int z = 0; z < bz; ++z)
                for (int y = 0; y < by; ++y) {
                    const float *tr = T + (z * by + y) * TP;
                    const float *fr = F + ((tz + z) * EY + (ty + y)) * FP + tx * RX;
                    for (int x0 = 0; x0 < TP; x0 += TU) {
                        float f[TU + RX - 1];
#pragma unroll
                        for (int j = 0; j < TU + RX - 1; ++j) f[j] = fr[x0 + j];
#pragma unroll
                        for (int xx = 0; xx < TU; ++xx) {
                            const float tv = tr[x0 + xx];
#pragma unroll
                            for (int j = 0; j < RX; ++j) acc[j] = fmaf(tv, f[xx + j], acc[j]);
                        }
                    }
                }
            const int dz = loz + z0 + tz, dy = loy + ty;
            const int64_t orow = ((int64_t)(cz - hz + dz) * p.oy + (cy - hy + dy)) * p.ox;
            const int irow = ((dz + wz) * (2 * wy + 1) + (dy + wy)) * (2 * wx + 1) + wx;
#pragma unroll
            for (int j = 0; j < RX; ++j) {
                const int ix = tx * RX + j;
                if (ix < ndx) {
                    const int dx = lox + ix;
                    Key k = (Key)acc[j] * Rec<Vox>::r(p.stats, orow + cx - hx + dx);
                    if (k != k) k = -INFINITY;  // overflowed sums rank last, never unranked
                    better(bk, bi, k, irow + dx);
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
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) better(bk, bi, s_key[w], s_idx[w]);
    const int sxn = 2 * wx + 1, syn = 2 * wy + 1;
    const int dx = bi % sxn - wx, dy = (bi / sxn) % syn - wy, dz = bi / (sxn * syn) - wz;

    // exact NCC of the winner: two FP64 passes over the block
    const int64_t fbase = rbase + dz * sz + (int64_t)dy * sy + dx;
    double sf = 0.0;
    for (int o = tid; o < nb; o += NT) {
        const int x = o % bx, y = (o / bx) % by, z = o / (bx * by);
        sf += (double)flt[fbase + z * sz + (int64_t)y * sy + x];
    }
    const double mf = wg_sum(sf, red) / nb;
    double a = 0.0, b = 0.0, x2 = 0.0;
    for (int o = tid; o < nb; o += NT) {
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

// LDS bytes of one workgroup for a z-run of cz displacement planes.
size_t aniso_lds(const int32_t b[3], const int32_t w[3], int rx, int cz) {
    const int tp = (b[0] + TU - 1) / TU * TU;
    const int ntx = (2 * w[0] + 1 + rx - 1) / rx;
    const size_t fp = (size_t)ntx * rx + tp, ey = 2 * w[1] + 1 + b[1] - 1;
    return 4 * ((size_t)b[2] * b[1] * tp + (size_t)(cz + b[2] - 1) * ey * fp);
}

// RX = 8 unless that leaves many more idle x slots than RX = 4.
int aniso_rx(int32_t wx) {
    const int n = 2 * wx + 1;
    const int pad8 = (n + 7) / 8 * 8, pad4 = (n + 3) / 4 * 4;
    return pad8 * 4 <= pad4 * 5 ? 8 : 4;
}

// Largest z-run that fits `budget` bytes of LDS (0: not even one plane).
int aniso_cz(const int32_t b[3], const int32_t w[3], int rx, size_t budget) {
    int cz = 2 * w[2] + 1;
    while (cz > 0 && aniso_lds(b, w, rx, cz) > budget) --cz;
    return cz;
}

}  // namespace

const char *aniso_unsupported_reason(const int32_t block[3], const int32_t window[3]) {
    for (int a = 0; a < 3; ++a) {
        if (block[a] > 15) return "block edge above 15 is not built";
        if (window[a] > 15) return "half window above 15 is not built";
    }
    if (aniso_cz(block, window, aniso_rx(window[0]), device_lds_limit()) < 1)
        return "window region does not fit in LDS";
    return nullptr;
}

hipError_t launch_match_aniso(nrr_dtype dtype, const AnisoArgs &a0, hipStream_t stream) {
    if (a0.n <= 0) return hipSuccess;
    AnisoArgs a = a0;
    const int rx = aniso_rx(a.w[0]);
    // two workgroups per CU when a run of at least 2 planes fits in half the LDS
    const size_t lim = device_lds_limit();
    int cz = aniso_cz(a.b, a.w, rx, lim / 2);
    if (cz < 2) cz = aniso_cz(a.b, a.w, rx, lim);
    if (cz < 1) return hipErrorInvalidValue;
    a.cz = cz;
    const size_t lds = aniso_lds(a.b, a.w, rx, cz);
    void (*fn)(AnisoArgs);
    if (dtype == NRR_U16)
        fn = rx == 8 ? k_match_aniso<uint16_t, 8> : k_match_aniso<uint16_t, 4>;
    else
        fn = rx == 8 ? k_match_aniso<float, 8> : k_match_aniso<float, 4>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3((unsigned)a.n), dim3(NT), lds, stream, a);
    return hipGetLastError();
}

}  // namespace nrr
