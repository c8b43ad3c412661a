/*
 * Block-matching oracle: a plain, slow, FP64 CPU implementation of what the
 * block-matching stage of physics-based non-rigid registration computes.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the HIP path.
 *
 * What it follows (paper: "Physics-Based Non-Rigid Registration" section and
 * the "Parallel feature selection" paragraph of the HPC section):
 *
 *  - Selection: every candidate block of edge b is scored by the variance of
 *    its intensities; the blocks are ordered by variance and the count kept
 *    is 0.5 + NFeatures * Fs, read as K = floor(0.5 + N * F).
 *  - Matching: a block centred at a selected point in the pre-operative
 *    volume (here `ref`) is compared with every equally sized block inside a
 *    search window of the intra-operative volume (here `flt`); the similarity
 *    is the normalised cross-correlation of the NCC equation, read as the
 *    Pearson correlation over the block's voxels; the displacement that
 *    maximises it is the sparse deformation vector at that point
 *    (exhaustive search: every displacement in the window is evaluated and
 *    the maximum taken, as in the GPU block-matching algorithm).
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes of the repository):
 *  - volumes are C-order [z][y][x], dims = (nx, ny, nz), vectors are (x,y,z);
 *  - b is odd, h = (b-1)/2, a block centred at c covers c+o, o in [-h,h]^3;
 *  - candidate grid: origins g*stride per axis, g = 0..G-1,
 *    G = floor((n-b)/stride)+1, centre = origin + h, linear grid index
 *    (gz*Gy+gy)*Gx+gx;
 *  - selection ties: equal variance -> lower grid index ranks first; the
 *    selected centres are returned in ascending grid index;
 *  - u16 input: the variance is ranked through the exact integer key
 *    N*sum(x^2) - (sum x)^2 (= N^2 * variance); f32 input: FP64 two-pass
 *    variance;
 *  - displacement set: d in [-W,W]^3 with the displaced block fully inside
 *    `flt`; shift index iota(d) = ((dz+W)(2W+1) + (dy+W))(2W+1) + (dx+W);
 *  - NCC(d) = X / sqrt(A*B) with A = sum (T-Tbar)^2, B = sum (F-Fbar)^2,
 *    X = sum (T-Tbar)(F-Fbar); NCC = 0 when A*B == 0 (flat block/window);
 *  - argmax: largest NCC, exact FP64 ties -> smallest iota;
 *  - confidence = max(0, NCC at the argmax);
 *  - a centre whose block is not inside the volume: disp (0,0,0), ncc NaN,
 *    conf 0.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC nrr_oracle.c -o liboracle.so -lm
 * (no intrinsics, no fast-math, no FMA contraction across statements).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_U16 0
#define ORACLE_F32 1

/* Value of voxel (x, y, z) as a double (u16 and f32 convert exactly). */
static double voxel(const void *vol, int dtype, const int32_t dims[3], int64_t x, int64_t y,
                    int64_t z) {
    int64_t idx = (z * (int64_t)dims[1] + y) * (int64_t)dims[0] + x;
    if (dtype == ORACLE_U16) return (double)((const uint16_t *)vol)[idx];
    return (double)((const float *)vol)[idx];
}

int oracle_grid_shape(const int32_t dims[3], int32_t b, int32_t stride, int32_t grid[3]) {
    for (int a = 0; a < 3; ++a) {
        if (dims[a] < b || b < 1 || stride < 1) return -1;
        grid[a] = (dims[a] - b) / stride + 1;
    }
    return 0;
}

/* K = floor(0.5 + N * F), clamped to [0, N]. */
int64_t oracle_select_count(int64_t n_candidates, double fraction) {
    double k = floor(0.5 + (double)n_candidates * fraction);
    if (k < 0) k = 0;
    if (k > (double)n_candidates) k = (double)n_candidates;
    return (int64_t)k;
}

typedef struct {
    double key;   /* ranking key: larger = more variable */
    int64_t idx;  /* linear grid index */
} ranked_t;

static int cmp_rank(const void *pa, const void *pb) {
    const ranked_t *a = (const ranked_t *)pa, *b = (const ranked_t *)pb;
    if (a->key > b->key) return -1;
    if (a->key < b->key) return 1;
    return (a->idx < b->idx) ? -1 : (a->idx > b->idx);
}

static int cmp_i64(const void *pa, const void *pb) {
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    return (a < b) ? -1 : (a > b);
}

/*
 * Variance of every candidate block.  out_key[g] is the ranking key
 * (u16: exact integer N*sum x^2 - (sum x)^2 held in a double, < 2^53;
 * f32: two-pass FP64 variance), out_var[g] the FP64 two-pass variance.
 */
int oracle_block_variance(const void *vol, int dtype, const int32_t dims[3], int32_t b,
                          int32_t stride, double *out_key, double *out_var) {
    int32_t grid[3];
    if (oracle_grid_shape(dims, b, stride, grid)) return -1;
    int64_t n = (int64_t)grid[0] * grid[1] * grid[2];
    double nb = (double)b * b * b;
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
        int64_t gx = g % grid[0], gy = (g / grid[0]) % grid[1], gz = g / ((int64_t)grid[0] * grid[1]);
        int64_t x0 = gx * stride, y0 = gy * stride, z0 = gz * stride;
        double sum = 0.0;
        int64_t isum = 0, isq = 0;
        for (int64_t z = z0; z < z0 + b; ++z)
            for (int64_t y = y0; y < y0 + b; ++y)
                for (int64_t x = x0; x < x0 + b; ++x) {
                    double v = voxel(vol, dtype, dims, x, y, z);
                    sum += v;
                    if (dtype == ORACLE_U16) {
                        int64_t iv = (int64_t)v;
                        isum += iv;
                        isq += iv * iv;
                    }
                }
        double mean = sum / nb;
        double ss = 0.0;
        for (int64_t z = z0; z < z0 + b; ++z)
            for (int64_t y = y0; y < y0 + b; ++y)
                for (int64_t x = x0; x < x0 + b; ++x) {
                    double d = voxel(vol, dtype, dims, x, y, z) - mean;
                    ss += d * d;
                }
        out_var[g] = ss / nb;
        if (dtype == ORACLE_U16)
            out_key[g] = (double)((int64_t)(b * b * b) * isq - isum * isum);
        else
            out_key[g] = out_var[g];
    }
    return 0;
}

/*
 * Selection.  Writes the K selected centres (x,y,z) in ascending grid index
 * to out_centers[K][3] and their variances to out_var[K] (may be NULL).
 * Returns K, or -1 on bad arguments, or -2 if capacity < K.
 */
int64_t oracle_select(const void *vol, int dtype, const int32_t dims[3], int32_t b,
                      int32_t stride, double fraction, int32_t *out_centers, double *out_var,
                      int64_t capacity) {
    int32_t grid[3];
    if (b < 1 || (b % 2) == 0 || oracle_grid_shape(dims, b, stride, grid)) return -1;
    if (!(fraction > 0.0) || fraction > 1.0) return -1;
    int64_t n = (int64_t)grid[0] * grid[1] * grid[2];
    int64_t k = oracle_select_count(n, fraction);
    if (k > capacity) return -2;
    double *key = (double *)malloc(sizeof(double) * n);
    double *var = (double *)malloc(sizeof(double) * n);
    ranked_t *r = (ranked_t *)malloc(sizeof(ranked_t) * n);
    int64_t *chosen = (int64_t *)malloc(sizeof(int64_t) * (k > 0 ? k : 1));
    oracle_block_variance(vol, dtype, dims, b, stride, key, var);
    for (int64_t g = 0; g < n; ++g) {
        r[g].key = key[g];
        r[g].idx = g;
    }
    qsort(r, (size_t)n, sizeof(ranked_t), cmp_rank);
    for (int64_t i = 0; i < k; ++i) chosen[i] = r[i].idx;
    qsort(chosen, (size_t)k, sizeof(int64_t), cmp_i64);
    int32_t h = (b - 1) / 2;
    for (int64_t i = 0; i < k; ++i) {
        int64_t g = chosen[i];
        int64_t gx = g % grid[0], gy = (g / grid[0]) % grid[1], gz = g / ((int64_t)grid[0] * grid[1]);
        out_centers[3 * i + 0] = (int32_t)(gx * stride + h);
        out_centers[3 * i + 1] = (int32_t)(gy * stride + h);
        out_centers[3 * i + 2] = (int32_t)(gz * stride + h);
        if (out_var) out_var[i] = var[g];
    }
    free(key);
    free(var);
    free(r);
    free(chosen);
    return k;
}

/*
 * Selection with the variants of the "Parallel feature selection" paragraph:
 * a connectivity pattern that keeps selected blocks apart, and candidates
 * restricted to a region (the intracranial cavity in the paper; here any
 * 0/1 mask).
 *
 *  - mask (may be NULL): uint8 volume like `vol`; a candidate takes part iff
 *    the mask is nonzero at its centre.  N = number of such candidates and
 *    K = floor(0.5 + N * fraction).
 *  - connectivity 0, 6, 18 or 26: candidates are visited in rank order
 *    (variance descending, grid index ascending); one is taken unless a
 *    candidate adjacent to it on the grid is already taken, where adjacent
 *    means one grid step along one axis (6, faces), along at most two axes
 *    (18, faces and edges) or along up to three (26, also vertices); the
 *    visit stops once K are taken (fewer when the candidates run out).
 *  - output: the taken centres in ascending grid index (and variances).
 * Returns the number taken, -1 on bad arguments, -2 if capacity < K.
 */
int64_t oracle_select_ex(const void *vol, int dtype, const int32_t dims[3], int32_t b,
                         int32_t stride, double fraction, const uint8_t *mask,
                         int32_t connectivity, int32_t *out_centers, double *out_var,
                         int64_t capacity) {
    int32_t grid[3];
    if (b < 1 || (b % 2) == 0 || oracle_grid_shape(dims, b, stride, grid)) return -1;
    if (!(fraction > 0.0) || fraction > 1.0) return -1;
    if (connectivity != 0 && connectivity != 6 && connectivity != 18 && connectivity != 26)
        return -1;
    const int64_t n = (int64_t)grid[0] * grid[1] * grid[2];
    const int32_t h = (b - 1) / 2;
    double *key = (double *)malloc(sizeof(double) * n);
    double *var = (double *)malloc(sizeof(double) * n);
    ranked_t *r = (ranked_t *)malloc(sizeof(ranked_t) * n);
    unsigned char *taken = (unsigned char *)calloc((size_t)n, 1);
    int64_t *chosen = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    oracle_block_variance(vol, dtype, dims, b, stride, key, var);
    int64_t m = 0;
    for (int64_t g = 0; g < n; ++g) {
        const int64_t gx = g % grid[0], gy = (g / grid[0]) % grid[1],
                      gz = g / ((int64_t)grid[0] * grid[1]);
        const int64_t cx = gx * stride + h, cy = gy * stride + h, cz = gz * stride + h;
        if (mask && !mask[(cz * dims[1] + cy) * (int64_t)dims[0] + cx]) continue;
        r[m].key = key[g];
        r[m].idx = g;
        ++m;
    }
    const int64_t k = oracle_select_count(m, fraction);
    if (k > capacity) {
        free(key), free(var), free(r), free(taken), free(chosen);
        return -2;
    }
    qsort(r, (size_t)m, sizeof(ranked_t), cmp_rank);
    int64_t got = 0;
    for (int64_t i = 0; i < m && got < k; ++i) {
        const int64_t g = r[i].idx;
        const int64_t gx = g % grid[0], gy = (g / grid[0]) % grid[1],
                      gz = g / ((int64_t)grid[0] * grid[1]);
        int blocked = 0;
        for (int dz = -1; dz <= 1 && !blocked && connectivity; ++dz)
            for (int dy = -1; dy <= 1 && !blocked; ++dy)
                for (int dx = -1; dx <= 1 && !blocked; ++dx) {
                    const int steps = (dx != 0) + (dy != 0) + (dz != 0);
                    if (steps == 0) continue;
                    if (connectivity == 6 && steps > 1) continue;
                    if (connectivity == 18 && steps > 2) continue;
                    const int64_t x = gx + dx, y = gy + dy, z = gz + dz;
                    if (x < 0 || y < 0 || z < 0 || x >= grid[0] || y >= grid[1] || z >= grid[2])
                        continue;
                    if (taken[(z * grid[1] + y) * grid[0] + x]) blocked = 1;
                }
        if (blocked) continue;
        taken[g] = 1;
        chosen[got++] = g;
    }
    qsort(chosen, (size_t)got, sizeof(int64_t), cmp_i64);
    for (int64_t i = 0; i < got; ++i) {
        const int64_t g = chosen[i];
        const int64_t gx = g % grid[0], gy = (g / grid[0]) % grid[1],
                      gz = g / ((int64_t)grid[0] * grid[1]);
        out_centers[3 * i + 0] = (int32_t)(gx * stride + h);
        out_centers[3 * i + 1] = (int32_t)(gy * stride + h);
        out_centers[3 * i + 2] = (int32_t)(gz * stride + h);
        if (out_var) out_var[i] = var[g];
    }
    free(key), free(var), free(r), free(taken), free(chosen);
    return got;
}

/* Is the block of edge b centred at (cx,cy,cz) inside the volume? */
static int block_inside(const int32_t dims[3], int32_t h, int64_t cx, int64_t cy, int64_t cz) {
    return cx - h >= 0 && cy - h >= 0 && cz - h >= 0 && cx + h <= dims[0] - 1 &&
           cy + h <= dims[1] - 1 && cz + h <= dims[2] - 1;
}

/*
 * NCC between the ref block at c and the flt block at c+d (Pearson
 * correlation over the b^3 voxels, two-pass FP64; 0 if either is flat).
 * T (the ref block) is passed in already centred, with A = sum T^2.
 */
static double ncc_at(const double *tc, double a, const void *flt, int dtype,
                     const int32_t dims[3], int32_t b, int64_t x0, int64_t y0, int64_t z0,
                     double *fbuf) {
    int64_t nb = (int64_t)b * b * b, i = 0;
    double sum = 0.0;
    for (int64_t z = z0; z < z0 + b; ++z)
        for (int64_t y = y0; y < y0 + b; ++y)
            for (int64_t x = x0; x < x0 + b; ++x) {
                fbuf[i] = voxel(flt, dtype, dims, x, y, z);
                sum += fbuf[i++];
            }
    double mean = sum / (double)nb;
    double bb = 0.0, xx = 0.0;
    for (i = 0; i < nb; ++i) {
        double f = fbuf[i] - mean;
        bb += f * f;
        xx += tc[i] * f;
    }
    double ab = a * bb;
    if (!(ab > 0.0)) return 0.0;
    return xx / sqrt(ab);
}

/* Centred ref block and its A = sum (T - Tbar)^2. */
static double centred_block(const void *ref, int dtype, const int32_t dims[3], int32_t b,
                            int64_t x0, int64_t y0, int64_t z0, double *tc) {
    int64_t nb = (int64_t)b * b * b, i = 0;
    double sum = 0.0;
    for (int64_t z = z0; z < z0 + b; ++z)
        for (int64_t y = y0; y < y0 + b; ++y)
            for (int64_t x = x0; x < x0 + b; ++x) {
                tc[i] = voxel(ref, dtype, dims, x, y, z);
                sum += tc[i++];
            }
    double mean = sum / (double)nb, a = 0.0;
    for (i = 0; i < nb; ++i) {
        tc[i] -= mean;
        a += tc[i] * tc[i];
    }
    return a;
}

/* Valid displacement range on one axis: block at c+d stays inside [0, n-1]. */
static void valid_range(int64_t c, int32_t h, int32_t n, int32_t w, int64_t *lo, int64_t *hi) {
    *lo = -w;
    if (*lo < h - c) *lo = h - c;
    *hi = w;
    if (*hi > (n - 1 - h) - c) *hi = (n - 1 - h) - c;
}

/*
 * Exhaustive matching for n centres.  disp[n][3] (dx,dy,dz), ncc[n],
 * conf[n].  Returns 0, or -1 on bad arguments.
 */
int oracle_match(const void *ref, const void *flt, int dtype, const int32_t dims[3],
                 const int32_t *centers, int64_t n, int32_t b, int32_t w, int32_t *disp,
                 double *ncc, double *conf) {
    if (b < 1 || (b % 2) == 0 || w < 0) return -1;
    int32_t h = (b - 1) / 2;
    int64_t nb = (int64_t)b * b * b;
#pragma omp parallel
    {
        double *tc = (double *)malloc(sizeof(double) * nb);
        double *fb = (double *)malloc(sizeof(double) * nb);
#pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < n; ++k) {
            int64_t cx = centers[3 * k], cy = centers[3 * k + 1], cz = centers[3 * k + 2];
            if (!block_inside(dims, h, cx, cy, cz)) {
                disp[3 * k] = disp[3 * k + 1] = disp[3 * k + 2] = 0;
                ncc[k] = NAN;
                conf[k] = 0.0;
                continue;
            }
            double a = centred_block(ref, dtype, dims, b, cx - h, cy - h, cz - h, tc);
            int64_t lx, hx, ly, hy, lz, hz;
            valid_range(cx, h, dims[0], w, &lx, &hx);
            valid_range(cy, h, dims[1], w, &ly, &hy);
            valid_range(cz, h, dims[2], w, &lz, &hz);
            double best = -INFINITY;
            int64_t bx = 0, by = 0, bz = 0;
            /* increasing shift index: dz slowest, dx fastest; strict '>'
               keeps the smallest index among exact ties */
            for (int64_t dz = lz; dz <= hz; ++dz)
                for (int64_t dy = ly; dy <= hy; ++dy)
                    for (int64_t dx = lx; dx <= hx; ++dx) {
                        double v = ncc_at(tc, a, flt, dtype, dims, b, cx - h + dx, cy - h + dy,
                                          cz - h + dz, fb);
                        if (v > best) {
                            best = v;
                            bx = dx;
                            by = dy;
                            bz = dz;
                        }
                    }
            disp[3 * k] = (int32_t)bx;
            disp[3 * k + 1] = (int32_t)by;
            disp[3 * k + 2] = (int32_t)bz;
            ncc[k] = best;
            conf[k] = best > 0.0 ? best : 0.0;
        }
        free(tc);
        free(fb);
    }
    return 0;
}

/*
 * Full NCC surface for each of n centres: out[k][(2W+1)^3] indexed by the
 * shift index iota; NaN where the displaced block leaves the volume (and for
 * every entry of a centre whose block is not inside).
 */
int oracle_ncc_surface(const void *ref, const void *flt, int dtype, const int32_t dims[3],
                       const int32_t *centers, int64_t n, int32_t b, int32_t w, double *out) {
    if (b < 1 || (b % 2) == 0 || w < 0) return -1;
    int32_t h = (b - 1) / 2;
    int64_t nb = (int64_t)b * b * b, side = 2 * (int64_t)w + 1, ns = side * side * side;
#pragma omp parallel
    {
        double *tc = (double *)malloc(sizeof(double) * nb);
        double *fb = (double *)malloc(sizeof(double) * nb);
#pragma omp for schedule(dynamic, 1)
        for (int64_t k = 0; k < n; ++k) {
            double *o = out + k * ns;
            for (int64_t s = 0; s < ns; ++s) o[s] = NAN;
            int64_t cx = centers[3 * k], cy = centers[3 * k + 1], cz = centers[3 * k + 2];
            if (!block_inside(dims, h, cx, cy, cz)) continue;
            double a = centred_block(ref, dtype, dims, b, cx - h, cy - h, cz - h, tc);
            int64_t lx, hx, ly, hy, lz, hz;
            valid_range(cx, h, dims[0], w, &lx, &hx);
            valid_range(cy, h, dims[1], w, &ly, &hy);
            valid_range(cz, h, dims[2], w, &lz, &hz);
            for (int64_t dz = lz; dz <= hz; ++dz)
                for (int64_t dy = ly; dy <= hy; ++dy)
                    for (int64_t dx = lx; dx <= hx; ++dx)
                        o[((dz + w) * side + (dy + w)) * side + (dx + w)] =
                            ncc_at(tc, a, flt, dtype, dims, b, cx - h + dx, cy - h + dy,
                                   cz - h + dz, fb);
        }
        free(tc);
        free(fb);
    }
    return 0;
}

/* Number of valid displacements (and so b^3 * that = evaluated voxel pairs)
   for each centre; 0 for a centre whose block is not inside. */
int oracle_valid_shifts(const int32_t dims[3], const int32_t *centers, int64_t n, int32_t b,
                        int32_t w, int64_t *out) {
    int32_t h = (b - 1) / 2;
    for (int64_t k = 0; k < n; ++k) {
        int64_t cx = centers[3 * k], cy = centers[3 * k + 1], cz = centers[3 * k + 2];
        if (!block_inside(dims, h, cx, cy, cz)) {
            out[k] = 0;
            continue;
        }
        int64_t lx, hx, ly, hy, lz, hz;
        valid_range(cx, h, dims[0], w, &lx, &hx);
        valid_range(cy, h, dims[1], w, &ly, &hy);
        valid_range(cz, h, dims[2], w, &lz, &hz);
        out[k] = (hx - lx + 1) * (hy - ly + 1) * (hz - lz + 1);
    }
    return 0;
}

/*
 * Directional confidence (the confidence matrix S of the FEM update equation,
 * for which the paper gives no formula): per block centred at c, the
 * structure tensor J = sum over the block's voxels p of g(p) g(p)^T, with
 * g the intensity gradient of `ref` by central differences,
 * g_x(p) = (ref(p+e_x) - ref(p-e_x)) / 2, and one-sided differences
 * ref(p+e_x) - ref(p) / ref(p) - ref(p-e_x) on the volume's first / last
 * plane of that axis.  S = conf * J / trace(J) (S = 0 when trace(J) = 0).
 * out[6k..6k+5] = S_xx, S_yy, S_zz, S_xy, S_xz, S_yz.  A block not inside
 * the volume gets S = 0.  FP64.
 */
static double grad_axis(const void *vol, int dtype, const int32_t dims[3], int64_t x, int64_t y,
                        int64_t z, int axis) {
    int64_t p[3] = {x, y, z};
    const int64_t n = dims[axis];
    int64_t lo[3] = {x, y, z}, hi[3] = {x, y, z};
    double scale = 0.5;
    if (p[axis] == 0) {
        hi[axis] = 1;
        scale = 1.0;
    } else if (p[axis] == n - 1) {
        lo[axis] = n - 2;
        scale = 1.0;
    } else {
        lo[axis] = p[axis] - 1;
        hi[axis] = p[axis] + 1;
    }
    if (n == 1) return 0.0;
    return scale * (voxel(vol, dtype, dims, hi[0], hi[1], hi[2]) -
                    voxel(vol, dtype, dims, lo[0], lo[1], lo[2]));
}

int oracle_structure_confidence(const void *ref, int dtype, const int32_t dims[3],
                                const int32_t *centers, int64_t n, int32_t b, const double *conf,
                                double *out) {
    if (b < 1 || (b % 2) == 0) return -1;
    const int32_t h = (b - 1) / 2;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < n; ++k) {
        const int64_t cx = centers[3 * k], cy = centers[3 * k + 1], cz = centers[3 * k + 2];
        double j[6] = {0, 0, 0, 0, 0, 0};
        if (cx - h >= 0 && cy - h >= 0 && cz - h >= 0 && cx + h < dims[0] && cy + h < dims[1] &&
            cz + h < dims[2]) {
            for (int64_t z = cz - h; z <= cz + h; ++z)
                for (int64_t y = cy - h; y <= cy + h; ++y)
                    for (int64_t x = cx - h; x <= cx + h; ++x) {
                        const double gx = grad_axis(ref, dtype, dims, x, y, z, 0);
                        const double gy = grad_axis(ref, dtype, dims, x, y, z, 1);
                        const double gz = grad_axis(ref, dtype, dims, x, y, z, 2);
                        j[0] += gx * gx;
                        j[1] += gy * gy;
                        j[2] += gz * gz;
                        j[3] += gx * gy;
                        j[4] += gx * gz;
                        j[5] += gy * gz;
                    }
        }
        const double tr = j[0] + j[1] + j[2];
        for (int e = 0; e < 6; ++e) out[6 * k + e] = tr > 0.0 ? conf[k] * j[e] / tr : 0.0;
    }
    return 0;
}

/*
 * Per-axis block and window sizes.  The paper's parameter list gives the
 * half block size and the half search window per anatomical axis (the
 * "Deep Learning Model Architecture" section), so a block need not be a
 * cube.  Here b[a] = 2*Bs[a] + 1 and w[a] = Ws[a] for a = x, y, z; the
 * candidate grid takes its own stride per axis.  Everything else follows
 * the cubic readings: the grid, the count rule, ranking and ties, the
 * displacement set and shift index, NCC, argmax and the flat and outside
 * rules, with b^3 replaced by bx*by*bz and (2W+1) per axis by (2w[a]+1).
 */

/* Sum and sum of squares of the bx*by*bz block with lowest corner (x0,y0,z0)
   in z, y, x order; the exact integer key for 12-bit data. */
static void aniso_block_variance(const void *vol, int dtype, const int32_t dims[3],
                                 const int32_t b[3], int64_t x0, int64_t y0, int64_t z0,
                                 double *key, double *var) {
    const double nb = (double)b[0] * b[1] * b[2];
    double sum = 0.0;
    int64_t isum = 0, isq = 0;
    for (int64_t z = z0; z < z0 + b[2]; ++z)
        for (int64_t y = y0; y < y0 + b[1]; ++y)
            for (int64_t x = x0; x < x0 + b[0]; ++x) {
                const double v = voxel(vol, dtype, dims, x, y, z);
                sum += v;
                if (dtype == ORACLE_U16) {
                    isum += (int64_t)v;
                    isq += (int64_t)v * (int64_t)v;
                }
            }
    const double mean = sum / nb;
    double ss = 0.0;
    for (int64_t z = z0; z < z0 + b[2]; ++z)
        for (int64_t y = y0; y < y0 + b[1]; ++y)
            for (int64_t x = x0; x < x0 + b[0]; ++x) {
                const double d = voxel(vol, dtype, dims, x, y, z) - mean;
                ss += d * d;
            }
    *var = ss / nb;
    if (dtype == ORACLE_U16)
        *key = (double)((int64_t)b[0] * b[1] * b[2] * isq - isum * isum);
    else
        *key = *var;
}

static int aniso_sizes_ok(const int32_t dims[3], const int32_t b[3], const int32_t s[3],
                          int32_t grid[3]) {
    for (int a = 0; a < 3; ++a) {
        if (b[a] < 1 || (b[a] % 2) == 0 || s[a] < 1 || dims[a] < b[a]) return 0;
        grid[a] = (dims[a] - b[a]) / s[a] + 1;
    }
    return 1;
}

/* Selection with per-axis block edges b[3] and strides stride[3]. */
int64_t oracle_select_aniso(const void *vol, int dtype, const int32_t dims[3],
                            const int32_t b[3], const int32_t stride[3], double fraction,
                            int32_t *out_centers, double *out_var, int64_t capacity) {
    int32_t grid[3];
    if (!aniso_sizes_ok(dims, b, stride, grid)) return -1;
    if (!(fraction > 0.0) || fraction > 1.0) return -1;
    const int64_t n = (int64_t)grid[0] * grid[1] * grid[2];
    const int64_t k = oracle_select_count(n, fraction);
    if (k > capacity) return -2;
    double *var = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    ranked_t *r = (ranked_t *)malloc(sizeof(ranked_t) * (n > 0 ? n : 1));
    int64_t *chosen = (int64_t *)malloc(sizeof(int64_t) * (k > 0 ? k : 1));
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
        const int64_t gx = g % grid[0], gy = (g / grid[0]) % grid[1],
                      gz = g / ((int64_t)grid[0] * grid[1]);
        aniso_block_variance(vol, dtype, dims, b, gx * stride[0], gy * stride[1], gz * stride[2],
                             &r[g].key, &var[g]);
        r[g].idx = g;
    }
    qsort(r, (size_t)n, sizeof(ranked_t), cmp_rank);
    for (int64_t i = 0; i < k; ++i) chosen[i] = r[i].idx;
    qsort(chosen, (size_t)k, sizeof(int64_t), cmp_i64);
    for (int64_t i = 0; i < k; ++i) {
        const int64_t g = chosen[i];
        const int64_t gx = g % grid[0], gy = (g / grid[0]) % grid[1],
                      gz = g / ((int64_t)grid[0] * grid[1]);
        out_centers[3 * i + 0] = (int32_t)(gx * stride[0] + (b[0] - 1) / 2);
        out_centers[3 * i + 1] = (int32_t)(gy * stride[1] + (b[1] - 1) / 2);
        out_centers[3 * i + 2] = (int32_t)(gz * stride[2] + (b[2] - 1) / 2);
        if (out_var) out_var[i] = var[g];
    }
    free(var), free(r), free(chosen);
    return k;
}

/*
 * Selection variants with per-axis sizes: the region restriction and the
 * connectivity patterns of the "Parallel feature selection" paragraph on the
 * candidate grid of per-axis block edges b[3] and strides stride[3].  The
 * mask is read at each candidate's centre (origin + (b[a] - 1) / 2 per
 * axis), N counts the candidates inside it, K = floor(0.5 + N * fraction);
 * candidates are visited in rank order (key descending, grid index
 * ascending) and one is taken unless a grid neighbour (one step along one
 * axis for 6, along at most two axes for 18, up to three for 26) is already
 * taken; the visit stops at K taken.  Output as oracle_select_ex.
 */
int64_t oracle_select_aniso_ex(const void *vol, int dtype, const int32_t dims[3],
                               const int32_t b[3], const int32_t stride[3], double fraction,
                               const uint8_t *mask, int32_t connectivity, int32_t *out_centers,
                               double *out_var, int64_t capacity) {
    int32_t grid[3];
    if (!aniso_sizes_ok(dims, b, stride, grid)) return -1;
    if (!(fraction > 0.0) || fraction > 1.0) return -1;
    if (connectivity != 0 && connectivity != 6 && connectivity != 18 && connectivity != 26)
        return -1;
    /* axes a neighbour may step along: faces 1, faces and edges 2, all 3 */
    const int max_steps = connectivity == 6 ? 1 : connectivity == 18 ? 2 : connectivity == 26 ? 3 : 0;
    const int64_t n = (int64_t)grid[0] * grid[1] * grid[2];
    const int64_t plane = (int64_t)grid[0] * grid[1];
    double *var = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    ranked_t *all = (ranked_t *)malloc(sizeof(ranked_t) * (n > 0 ? n : 1));
    ranked_t *r = (ranked_t *)malloc(sizeof(ranked_t) * (n > 0 ? n : 1));
    unsigned char *taken = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t *chosen = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
        const int64_t gx = g % grid[0], gy = (g / grid[0]) % grid[1], gz = g / plane;
        aniso_block_variance(vol, dtype, dims, b, gx * stride[0], gy * stride[1], gz * stride[2],
                             &all[g].key, &var[g]);
        all[g].idx = g;
    }
    int64_t m = 0;
    for (int64_t g = 0; g < n; ++g) {
        const int64_t gx = g % grid[0], gy = (g / grid[0]) % grid[1], gz = g / plane;
        const int64_t cx = gx * stride[0] + (b[0] - 1) / 2, cy = gy * stride[1] + (b[1] - 1) / 2,
                      cz = gz * stride[2] + (b[2] - 1) / 2;
        if (mask && !mask[(cz * dims[1] + cy) * (int64_t)dims[0] + cx]) continue;
        r[m++] = all[g];
    }
    const int64_t k = oracle_select_count(m, fraction);
    if (k > capacity) {
        free(var), free(all), free(r), free(taken), free(chosen);
        return -2;
    }
    qsort(r, (size_t)m, sizeof(ranked_t), cmp_rank);
    int64_t got = 0;
    for (int64_t i = 0; i < m && got < k; ++i) {
        const int64_t g = r[i].idx;
        const int64_t gx = g % grid[0], gy = (g / grid[0]) % grid[1], gz = g / plane;
        int blocked = 0;
        for (int j = 0; j < 27 && !blocked; ++j) {
            const int dx = j % 3 - 1, dy = (j / 3) % 3 - 1, dz = j / 9 - 1;
            const int steps = (dx != 0) + (dy != 0) + (dz != 0);
            if (steps == 0 || steps > max_steps) continue;
            const int64_t x = gx + dx, y = gy + dy, z = gz + dz;
            if (x < 0 || y < 0 || z < 0 || x >= grid[0] || y >= grid[1] || z >= grid[2]) continue;
            blocked = taken[z * plane + y * grid[0] + x];
        }
        if (blocked) continue;
        taken[g] = 1;
        chosen[got++] = g;
    }
    qsort(chosen, (size_t)got, sizeof(int64_t), cmp_i64);
    for (int64_t i = 0; i < got; ++i) {
        const int64_t g = chosen[i];
        const int64_t gx = g % grid[0], gy = (g / grid[0]) % grid[1], gz = g / plane;
        out_centers[3 * i + 0] = (int32_t)(gx * stride[0] + (b[0] - 1) / 2);
        out_centers[3 * i + 1] = (int32_t)(gy * stride[1] + (b[1] - 1) / 2);
        out_centers[3 * i + 2] = (int32_t)(gz * stride[2] + (b[2] - 1) / 2);
        if (out_var) out_var[i] = var[g];
    }
    free(var), free(all), free(r), free(taken), free(chosen);
    return got;
}

/* Pearson correlation of the ref block at lowest corner (rx,ry,rz) and the
   flt block at (fx,fy,fz), both bx*by*bz, two-pass FP64; 0 if either is flat. */
static double aniso_ncc(const void *ref, const void *flt, int dtype, const int32_t dims[3],
                        const int32_t b[3], int64_t rx, int64_t ry, int64_t rz, int64_t fx,
                        int64_t fy, int64_t fz) {
    const double nb = (double)b[0] * b[1] * b[2];
    double st = 0.0, sf = 0.0;
    for (int64_t z = 0; z < b[2]; ++z)
        for (int64_t y = 0; y < b[1]; ++y)
            for (int64_t x = 0; x < b[0]; ++x) {
                st += voxel(ref, dtype, dims, rx + x, ry + y, rz + z);
                sf += voxel(flt, dtype, dims, fx + x, fy + y, fz + z);
            }
    const double mt = st / nb, mf = sf / nb;
    double a = 0.0, bb = 0.0, xx = 0.0;
    for (int64_t z = 0; z < b[2]; ++z)
        for (int64_t y = 0; y < b[1]; ++y)
            for (int64_t x = 0; x < b[0]; ++x) {
                const double t = voxel(ref, dtype, dims, rx + x, ry + y, rz + z) - mt;
                const double f = voxel(flt, dtype, dims, fx + x, fy + y, fz + z) - mf;
                a += t * t;
                bb += f * f;
                xx += t * f;
            }
    const double ab = a * bb;
    if (!(ab > 0.0)) return 0.0;
    return xx / sqrt(ab);
}

/* Exhaustive matching with per-axis block edges b[3] and half windows w[3]:
   shift index ((dz+wz)(2wy+1) + (dy+wy))(2wx+1) + (dx+wx), smallest on ties. */
int oracle_match_aniso(const void *ref, const void *flt, int dtype, const int32_t dims[3],
                       const int32_t *centers, int64_t n, const int32_t b[3], const int32_t w[3],
                       int32_t *disp, double *ncc, double *conf) {
    for (int a = 0; a < 3; ++a)
        if (b[a] < 1 || (b[a] % 2) == 0 || w[a] < 0) return -1;
    const int64_t h[3] = {(b[0] - 1) / 2, (b[1] - 1) / 2, (b[2] - 1) / 2};
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < n; ++k) {
        const int64_t c[3] = {centers[3 * k], centers[3 * k + 1], centers[3 * k + 2]};
        int inside = 1;
        int64_t lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            if (c[a] - h[a] < 0 || c[a] + h[a] > dims[a] - 1) inside = 0;
            lo[a] = -w[a] > h[a] - c[a] ? -w[a] : h[a] - c[a];
            hi[a] = w[a] < dims[a] - 1 - h[a] - c[a] ? w[a] : dims[a] - 1 - h[a] - c[a];
        }
        if (!inside) {
            disp[3 * k] = disp[3 * k + 1] = disp[3 * k + 2] = 0;
            ncc[k] = NAN;
            conf[k] = 0.0;
            continue;
        }
        double best = -INFINITY;
        int64_t bd[3] = {0, 0, 0};
        for (int64_t dz = lo[2]; dz <= hi[2]; ++dz)
            for (int64_t dy = lo[1]; dy <= hi[1]; ++dy)
                for (int64_t dx = lo[0]; dx <= hi[0]; ++dx) {
                    const double v = aniso_ncc(ref, flt, dtype, dims, b, c[0] - h[0], c[1] - h[1],
                                               c[2] - h[2], c[0] - h[0] + dx, c[1] - h[1] + dy,
                                               c[2] - h[2] + dz);
                    if (v > best) {
                        best = v;
                        bd[0] = dx, bd[1] = dy, bd[2] = dz;
                    }
                }
        for (int a = 0; a < 3; ++a) disp[3 * k + a] = (int32_t)bd[a];
        ncc[k] = best;
        conf[k] = best > 0.0 ? best : 0.0;
    }
    return 0;
}

/* NCC of the ref block at centers[k] and the flt block displaced by
   disp[k], per-axis block edges b[3]; NaN when either block leaves the
   volume. */
int oracle_ncc_aniso_at(const void *ref, const void *flt, int dtype, const int32_t dims[3],
                        const int32_t *centers, const int32_t *disp, int64_t n,
                        const int32_t b[3], double *out) {
    for (int a = 0; a < 3; ++a)
        if (b[a] < 1 || (b[a] % 2) == 0) return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < n; ++k) {
        int ok = 1;
        int64_t lo_r[3], lo_f[3];
        for (int a = 0; a < 3; ++a) {
            const int64_t h = (b[a] - 1) / 2;
            lo_r[a] = centers[3 * k + a] - h;
            lo_f[a] = lo_r[a] + disp[3 * k + a];
            if (lo_r[a] < 0 || lo_r[a] + b[a] > dims[a] || lo_f[a] < 0 || lo_f[a] + b[a] > dims[a])
                ok = 0;
        }
        out[k] = ok ? aniso_ncc(ref, flt, dtype, dims, b, lo_r[0], lo_r[1], lo_r[2], lo_f[0],
                                lo_f[1], lo_f[2])
                    : NAN;
    }
    return 0;
}

/* Cap the OpenMP threads of later oracle calls (timing on one core). */
void oracle_set_threads(int n) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int oracle_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
