/*
 * FP64 CPU oracle for grid-binned short-range pair interactions with a cutoff
 * radius (Algis, Bramas, Darles, Aveneau, "Efficient GPU Implementation of
 * Particle Interactions with Cutoff Radius and Few Particles per Cell",
 * arXiv 2406.16091).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * constant with the GPU path.
 *
 * What it computes (paper, Sec. 2 "Background" and Sec. 3 "Motivation and
 * Problem Statement"):
 *   - the cell of every particle from its position on a regular grid whose
 *     cell width is at least the cutoff (Sec. 3), X fastest (Fig. 1);
 *   - the number of particles per cell and its exclusive prefix sum with
 *     n_cells + 1 entries (Fig. 1);
 *   - the cell-sorted particle order (Sec. 2).  The paper places particles
 *     inside a cell with atomics (any order); this oracle fixes the order to
 *     ascending original index (a stable counting sort), which is the order
 *     the GPU path must reproduce bit for bit;
 *   - for every target i, the sum over all j != i with r_ij < r_c (Sec. 2) of
 *     a cubic B-spline kernel and its gradient, plus the neighbour count.
 *
 * The kernel is not printed in the paper (it names B-splines in Sec. 2 and
 * the cubic spline in Sec. 8).  The form used here is the cubic B-spline with
 * compact support h = r_c:
 *     q = r / h,  sigma = 8 / (pi h^3)
 *     W(q) = sigma (6 q^3 - 6 q^2 + 1)   for 0 <= q <= 1/2
 *     W(q) = 2 sigma (1 - q)^3           for 1/2 < q <= 1
 *     W(q) = 0                           for q > 1
 *   dW/dr = (sigma / h) (18 q^2 - 12 q)  for q <= 1/2
 *   dW/dr = -(6 sigma / h) (1 - q)^2     for 1/2 < q <= 1
 * For q > 1/2 the factor 1 - q is evaluated as (h^2 - r^2) / (h (h + r)),
 * the same number written so that it keeps its digits when r is close to h.
 *
 * Parity pins (tests/test_oracle_*.py): Fig. 1 worked binning example,
 * the Sec. 6 scan vectors, Table 1 first-column candidate counts, O(N^2)
 * brute force, closed-form kernel values, the kernel's unit integral,
 * finite-difference derivative, exact lattice arithmetic at the cutoff,
 * Newton's third law and statistical means.
 *
 * Precision: every float input is widened to double.  On inputs that lie on
 * a common power-of-two lattice (all workloads used here) the coordinate
 * differences and r^2 are exact in double, so the cutoff test r^2 < r_c^2 is
 * the exact real predicate.  The cell index follows the reading taken of the
 * paper's "cell from its physical position" (Sec. 2) together with its
 * statement that every computation is done in single precision (Sec. 7.1):
 * the axis index is a float32 decision, t = (x - o) / w with each operation
 * rounded to float32, cell = floor(t), and the particle is inside the box
 * iff 0 <= t < n on that axis.  Fig. 1's geometry, whose cell width is not a
 * power of two, pins it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ERANGE (-3)

/* The kernel function and its radial derivative (see the header comment). */
void oracle_kernel(double r, double h, double *W, double *dWdr)
{
    const double sigma = 8.0 / (M_PI * h * h * h);
    const double q = r / h;
    if (q <= 0.5) {
        *W = sigma * (6.0 * q * q * q - 6.0 * q * q + 1.0);
        *dWdr = (sigma / h) * (18.0 * q * q - 12.0 * q);
    } else if (q < 1.0) {
        const double omq = (h * h - r * r) / (h * (h + r)); /* = 1 - q */
        *W = 2.0 * sigma * omq * omq * omq;
        *dWdr = -(6.0 * sigma / h) * omq * omq;
    } else {
        *W = 0.0;
        *dWdr = 0.0;
    }
}

/* Same kernel, from r^2 (exact on lattice inputs) so that h^2 - r^2 is exact. */
static void kernel_from_d2(double d2, double h, double *W, double *dWdr, double *r_out)
{
    const double sigma = 8.0 / (M_PI * h * h * h);
    const double r = sqrt(d2);
    const double q = r / h;
    *r_out = r;
    if (q <= 0.5) {
        *W = sigma * (6.0 * q * q * q - 6.0 * q * q + 1.0);
        *dWdr = (sigma / h) * (18.0 * q * q - 12.0 * q);
    } else if (q < 1.0) {
        const double omq = (h * h - d2) / (h * (h + r)); /* = 1 - q */
        *W = 2.0 * sigma * omq * omq * omq;
        *dWdr = -(6.0 * sigma / h) * omq * omq;
    } else {
        *W = 0.0;
        *dWdr = 0.0;
    }
}

static int grid_ok(const int32_t dims[3], float cell_w, float rc)
{
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1) return 0;
    if (dims[0] > (1 << 24) || dims[1] > (1 << 24) || dims[2] > (1 << 24)) return 0;
    if ((int64_t)dims[0] * dims[1] * dims[2] >= ((int64_t)1 << 31)) return 0;
    if (!(cell_w > 0.0f) || !isfinite(cell_w)) return 0;
    if (!(rc > 0.0f) || !isfinite(rc)) return 0;
    if (cell_w < rc) return 0; /* cell width at least the cutoff (Sec. 3) */
    return 1;
}

/* One axis of the cell decision, in float32 (see the header comment). */
static int axis_cell(float x, float o, float w, int32_t n, int32_t *out)
{
    volatile float u = x - o;
    volatile float t = u / w;
    if (!(t >= 0.0f && t < (float)n)) return 0;
    *out = (int32_t)floorf(t);
    return 1;
}

/* Cell of every particle, X fastest: c = ix + nx (iy + ny iz) (Fig. 1).
 * Returns ORACLE_ERANGE if any particle lies outside the box; cell[i] is then
 * -1 for those particles. */
int oracle_cells(int64_t n, const float *x, const float *y, const float *z,
                 const float origin[3], const int32_t dims[3], float cell_w,
                 int32_t *cell)
{
    int status = ORACLE_OK;
    for (int64_t i = 0; i < n; ++i) {
        int32_t ix, iy, iz;
        if (axis_cell(x[i], origin[0], cell_w, dims[0], &ix) &&
            axis_cell(y[i], origin[1], cell_w, dims[1], &iy) &&
            axis_cell(z[i], origin[2], cell_w, dims[2], &iz)) {
            cell[i] = ix + dims[0] * (iy + dims[1] * iz);
        } else {
            cell[i] = -1;
            status = ORACLE_ERANGE;
        }
    }
    return status;
}

/*
 * Binning (Sec. 2): cell of each particle, per-cell counts, exclusive prefix
 * sum with n_cells + 1 entries (Fig. 1), and the stable scatter into the
 * cell-sorted order.  perm[k] is the original index of the k-th sorted
 * particle.  xs/ys/zs are the cell-relative float32 coordinates
 * fma(-ix, w, x - o) (one rounding), ws the weights in sorted order.
 * Any output pointer may be NULL except cell/counts/offsets.
 */
int oracle_bin(int64_t n, const float *x, const float *y, const float *z, const float *w,
               const float origin[3], const int32_t dims[3], float cell_w, float rc,
               int32_t *cell, int32_t *counts, int32_t *offsets, int32_t *perm,
               float *xs, float *ys, float *zs, float *ws, int32_t *max_per_cell)
{
    if (n < 0 || n >= ((int64_t)1 << 31)) return ORACLE_EINVAL;
    if (!grid_ok(dims, cell_w, rc)) return ORACLE_EINVAL;
    const int64_t nc = (int64_t)dims[0] * dims[1] * dims[2];

    int status = oracle_cells(n, x, y, z, origin, dims, cell_w, cell);
    if (status != ORACLE_OK) return status;

    memset(counts, 0, (size_t)nc * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) counts[cell[i]] += 1;

    int32_t mc = 0;
    offsets[0] = 0;
    for (int64_t c = 0; c < nc; ++c) {
        offsets[c + 1] = offsets[c] + counts[c];
        if (counts[c] > mc) mc = counts[c];
    }
    if (max_per_cell) *max_per_cell = mc;

    int32_t *cursor = (int32_t *)calloc((size_t)nc, sizeof(int32_t));
    if (!cursor) return ORACLE_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t c = cell[i];
        const int64_t k = (int64_t)offsets[c] + cursor[c]++;
        if (perm) perm[k] = (int32_t)i;
        const int32_t ix = c % dims[0];
        const int32_t iy = (c / dims[0]) % dims[1];
        const int32_t iz = c / (dims[0] * dims[1]);
        if (xs) xs[k] = fmaf(-(float)ix, cell_w, x[i] - origin[0]);
        if (ys) ys[k] = fmaf(-(float)iy, cell_w, y[i] - origin[1]);
        if (zs) zs[k] = fmaf(-(float)iz, cell_w, z[i] - origin[2]);
        if (ws) ws[k] = w[i];
    }
    free(cursor);
    return ORACLE_OK;
}

/*
 * Cell-list sweep (Sec. 2; Algorithm 1 gives the per-target loop): for each
 * requested target i, visit the 27 neighbour cells (dz, dy, dx) in
 * {-1, 0, 1}^3, clipped at the faces of the grid (no periodic images), and
 * every source j != i in them with r_ij < r_c.  Exact because cell_w >= r_c
 * (Sec. 3).  Inputs offsets/perm/cell come from oracle_bin.
 *
 * targets: original indices of the targets (NULL: all n, in index order).
 * Outputs are indexed by target position t:
 *   rho[t]   = sum_j w_j W(r_ij)
 *   g*[t]    = sum_{j, r_ij > 0} w_j W'(r_ij) (x_i - x_j) / r_ij
 *   ascale[t]= sum_j w_j |W'(r_ij)|   (condition scale of the gradient sums)
 *   count[t] = number of such j
 *   cand[t]  = number of j != i in the clipped 27-cell stencil (candidates)
 * Any of ascale/cand may be NULL.
 */
int oracle_sweep(int64_t n, const float *x, const float *y, const float *z, const float *w,
                 const int32_t dims[3], float rc,
                 const int32_t *cell, const int32_t *offsets, const int32_t *perm,
                 int64_t n_targets, const int64_t *targets,
                 double *rho, double *gx, double *gy, double *gz, double *ascale,
                 int64_t *count, int64_t *cand, int nthreads)
{
    if (n < 0) return ORACLE_EINVAL;
    const int64_t nt = targets ? n_targets : n;
    const double h = (double)rc;
    const double rc2 = (double)rc * (double)rc;
    const int32_t nx = dims[0], ny = dims[1], nz = dims[2];
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = targets ? targets[t] : t;
        const int32_t c = cell[i];
        const int32_t ix = c % nx, iy = (c / nx) % ny, iz = c / (nx * ny);
        const double xi = x[i], yi = y[i], zi = z[i];
        double r_rho = 0.0, r_gx = 0.0, r_gy = 0.0, r_gz = 0.0, r_a = 0.0;
        int64_t r_cnt = 0, r_cand = 0;
        for (int dz = -1; dz <= 1; ++dz) {
            const int32_t cz = iz + dz;
            if (cz < 0 || cz >= nz) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                const int32_t cy = iy + dy;
                if (cy < 0 || cy >= ny) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    const int32_t cx = ix + dx;
                    if (cx < 0 || cx >= nx) continue;
                    const int64_t nc = cx + (int64_t)nx * (cy + (int64_t)ny * cz);
                    for (int64_t k = offsets[nc]; k < offsets[nc + 1]; ++k) {
                        const int64_t j = perm[k];
                        if (j == i) continue;
                        r_cand += 1;
                        const double ddx = xi - (double)x[j];
                        const double ddy = yi - (double)y[j];
                        const double ddz = zi - (double)z[j];
                        const double d2 = ddx * ddx + ddy * ddy + ddz * ddz;
                        if (!(d2 < rc2)) continue;
                        double W, dW, r;
                        kernel_from_d2(d2, h, &W, &dW, &r);
                        const double wj = (double)w[j];
                        r_cnt += 1;
                        r_rho += wj * W;
                        r_a += wj * fabs(dW);
                        if (r > 0.0) {
                            const double f = wj * dW / r;
                            r_gx += f * ddx;
                            r_gy += f * ddy;
                            r_gz += f * ddz;
                        }
                    }
                }
            }
        }
        rho[t] = r_rho;
        gx[t] = r_gx;
        gy[t] = r_gy;
        gz[t] = r_gz;
        if (ascale) ascale[t] = r_a;
        count[t] = r_cnt;
        if (cand) cand[t] = r_cand;
    }
    return ORACLE_OK;
}

/*
 * The plain definition with no grid at all (Sec. 2: all pairs i != j with
 * r_ij < r_c), O(N^2).  Sources are visited in ascending original index.
 * Same output conventions as oracle_sweep (no candidate count).
 */
int oracle_brute(int64_t n, const float *x, const float *y, const float *z, const float *w,
                 float rc, int64_t n_targets, const int64_t *targets,
                 double *rho, double *gx, double *gy, double *gz, double *ascale,
                 int64_t *count, int nthreads)
{
    if (n < 0) return ORACLE_EINVAL;
    const int64_t nt = targets ? n_targets : n;
    const double h = (double)rc;
    const double rc2 = (double)rc * (double)rc;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = targets ? targets[t] : t;
        const double xi = x[i], yi = y[i], zi = z[i];
        double r_rho = 0.0, r_gx = 0.0, r_gy = 0.0, r_gz = 0.0, r_a = 0.0;
        int64_t r_cnt = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const double ddx = xi - (double)x[j];
            const double ddy = yi - (double)y[j];
            const double ddz = zi - (double)z[j];
            const double d2 = ddx * ddx + ddy * ddy + ddz * ddz;
            if (!(d2 < rc2)) continue;
            double W, dW, r;
            kernel_from_d2(d2, h, &W, &dW, &r);
            const double wj = (double)w[j];
            r_cnt += 1;
            r_rho += wj * W;
            r_a += wj * fabs(dW);
            if (r > 0.0) {
                const double f = wj * dW / r;
                r_gx += f * ddx;
                r_gy += f * ddy;
                r_gz += f * ddz;
            }
        }
        rho[t] = r_rho;
        gx[t] = r_gx;
        gy[t] = r_gy;
        gz[t] = r_gz;
        if (ascale) ascale[t] = r_a;
        count[t] = r_cnt;
    }
    return ORACLE_OK;
}

/*
 * The pair kernels of the paper's timing experiments (Sec. 7.1, Fig. 8),
 * evaluated on every candidate pair: every source j != i whose cell lies in
 * the clipped 27-cell neighbourhood of the target's cell.  The interactions
 * those experiments count are exactly these candidates (Table 1's first
 * column; the x axis of the performance figure is interactions computed per
 * particle), so no cutoff test is applied.
 *
 *   kind 1, Lennard-Jones with softening (Sec. 7.1): with
 *       u = sigma^2 / (r^2 + eps^2),
 *       K = 4 e0 (u^6 - u^3)        [= 4 e0 ((sigma/s)^12 - (sigma/s)^6),
 *                                     s^2 = r^2 + eps^2]
 *     and condition scale A = 4 e0 (u^6 + u^3) (sum of the magnitudes).
 *   kind 2, the low-FLOP kernel of Fig. 8, a sum of the positions:
 *       K = (x_i - x_j) + (y_i - y_j) + (z_i - z_j),
 *       A = |x_i - x_j| + |y_i - y_j| + |z_i - z_j|.
 *   kind 3, the high-FLOP kernel of Fig. 8, Lennard-Jones followed by 150
 *     more FLOP: 75 multiply-adds y <- y a + b on the Lennard-Jones value
 *     with run-time a = 1, b = 0 (so K and A equal those of kind 1).
 * v_i = sum_j K(i, j); a_i = sum_j A(i, j); cand_i = number of such j.
 */
#define PAIRFN_LJ 1
#define PAIRFN_LOWFLOP 2
#define PAIRFN_HIGHFLOP 3

typedef struct {
    double sigma, eps, e0; /* Lennard-Jones length, softening and depth */
    double a, b;           /* the high-FLOP kernel's multiply-add constants */
} pairfn_params;

static void pairfn_value(int kind, double dx, double dy, double dz, const pairfn_params *p,
                         double *K, double *A)
{
    if (kind == PAIRFN_LOWFLOP) {
        *K = dx + dy + dz;
        *A = fabs(dx) + fabs(dy) + fabs(dz);
        return;
    }
    const double s2 = dx * dx + dy * dy + dz * dz + p->eps * p->eps;
    const double u = p->sigma * p->sigma / s2;
    const double u3 = u * u * u;
    double k = 4.0 * p->e0 * (u3 * u3 - u3);
    *A = 4.0 * fabs(p->e0) * (u3 * u3 + u3);
    if (kind == PAIRFN_HIGHFLOP)
        for (int t = 0; t < 75; ++t) k = fma(k, p->a, p->b);
    *K = k;
}

/* Cell-list form: the 27 cells of each target in (dz, dy, dx) order, the
 * sources of a cell in sorted order (offsets/perm/cell from oracle_bin). */
int oracle_sweep_pairfn(int kind, int64_t n, const float *x, const float *y, const float *z,
                        const int32_t dims[3], double sigma, double eps, double e0,
                        const int32_t *cell, const int32_t *offsets, const int32_t *perm,
                        int64_t n_targets, const int64_t *targets,
                        double *v, double *ascale, int64_t *cand, int nthreads)
{
    if (n < 0 || kind < PAIRFN_LJ || kind > PAIRFN_HIGHFLOP) return ORACLE_EINVAL;
    const pairfn_params p = {sigma, eps, e0, 1.0, 0.0};
    const int64_t nt = targets ? n_targets : n;
    const int32_t nx = dims[0], ny = dims[1], nz = dims[2];
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = targets ? targets[t] : t;
        const int32_t c = cell[i];
        const int32_t ix = c % nx, iy = (c / nx) % ny, iz = c / (nx * ny);
        const double xi = x[i], yi = y[i], zi = z[i];
        double r_v = 0.0, r_a = 0.0;
        int64_t r_cand = 0;
        for (int dz = -1; dz <= 1; ++dz) {
            const int32_t cz = iz + dz;
            if (cz < 0 || cz >= nz) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                const int32_t cy = iy + dy;
                if (cy < 0 || cy >= ny) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    const int32_t cx = ix + dx;
                    if (cx < 0 || cx >= nx) continue;
                    const int64_t nc = cx + (int64_t)nx * (cy + (int64_t)ny * cz);
                    for (int64_t k = offsets[nc]; k < offsets[nc + 1]; ++k) {
                        const int64_t j = perm[k];
                        if (j == i) continue;
                        double K, A;
                        pairfn_value(kind, xi - (double)x[j], yi - (double)y[j], zi - (double)z[j], &p, &K, &A);
                        r_v += K;
                        r_a += A;
                        r_cand += 1;
                    }
                }
            }
        }
        v[t] = r_v;
        if (ascale) ascale[t] = r_a;
        if (cand) cand[t] = r_cand;
    }
    return ORACLE_OK;
}

/* The same sums from the definition with no cell list: every j != i whose
 * cell (oracle_cells) differs from the target's by at most one on each axis,
 * sources in ascending original index.  O(N^2). */
int oracle_brute_pairfn(int kind, int64_t n, const float *x, const float *y, const float *z,
                        const int32_t dims[3], double sigma, double eps, double e0, const int32_t *cell,
                        int64_t n_targets, const int64_t *targets,
                        double *v, double *ascale, int64_t *cand, int nthreads)
{
    if (n < 0 || kind < PAIRFN_LJ || kind > PAIRFN_HIGHFLOP) return ORACLE_EINVAL;
    const pairfn_params p = {sigma, eps, e0, 1.0, 0.0};
    const int64_t nt = targets ? n_targets : n;
    const int32_t nx = dims[0], ny = dims[1];
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = targets ? targets[t] : t;
        const int32_t ix = cell[i] % nx, iy = (cell[i] / nx) % ny, iz = cell[i] / (nx * ny);
        const double xi = x[i], yi = y[i], zi = z[i];
        double r_v = 0.0, r_a = 0.0;
        int64_t r_cand = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            const int32_t jx = cell[j] % nx, jy = (cell[j] / nx) % ny, jz = cell[j] / (nx * ny);
            if (abs(jx - ix) > 1 || abs(jy - iy) > 1 || abs(jz - iz) > 1) continue;
            double K, A;
            pairfn_value(kind, xi - (double)x[j], yi - (double)y[j], zi - (double)z[j], &p, &K, &A);
            r_v += K;
            r_a += A;
            r_cand += 1;
        }
        v[t] = r_v;
        if (ascale) ascale[t] = r_a;
        if (cand) cand[t] = r_cand;
    }
    return ORACLE_OK;
}

/* Number of OpenMP threads a parallel region started now would use. */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
