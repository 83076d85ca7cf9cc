/*
 * Oracle: plain FP64 Gaussian attraction sums, written out from their
 * definition.  TEST INFRASTRUCTURE ONLY: the product library never links or
 * calls this file; only the tests, the smoke check and the bench's CPU
 * baseline do.
 *
 * The sum is the n-body form of the paper (section "Mathematical Formulation
 * of the Fast Multipole Method", Eq. (2)) with the Gaussian kernel of the
 * direct evaluation in the algorithm section (Eq. (8)):
 *
 *     u(t_i) = sum_j w_j * exp(-|t_i - s_j|^2 / sigma^2)
 *
 * w_j is the number of vacant dendritic elements of source j.  There is no
 * cutoff, libm exp is used, and the terms are added in source index order.
 * Positions arrive as the float32 inputs widened exactly to double.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC direct.c -o liboracle.so
 */
#include <math.h>
#include <stdint.h>
#include <omp.h>

/* u[i] for every target i; self[i] (if self != NULL) names one source index
 * that target i skips (-1 = none).  Returns 0, or -1 on bad arguments. */
int oracle_gauss_sum(int64_t nt, const double *tx, const double *ty, const double *tz,
                     const int64_t *self, int64_t ns, const double *sx, const double *sy,
                     const double *sz, const double *w, double sigma, double *u, int nthreads)
{
    if (nt < 0 || ns < 0 || !(sigma > 0.0)) return -1;
    const double s2 = sigma * sigma;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        const int64_t skip = self ? self[i] : -1;
        double acc = 0.0;
        for (int64_t j = 0; j < ns; ++j) {
            if (j == skip) continue;
            const double dx = tx[i] - sx[j];
            const double dy = ty[i] - sy[j];
            const double dz = tz[i] - sz[j];
            const double d2 = dx * dx + dy * dy + dz * dz;
            acc += w[j] * exp(-d2 / s2);
        }
        u[i] = acc;
    }
    return 0;
}

/* Derivatives of L = sum_i g_i u(t_i) by direct summation (for gradient
 * checks).  With K_ij = exp(-|t_i - s_j|^2 / sigma^2):
 *   dL/dw_j   = sum_i g_i K_ij
 *   dL/dt_i   = -(2 / sigma^2) g_i sum_j w_j K_ij (t_i - s_j)
 *   dL/ds_j   = (2 / sigma^2) w_j sum_i g_i K_ij (t_i - s_j)
 *   dL/dsigma = sum_ij g_i w_j K_ij * 2 |t_i - s_j|^2 / sigma^3
 * Target-side outputs (gt, length 3*nt, xyz interleaved) and the sigma
 * contribution of each target (gsig, length nt) come from a loop over
 * targets; gw and gs (lengths ns and 3*ns) from a loop over sources.  Any
 * output may be NULL. */
int oracle_gauss_grad(int64_t nt, const double *tx, const double *ty, const double *tz,
                      const double *g, int64_t ns, const double *sx, const double *sy,
                      const double *sz, const double *w, double sigma, double *gw,
                      double *gs, double *gt, double *gsig, int nthreads)
{
    if (nt < 0 || ns < 0 || !(sigma > 0.0)) return -1;
    const double s2 = sigma * sigma;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    if (gt || gsig) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < nt; ++i) {
            double ax = 0.0, ay = 0.0, az = 0.0, as = 0.0;
            for (int64_t j = 0; j < ns; ++j) {
                const double dx = tx[i] - sx[j];
                const double dy = ty[i] - sy[j];
                const double dz = tz[i] - sz[j];
                const double d2 = dx * dx + dy * dy + dz * dz;
                const double k = w[j] * exp(-d2 / s2);
                ax += k * dx;
                ay += k * dy;
                az += k * dz;
                as += k * d2;
            }
            if (gt) {
                gt[3 * i + 0] = -2.0 / s2 * g[i] * ax;
                gt[3 * i + 1] = -2.0 / s2 * g[i] * ay;
                gt[3 * i + 2] = -2.0 / s2 * g[i] * az;
            }
            if (gsig) gsig[i] = g[i] * as * 2.0 / (s2 * sigma);
        }
    }
    if (gw || gs) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t j = 0; j < ns; ++j) {
            double acc = 0.0, bx = 0.0, by = 0.0, bz = 0.0;
            for (int64_t i = 0; i < nt; ++i) {
                const double dx = tx[i] - sx[j];
                const double dy = ty[i] - sy[j];
                const double dz = tz[i] - sz[j];
                const double d2 = dx * dx + dy * dy + dz * dz;
                const double k = g[i] * exp(-d2 / s2);
                acc += k;
                bx += k * dx;
                by += k * dy;
                bz += k * dz;
            }
            if (gw) gw[j] = acc;
            if (gs) {
                gs[3 * j + 0] = 2.0 / s2 * w[j] * bx;
                gs[3 * j + 1] = 2.0 / s2 * w[j] * by;
                gs[3 * j + 2] = 2.0 / s2 * w[j] * bz;
            }
        }
    }
    return 0;
}
