/* The oracle's direct sums (oracle/direct.c, compiled into this program) run
 * under AddressSanitizer and UndefinedBehaviorSanitizer on small inputs: every
 * array access of the sums and derivatives, and the argument checks. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_gauss_sum(int64_t nt, const double *tx, const double *ty, const double *tz,
                     const int64_t *self, int64_t ns, const double *sx, const double *sy,
                     const double *sz, const double *w, double sigma, double *u, int nthreads);
int oracle_gauss_grad(int64_t nt, const double *tx, const double *ty, const double *tz,
                      const double *g, int64_t ns, const double *sx, const double *sy,
                      const double *sz, const double *w, double sigma, double *gw, double *gs,
                      double *gt, double *gsig, int nthreads);

static double *draw(int64_t n, double scale) {
    double *a = malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int64_t i = 0; i < n; ++i) a[i] = scale * (double)rand() / RAND_MAX;
    return a;
}

int main(void) {
    int fails = 0;
    srand(7);
    const int64_t sizes[][2] = {{1, 1}, {3, 0}, {0, 5}, {37, 53}, {128, 7}};
    for (int c = 0; c < 5; ++c) {
        const int64_t nt = sizes[c][0], ns = sizes[c][1];
        double *tx = draw(nt, 100), *ty = draw(nt, 100), *tz = draw(nt, 100), *g = draw(nt, 1);
        double *sx = draw(ns, 100), *sy = draw(ns, 100), *sz = draw(ns, 100), *w = draw(ns, 5);
        int64_t *self = malloc((size_t)(nt > 0 ? nt : 1) * sizeof(int64_t));
        for (int64_t i = 0; i < nt; ++i) self[i] = ns > 0 ? i % ns : -1;
        double *u = draw(nt, 0), *gw = draw(ns, 0), *gs = draw(3 * ns, 0), *gt = draw(3 * nt, 0),
               *gsig = draw(nt, 0);
        if (oracle_gauss_sum(nt, tx, ty, tz, self, ns, sx, sy, sz, w, 30.0, u, 2) != 0) ++fails;
        for (int64_t i = 0; i < nt; ++i)
            if (!isfinite(u[i]) || u[i] < 0) ++fails;
        if (oracle_gauss_grad(nt, tx, ty, tz, g, ns, sx, sy, sz, w, 30.0, gw, gs, gt, gsig, 2) != 0) ++fails;
        if (oracle_gauss_grad(nt, tx, ty, tz, g, ns, sx, sy, sz, w, 30.0, NULL, NULL, NULL, NULL, 1) != 0) ++fails;
        free(tx); free(ty); free(tz); free(g); free(sx); free(sy); free(sz); free(w); free(self);
        free(u); free(gw); free(gs); free(gt); free(gsig);
    }
    double one = 1.0, out = 0.0;
    if (oracle_gauss_sum(-1, &one, &one, &one, NULL, 1, &one, &one, &one, &one, 1.0, &out, 1) == 0) ++fails;
    if (oracle_gauss_sum(1, &one, &one, &one, NULL, 1, &one, &one, &one, &one, 0.0, &out, 1) == 0) ++fails;
    printf("%d failures\n", fails);
    return fails != 0;
}
