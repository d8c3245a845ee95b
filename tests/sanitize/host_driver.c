/*
 * Host-only paths of the C-ABI under AddressSanitizer and UndefinedBehavior-
 * Sanitizer (no device work): the plan-time line factors of the wind and
 * product bispectra (the partial-bicoherence recursion, Section 4.1, on a
 * small grid), and argument validation that returns before any device call.
 * Exit status 0 when every call behaves as documented.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "srm3.h"

static int expect(srm3_status got, srm3_status want, const char *what)
{
    if (got != want) {
        fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, srm3_last_error());
        return 1;
    }
    return 0;
}

int main(void)
{
    const int nk = 12, nw = 16, W = 10, nc = 2 * nw - 1;
    const size_t n = (size_t)nk * nc;
    srm3_grid grid = {nk, nw, 0.05, 0.1, 32, 64};
    double *S = malloc(n * sizeof(double)), *c = malloc(n * sizeof(double)), *r = malloc(n * sizeof(double));
    double *sig = malloc(n * sizeof(double));
    double *F = malloc(2 * n * sizeof(double)), *G = malloc(2 * n * sizeof(double));
    double *H = malloc(2 * (size_t)(2 * W - 1) * (2 * W - 1) * sizeof(double));
    double *lc = malloc(2 * n * sizeof(double)), *lr = malloc(2 * n * sizeof(double));
    int bad = 0;
    for (int k = 0; k < nk; ++k)
        for (int j = 0; j < nc; ++j) {
            const double w = fabs((double)(j - (nw - 1))) * grid.d_omega, kap = k * grid.d_kappa;
            const size_t i = (size_t)k * nc + j;
            S[i] = j == nw - 1 ? 0.0 : 1.0 / ((1.0 + w) * (1.0 + w) * (0.2 + kap * kap + w));
            F[2 * i] = 0.3 * sqrt(S[i]);
            F[2 * i + 1] = 0.1 * sqrt(S[i]);
            G[2 * i] = sqrt(S[i]);
            G[2 * i + 1] = 0.0;
        }
    for (int i = 0; i < (2 * W - 1) * (2 * W - 1); ++i) {
        H[2 * i] = cos(0.01 * i);
        H[2 * i + 1] = sin(0.01 * i);
    }
    int sweeps = 0;
    bad |= expect(srm3_wind_factors(&grid, S, 0.5, 0.9, W, c, r, sig, &sweeps), SRM3_OK, "wind factors");
    for (size_t i = 0; i < n; ++i)
        if (!(sig[i] >= 0.0 && sig[i] < 1.0)) {
            fprintf(stderr, "wind Sigma[%zu] = %g\n", i, sig[i]);
            bad = 1;
            break;
        }
    bad |= expect(srm3_wind_factors(&grid, S, 0.5, 0.9, W, c, r, NULL, NULL), SRM3_OK, "wind factors, no Sigma");
    bad |= expect(srm3_product_factors(&grid, S, F, G, H, W, 0.9, lc, lr, sig, &sweeps), SRM3_OK, "product factors");
    bad |= expect(srm3_product_factors(&grid, S, F, G, NULL, W, 0.9, lc, lr, NULL, NULL), SRM3_OK,
                  "product factors, H = 1");
    /* argument errors, caught before any device work */
    bad |= expect(srm3_wind_factors(NULL, S, 0.5, 0.9, W, c, r, sig, NULL), SRM3_E_INVALID, "NULL grid");
    bad |= expect(srm3_wind_factors(&grid, S, 0.5, 0.9, nw + 1, c, r, sig, NULL), SRM3_E_INVALID, "support > n_omega");
    srm3_plan_t plan = NULL;
    srm3_spectrum spec = {S};
    srm3_grid bad_grid = grid;
    bad_grid.n_x = 48;
    bad |= expect(srm3_plan(&bad_grid, &spec, NULL, SRM3_FP64, NULL, &plan), SRM3_E_UNSUPPORTED, "n_x not a power of two");
    bad_grid = grid;
    bad_grid.n_kappa = 0;
    bad |= expect(srm3_plan(&bad_grid, &spec, NULL, SRM3_FP64, NULL, &plan), SRM3_E_INVALID, "n_kappa = 0");
    bad |= expect(srm3_plan(&grid, NULL, NULL, SRM3_FP64, NULL, &plan), SRM3_E_INVALID, "NULL spectrum");
    S[3] = -1.0;
    bad |= expect(srm3_plan(&grid, &spec, NULL, SRM3_FP64, NULL, &plan), SRM3_E_INVALID, "negative S");
    S[3] = 0.1;
    bad |= expect(srm3_plan(&grid, &spec, NULL, 7, NULL, &plan), SRM3_E_INVALID, "unknown precision");
    srm3_destroy(NULL);
    if (plan) bad = 1;
    free(S); free(c); free(r); free(sig); free(F); free(G); free(H); free(lc); free(lr);
    if (!bad) printf("host driver: ok (%d sweeps)\n", sweeps);
    return bad;
}
