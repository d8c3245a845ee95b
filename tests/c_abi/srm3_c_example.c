/*
 * The C-ABI used from plain C (no Python, no torch): the 32x64-line wave of
 * the test workloads -- spectrum evaluated on the device, separable
 * exponential bicoherence with a seeded biphase and a per-line cap -- one
 * realization generated into a hipMalloc'd buffer and written to a file as
 * FP64 [n_x][n_t].  Usage: srm3_c_example <seed> <out.bin>.  Exit status 0
 * on success; errors print srm3_last_error().
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "srm3.h"

#define CHECK(call)                                                                   \
    do {                                                                              \
        srm3_status s_ = (call);                                                      \
        if (s_ != SRM3_OK) {                                                          \
            fprintf(stderr, "%s failed: %d %s\n", #call, (int)s_, srm3_last_error()); \
            return 1;                                                                 \
        }                                                                             \
    } while (0)

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s <seed> <out.bin>\n", argv[0]);
        return 2;
    }
    const uint64_t seed = strtoull(argv[1], NULL, 10);
    const double pi = 3.14159265358979323846;
    srm3_grid grid = {32, 64, 2.0 * pi / (32 * 10.0), 4.0 * pi / 64, 64, 128};
    const int nc = 2 * grid.n_omega - 1, W = grid.n_omega;
    const size_t nlines = (size_t)grid.n_kappa * nc;

    /* spectrum on the lines, evaluated on the device, copied back for the plan */
    double *S_dev = NULL, *S = (double *)malloc(nlines * sizeof(double));
    if (hipMalloc((void **)&S_dev, nlines * sizeof(double)) != hipSuccess) return 1;
    srm3_kaimal_davenport kd = {1.5, 50.0, 30.0, 10.0};
    CHECK(srm3_spectrum_kaimal_davenport(&grid, &kd, S_dev, NULL));
    if (hipMemcpy(S, S_dev, nlines * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return 1;

    /* b^2_raw = 0.3 exp(-(|w1| + |w2|) / (0.5 w_u)), w_u = 4 pi */
    double *g2 = (double *)malloc((2 * W - 1) * sizeof(double));
    for (int i = -(W - 1); i <= W - 1; ++i)
        g2[i + W - 1] = sqrt(0.3) * exp(-fabs(i * grid.d_omega) / (0.5 * 4.0 * pi));
    srm3_bispectrum bis = {0};
    bis.kind = SRM3_BISPEC_SEPARABLE;
    bis.g2 = g2;
    bis.support_w = W;
    bis.cap = 0.9;
    bis.beta_mode = SRM3_BETA_SEEDED;
    bis.beta_seed = 0x5EEDB1FAull;
    srm3_spectrum spec = {S};
    srm3_plan_t plan = NULL;
    CHECK(srm3_plan(&grid, &spec, &bis, SRM3_FP64, NULL, &plan));

    const size_t npts = (size_t)grid.n_x * grid.n_t;
    double *u_dev = NULL, *u = (double *)malloc(npts * sizeof(double));
    if (hipMalloc((void **)&u_dev, npts * sizeof(double)) != hipSuccess) return 1;
    CHECK(srm3_generate(plan, &seed, 1, u_dev, NULL));
    if (hipMemcpy(u, u_dev, npts * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return 1;
    FILE *f = fopen(argv[2], "wb");
    if (!f || fwrite(u, sizeof(double), npts, f) != npts) return 1;
    fclose(f);
    srm3_destroy(plan);
    (void)hipFree(u_dev);
    (void)hipFree(S_dev);
    free(u);
    free(S);
    free(g2);
    printf("wrote %zu points\n", npts);
    return 0;
}
