/*
 * The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
 * every entry point on small grids (phases, biphase, line terms and
 * coefficients for the table, wind, product and per-pair modes, the three
 * field sums, the 1-D process).  Exit status 0 when all calls succeed.
 * Links oracle/srm3_oracle.c; the problem structs are restated here in the
 * layout that file defines.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int nk, nw, W;
    double dk, dw;
    const double *S, *b2;
    const uint32_t *beta;
    double cap;
    const double *line_c, *line_r;
    int mode;
    double alpha;
    double *Sp;
    const double *F, *G, *H;
    uint64_t hash_key;
} problem;

typedef struct {
    int n, W;
    double dw;
    const double *S, *b2;
    const uint32_t *beta;
    double cap;
} process;

void oracle_phases(int nk, int nw, uint64_t seed, uint32_t *U);
void oracle_biphase(int W, int mode, uint64_t beta_seed, uint32_t *beta);
int oracle_coefficients(const problem *p, const uint32_t *U, long nlines, const long *lines, double *C);
int oracle_wind_solve(problem *p, double *Sp, int max_iter, double tol);
void oracle_field_flat(int nk, int nw, int nx, int nt, const double *C, double *u);
void oracle_field_nested(int nk, int nw, int nx, int nt, const double *C, double *u);
void oracle_field_points(int nk, int nw, int nx, int nt, const double *C, long npts, const int *mx, const int *mt,
                         double *u);
void oracle_process_phases(int n, uint64_t seed, uint32_t *U);
void oracle_process_biphase(int W, int mode, uint64_t beta_seed, uint32_t *beta);
int oracle_process_coefficients(const process *p, const uint32_t *U, double *C);
void oracle_process_field(int n, int nt, const double *C, double *u);

int main(void)
{
    const int nk = 6, nw = 9, W = 7, nc = 2 * nw - 1, nwc = 2 * W - 1, nx = 16, nt = 32;
    const long nl = (long)nk * nc;
    double *S = malloc(nl * sizeof(double)), *b2 = malloc((size_t)nwc * nwc * sizeof(double));
    double *Sp = malloc(nl * sizeof(double)), *C = malloc(2 * nl * sizeof(double));
    double *F = malloc(2 * nl * sizeof(double)), *G = malloc(2 * nl * sizeof(double));
    double *u = malloc((size_t)nx * nt * sizeof(double)), *v = malloc((size_t)nx * nt * sizeof(double));
    uint32_t *U = malloc(nl * sizeof(uint32_t)), *beta = malloc((size_t)nwc * nwc * sizeof(uint32_t));
    long *lines = malloc(nl * sizeof(long));
    int bad = 0;
    for (long i = 0; i < nl; ++i) {
        const int kw = (int)(i % nc) - (nw - 1);
        S[i] = kw == 0 ? 0.0 : 1.0 / (1.0 + fabs((double)kw) + 0.3 * (double)(i / nc));
        F[2 * i] = 0.2 * sqrt(S[i]);
        F[2 * i + 1] = -0.1 * sqrt(S[i]);
        G[2 * i] = sqrt(S[i]);
        G[2 * i + 1] = 0.05;
        lines[i] = i;
    }
    for (int i = 0; i < nwc * nwc; ++i) b2[i] = 0.01 * (1.0 + (i % 5));
    oracle_phases(nk, nw, 7, U);
    oracle_biphase(W, 0, 11, beta);
    for (int mode = 0; mode < 4; ++mode) {
        problem p = {nk, nw, W, 0.1, 0.2, S, b2, beta, 0.9, NULL, NULL, mode, 0.3, Sp, F, G, NULL, 99};
        for (long i = 0; i < nl; ++i) Sp[i] = S[i];
        if ((mode == 1 || mode == 2) && oracle_wind_solve(&p, Sp, 200, 1e-14) < 0) bad = 1;
        if (oracle_coefficients(&p, U, nl, lines, C) != 0) bad = 1;
        for (long i = 0; i < 2 * nl; ++i)
            if (!isfinite(C[i])) bad = 1;
    }
    oracle_field_flat(nk, nw, nx, nt, C, u);
    oracle_field_nested(nk, nw, nx, nt, C, v);
    for (int i = 0; i < nx * nt; ++i)
        if (fabs(u[i] - v[i]) > 1e-9 * (1.0 + fabs(u[i]))) bad = 1;
    int mx[3] = {0, 5, nx - 1}, mt[3] = {0, 7, nt - 1};
    oracle_field_points(nk, nw, nx, nt, C, 3, mx, mt, v);
    const int n = 12, Wp = 8;
    double *Sq = malloc(n * sizeof(double)), *bq = malloc((size_t)Wp * Wp * sizeof(double));
    double *Cq = malloc(2 * (size_t)n * sizeof(double)), *uq = malloc(32 * sizeof(double));
    uint32_t *Uq = malloc(n * sizeof(uint32_t)), *betaq = malloc((size_t)Wp * Wp * sizeof(uint32_t));
    for (int i = 0; i < n; ++i) Sq[i] = i == 0 ? 0.0 : 1.0 / (1.0 + i);
    for (int i = 0; i < Wp * Wp; ++i) bq[i] = 0.02;
    oracle_process_phases(n, 5, Uq);
    oracle_process_biphase(Wp, 0, 3, betaq);
    process q = {n, Wp, 0.3, Sq, bq, betaq, 0.9};
    if (oracle_process_coefficients(&q, Uq, Cq) != 0) bad = 1;
    oracle_process_field(n, 32, Cq, uq);
    free(S); free(b2); free(Sp); free(C); free(F); free(G); free(u); free(v); free(U); free(beta); free(lines);
    free(Sq); free(bq); free(Cq); free(uq); free(Uq); free(betaq);
    if (!bad) printf("oracle driver: ok\n");
    return bad;
}
