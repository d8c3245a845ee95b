/*
 * FP64 CPU oracle for the 3rd-order Spectral Representation Method (SRM) for
 * 1-D stochastic waves u(x, t) (Vandanapu & Shields, Section 4.1 and 4.3).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may build, load or call this file.  It shares
 * no code, header, table or constant generator with the GPU library.
 *
 * It is deliberately plain: every coefficient is built by enumerating the set
 * of interacting line pairs explicitly and calling libm cos/sin on the summed
 * angle; the field is a direct cosine sum.  Everything is IEEE FP64.
 *
 * Definitions (readings of the paper are listed in the design notes):
 *  - Lines: k = (kk, kw) with 0 <= kk < NK and -NW < kw < NW (signed frequency,
 *    half-plane kappa >= 0, Section 2 symmetries).  Line value S_k = S(kappa, omega).
 *  - Phase of line k: phi_k = 2 pi U_k / 2^32.  One Philox4x32-10 call (key =
 *    realization seed) serves four consecutive frequencies of a row: U_k is
 *    word r of counter (kk, q as uint32, 0, 0), kw = 4 q + r, 0 <= r < 4
 *    (q = floor(kw / 4)).
 *  - Biphase: beta(iw, jw) = 2 pi V / 2^32, V = Philox word 0 with key = beta
 *    seed, counter = (max(iw,jw), min(iw,jw), 1, 0) -- symmetric in (iw, jw).
 *  - P(k): unordered pairs {i, j} of lines with i + j = k (both components),
 *    |iw| < W and |jw| < W, self pair i = j included, each pair once
 *    (Eq. truncated_cosines_1d_wave, read as "each unordered pair once").
 *  - rho_k = min(1, cap / sum_{P(k)} b2_raw) (cap > 0), b_p^2 = rho_k b2_raw,
 *    Sigma_k = sum_{P(k)} b_p^2, pure part sqrt(1 - Sigma_k) (Eq. pure with b_p^2).
 *  - C_k = 2 sqrt(S_k dk dw) [ sqrt(1 - Sigma_k) e^{i phi_k}
 *          + sum_{p in P(k)} b_p e^{i (phi_i + phi_j + beta_p)} ]   (Section 4.3)
 *  - u(mx, mt) = sum_k Re[ C_k exp(2 pi i (kk mx / NX + kw mt / NT)) ]
 *    (Section 4.3 with dk dx = 2 pi / NX, dw dt = 2 pi / NT).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TWO_PI 6.283185307179586476925286766559

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the published description (Salmon, Moraes, Dror and   */
/* Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of */
/* two 32x32->64 multiplies with key-dependent xors, a Weyl key schedule.     */
/* ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                          uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static uint32_t philox_word0(uint32_t c0, uint32_t c1, uint32_t c2, uint64_t key)
{
    uint32_t ctr[4] = {c0, c1, c2, 0u};
    uint32_t k[2] = {(uint32_t)(key & 0xffffffffu), (uint32_t)(key >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, k, out);
    return out[0];
}

/* Fixed-point phase of line (kk, kw): word r of the Philox call with counter
 * (kk, q, 0, 0), where kw = 4 q + r with 0 <= r < 4 (floor division, also for
 * negative kw). */
static uint32_t phase_word(int kk, int kw, uint64_t seed)
{
    const int q = kw >= 0 ? kw / 4 : -((3 - kw) / 4);
    const int r = kw - 4 * q;
    uint32_t ctr[4] = {(uint32_t)kk, (uint32_t)(int32_t)q, 0u, 0u};
    uint32_t k[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, k, out);
    return out[r];
}

/* Random phase angles (fixed point, 2^32 == 2 pi) of every line, [nk][2nw-1]. */
void oracle_phases(int nk, int nw, uint64_t seed, uint32_t *U)
{
    const int nc = 2 * nw - 1;
#pragma omp parallel for schedule(static)
    for (int kk = 0; kk < nk; ++kk)
        for (int kw = -(nw - 1); kw <= nw - 1; ++kw)
            U[(size_t)kk * nc + (kw + nw - 1)] = phase_word(kk, kw, seed);
}

/* Biphase table (fixed point) over signed frequency indices |iw|,|jw| < W,
 * [2W-1][2W-1], symmetric.  mode 0: drawn from the seed; mode 1: zero. */
void oracle_biphase(int W, int mode, uint64_t beta_seed, uint32_t *beta)
{
    const int n = 2 * W - 1;
#pragma omp parallel for schedule(static)
    for (int iw = -(W - 1); iw <= W - 1; ++iw)
        for (int jw = -(W - 1); jw <= W - 1; ++jw) {
            uint32_t v = 0u;
            if (mode == 0) {
                int hi = iw >= jw ? iw : jw, lo = iw >= jw ? jw : iw;
                v = philox_word0((uint32_t)(int32_t)hi, (uint32_t)(int32_t)lo, 1u, beta_seed);
            }
            beta[(size_t)(iw + W - 1) * n + (jw + W - 1)] = v;
        }
}

typedef struct {
    int nk, nw, W;
    double dk, dw;
    const double *S;        /* [nk][2nw-1] */
    const double *b2;       /* [2W-1][2W-1] raw squared bicoherence */
    const uint32_t *beta;   /* [2W-1][2W-1] fixed-point biphase */
    double cap;             /* > 0: per-line cap on sum b^2; <= 0: none */
    /* kappa-dependent bicoherence (NULL / 0 = off):
     *  line_c, line_r [nk][2nw-1]: b2_raw(i, j -> k) = c_k^2 r_i^2 r_j^2 b2(iw, jw);
     *  mode 1: the wind bispectrum of Section 5 (Eq. bispectrum, scaled by
     *  alpha, beta = 0) through the partial bicoherence of Section 4.1,
     *  b_p^2 = |B|^2 dk dw / (S_p,i S_p,j S_k), with S_p from Sp [nk][2nw-1].
     *  mode 2: a prescribed product bispectrum B(i, j) = F_k G_i G_j H(i_w, j_w)
     *  (complex, interleaved re/im; H may be NULL = 1) through the same partial
     *  bicoherence, with beta = atan2(Im B, Re B). */
    const double *line_c;
    const double *line_r;
    int mode;
    double alpha;
    const double *Sp;
    const double *F;        /* mode 2: [nk][2nw-1] complex */
    const double *G;        /* mode 2: [nk][2nw-1] complex */
    const double *H;        /* mode 2: [2W-1][2W-1] complex, or NULL */
    uint64_t hash_key;      /* mode 3: a bispectrum drawn per 4-index pair (see pair_words) */
} oracle_problem;

/* Mode 3: the two 8-bit draws of the canonical pair (i, j), k = i + j.
 * Philox4x32-10 with key = hash_key and counter (i_kappa, m, j_kappa, k_w),
 * m = floor(i_w / 8), holds the eight pairs of line k whose i_w share m: pair
 * t = i_w - 8 m takes the 16-bit half h of word floor(t / 2) (the high half
 * for even t, the low half for odd t), split into u = h >> 8 (the
 * bicoherence) and v = h & 255 (the biphase). */
static void pair_words(const oracle_problem *p, int ik, int iw, int jk, int jw, uint32_t *u, uint32_t *v)
{
    const int m = iw >= 0 ? iw / 8 : -((-iw + 7) / 8);
    const int t = iw - 8 * m;
    const uint32_t ctr[4] = {(uint32_t)ik, (uint32_t)(int32_t)m, (uint32_t)jk, (uint32_t)(int32_t)(iw + jw)};
    const uint32_t key[2] = {(uint32_t)(p->hash_key & 0xffffffffu), (uint32_t)(p->hash_key >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    const uint32_t w = out[t / 2];
    const uint32_t h = (t % 2 == 0) ? (w >> 16) : (w & 0xffffu);
    *u = h >> 8;
    *v = h & 0xffu;
}

/* The prescribed product bispectrum B(i, j) = F_k G_i G_j H(i_w, j_w). */
static void product_B(const oracle_problem *p, int ik, int iw, int jk, int jw, double *re, double *im)
{
    const int nc = 2 * p->nw - 1, W = p->W, n = 2 * W - 1;
    const size_t li = (size_t)ik * nc + iw + p->nw - 1, lj = (size_t)jk * nc + jw + p->nw - 1;
    const size_t lk = (size_t)(ik + jk) * nc + iw + jw + p->nw - 1;
    double r = p->F[2 * lk], m = p->F[2 * lk + 1];
    double t;
    t = r * p->G[2 * li] - m * p->G[2 * li + 1]; m = r * p->G[2 * li + 1] + m * p->G[2 * li]; r = t;
    t = r * p->G[2 * lj] - m * p->G[2 * lj + 1]; m = r * p->G[2 * lj + 1] + m * p->G[2 * lj]; r = t;
    if (p->H) {
        const size_t e = (size_t)(iw + W - 1) * n + (jw + W - 1);
        t = r * p->H[2 * e] - m * p->H[2 * e + 1]; m = r * p->H[2 * e + 1] + m * p->H[2 * e]; r = t;
    }
    *re = r;
    *im = m;
}

/* The wind bispectrum (Section 5, Eq. bispectrum) between lines i and j,
 * scaled by alpha, with |omega_i + omega_j| under the root (the half-plane
 * kappa >= 0 holds negative frequencies too; S is even in omega) and zero
 * where it is singular (omega_k = 0 or kappa_k = 0). */
static double wind_B(const oracle_problem *p, int ik, int iw, int jk, int jw)
{
    const int nc = 2 * p->nw - 1;
    const int kk = ik + jk, kw = iw + jw;
    if (kk == 0 || kw == 0) return 0.0;
    const double Si = p->S[(size_t)ik * nc + iw + p->nw - 1];
    const double Sj = p->S[(size_t)jk * nc + jw + p->nw - 1];
    const double Sk = p->S[(size_t)kk * nc + kw + p->nw - 1];
    const double wk = fabs((double)kw * p->dw), kap = (double)kk * p->dk;
    return p->alpha * 2.0 * sqrt(Si * Sj * Sk) / (3.0 * sqrt(3.0 * wk * kap));
}

/* Squared bicoherence of the pair {i, j} before the per-line cap. */
static double pair_b2(const oracle_problem *p, int ik, int iw, int jk, int jw)
{
    const int W = p->W, n = 2 * W - 1, nc = 2 * p->nw - 1;
    const size_t li = (size_t)ik * nc + iw + p->nw - 1, lj = (size_t)jk * nc + jw + p->nw - 1;
    const size_t lk = (size_t)(ik + jk) * nc + iw + jw + p->nw - 1;
    if (p->mode == 1) {
        const double B = wind_B(p, ik, iw, jk, jw);
        if (B == 0.0) return 0.0;
        return B * B * p->dk * p->dw / (p->Sp[li] * p->Sp[lj] * p->S[lk]);
    }
    if (p->mode == 3) {   /* b_p = sqrt(alpha) u / 2^8, so b_p^2 = alpha (u / 2^8)^2 */
        uint32_t u, v;
        pair_words(p, ik, iw, jk, jw, &u, &v);
        const double b = (double)u / 256.0;
        return p->alpha * b * b;
    }
    if (p->mode == 2) {
        double re, im;
        product_B(p, ik, iw, jk, jw, &re, &im);
        const double B2 = re * re + im * im;
        if (B2 == 0.0 || p->S[lk] <= 0.0 || p->Sp[li] <= 0.0 || p->Sp[lj] <= 0.0) return 0.0;
        return B2 * p->dk * p->dw / (p->Sp[li] * p->Sp[lj] * p->S[lk]);
    }
    double v = p->b2[(size_t)(iw + W - 1) * n + (jw + W - 1)];
    if (p->line_c) v *= p->line_c[lk] * p->line_c[lk];
    if (p->line_r) v *= p->line_r[li] * p->line_r[li] * p->line_r[lj] * p->line_r[lj];
    return v;
}

static uint32_t pair_beta(const oracle_problem *p, int ik, int iw, int jk, int jw)
{
    const int W = p->W, n = 2 * W - 1;
    if (p->mode == 3) {   /* beta = 2 pi v / 2^8: the fixed-point angle v 2^24 */
        uint32_t u, v;
        pair_words(p, ik, iw, jk, jw, &u, &v);
        return v << 24;
    }
    return p->mode != 0 ? 0u : p->beta[(size_t)(iw + W - 1) * n + (jw + W - 1)];
}

/* Biphase of a prescribed product bispectrum, in radians. */
static double pair_beta_rad(const oracle_problem *p, int ik, int iw, int jk, int jw)
{
    if (p->mode != 2) return 0.0;
    double re, im;
    product_B(p, ik, iw, jk, jw, &re, &im);
    return atan2(im, re);
}

/* Is the pair (i, j), i + j = k, the canonical member of its unordered pair? */
static int canonical(int ik, int iw, int jk, int jw)
{
    return (ik > jk) || (ik == jk && iw >= jw);
}

/* Enumerate P(k) and return the raw bicoherence sum and the pair count. */
static double raw_sum(const oracle_problem *p, int kk, int kw, long *npairs)
{
    const int W = p->W;
    double s = 0.0;
    long cnt = 0;
    for (int ik = 0; ik <= kk; ++ik) {
        const int jk = kk - ik;
        for (int iw = -(W - 1); iw <= W - 1; ++iw) {
            const int jw = kw - iw;
            if (jw <= -W || jw >= W) continue;
            if (!canonical(ik, iw, jk, jw)) continue;
            s += pair_b2(p, ik, iw, jk, jw);
            ++cnt;
        }
    }
    if (npairs) *npairs = cnt;
    return s;
}

/* Per-line quantities: raw sum, rescale factor rho, Sigma, pair count.
 * Returns 0, or 2 if Sigma_k >= 1 (pure spectrum not positive). */
int oracle_line_terms(const oracle_problem *p, int kk, int kw, double *sigma_raw,
                      double *rho, double *sigma, long *npairs)
{
    double sr = raw_sum(p, kk, kw, npairs);
    double r = 1.0;
    if (p->cap > 0.0 && sr > p->cap) r = p->cap / sr;
    if (sigma_raw) *sigma_raw = sr;
    if (rho) *rho = r;
    if (sigma) *sigma = r * sr;
    return (r * sr >= 1.0) ? 2 : 0;
}

/* Coefficients C_k for the given lines (flat index kk*(2nw-1) + kw + nw - 1),
 * output interleaved re/im.  U: phases of this realization [nk][2nw-1]. */
int oracle_coefficients(const oracle_problem *p, const uint32_t *U, long nlines,
                        const long *lines, double *C)
{
    const int nw = p->nw, nc = 2 * nw - 1, W = p->W;
    int status = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(max : status)
    for (long q = 0; q < nlines; ++q) {
        const long flat = lines[q];
        const int kk = (int)(flat / nc), kw = (int)(flat % nc) - (nw - 1);
        double rho, sigma;
        int st = oracle_line_terms(p, kk, kw, NULL, &rho, &sigma, NULL);
        if (st) { status = st; C[2 * q] = NAN; C[2 * q + 1] = NAN; continue; }
        const double S = p->S[flat];
        const double amp = 2.0 * sqrt(S * p->dk * p->dw);
        const double phik = TWO_PI * (double)U[flat] / 4294967296.0;
        double re = sqrt(1.0 - sigma) * cos(phik);
        double im = sqrt(1.0 - sigma) * sin(phik);
        for (int ik = 0; ik <= kk; ++ik) {
            const int jk = kk - ik;
            for (int iw = -(W - 1); iw <= W - 1; ++iw) {
                const int jw = kw - iw;
                if (jw <= -W || jw >= W) continue;
                if (!canonical(ik, iw, jk, jw)) continue;
                const double bp = sqrt(rho * pair_b2(p, ik, iw, jk, jw));
                const uint32_t ang = U[(size_t)ik * nc + (iw + nw - 1)]
                                   + U[(size_t)jk * nc + (jw + nw - 1)]
                                   + pair_beta(p, ik, iw, jk, jw);  /* exact mod 2^32 */
                const double th = TWO_PI * (double)ang / 4294967296.0 + pair_beta_rad(p, ik, iw, jk, jw);
                re += bp * cos(th);
                im += bp * sin(th);
            }
        }
        C[2 * q] = amp * re;
        C[2 * q + 1] = amp * im;
    }
    return status;
}

/* Partial-bicoherence recursion of Section 4.1 for the wind bispectrum: the
 * pure spectrum S_p = S (1 - Sigma) enters the bicoherence of every pair that
 * builds on a line, so S_p is the solution of a fixed point.  Plain Jacobi
 * sweeps from S_p = S (Sigma = 0): each sweep recomputes every line's Sigma
 * (cap applied) from the previous S_p by enumerating P(k).  Sigma grows
 * monotonically and converges to the least solution.  Sp (in/out) is the
 * problem's own array.  Returns the sweep count, or -2 if an uncapped Sigma
 * reaches 1 (no admissible pure spectrum), -1 if not converged in max_iter. */
int oracle_wind_solve(oracle_problem *p, double *Sp, int max_iter, double tol)
{
    const int nk = p->nk, nw = p->nw, nc = 2 * nw - 1;
    const size_t nl = (size_t)nk * nc;
    double *next = (double *)malloc(sizeof(double) * nl);
    for (size_t l = 0; l < nl; ++l) Sp[l] = p->S[l];
    if (p->mode != 2) p->mode = 1;   /* mode 2: the caller's product bispectrum */
    p->Sp = Sp;
    int it;
    for (it = 1; it <= max_iter; ++it) {
        int bad = 0;
        double diff = 0.0;
#pragma omp parallel for schedule(dynamic, 4) reduction(max : diff) reduction(| : bad)
        for (long l = 0; l < (long)nl; ++l) {
            const int kk = (int)(l / nc), kw = (int)(l % nc) - (nw - 1);
            double sigma;
            if (oracle_line_terms(p, kk, kw, NULL, NULL, &sigma, NULL)) { bad = 1; next[l] = 0.0; continue; }
            next[l] = p->S[l] * (1.0 - sigma);
            const double d = fabs(next[l] - Sp[l]) / (p->S[l] > 0.0 ? p->S[l] : 1.0);
            if (d > diff) diff = d;
        }
        if (bad) { free(next); return -2; }
        for (size_t l = 0; l < nl; ++l) Sp[l] = next[l];
        if (diff <= tol) break;
    }
    free(next);
    return it > max_iter ? -1 : it;
}

static long long posmod(long long a, long long m)
{
    long long r = a % m;
    return r < 0 ? r + m : r;
}

/* Direct cosine sum at every grid point (flat form), u: [nx][nt]. */
void oracle_field_flat(int nk, int nw, int nx, int nt, const double *C, double *u)
{
    const int nc = 2 * nw - 1;
    const long long M = (long long)nx * nt;
#pragma omp parallel for schedule(static)
    for (int mx = 0; mx < nx; ++mx)
        for (int mt = 0; mt < nt; ++mt) {
            double acc = 0.0;
            for (int kk = 0; kk < nk; ++kk)
                for (int kw = -(nw - 1); kw <= nw - 1; ++kw) {
                    const size_t f = (size_t)kk * nc + (kw + nw - 1);
                    const long long a = posmod((long long)kk * mx * nt + (long long)kw * mt * nx, M);
                    const double th = TWO_PI * (double)a / (double)M;
                    acc += C[2 * f] * cos(th) - C[2 * f + 1] * sin(th);
                }
            u[(size_t)mx * nt + mt] = acc;
        }
}

/* Direct cosine sum at selected points (flat form). */
void oracle_field_points(int nk, int nw, int nx, int nt, const double *C, long npts,
                         const int *mx, const int *mt, double *u)
{
    const int nc = 2 * nw - 1;
    const long long M = (long long)nx * nt;
#pragma omp parallel for schedule(static)
    for (long q = 0; q < npts; ++q) {
        double acc = 0.0;
        for (int kk = 0; kk < nk; ++kk)
            for (int kw = -(nw - 1); kw <= nw - 1; ++kw) {
                const size_t f = (size_t)kk * nc + (kw + nw - 1);
                const long long a = posmod((long long)kk * mx[q] * nt + (long long)kw * mt[q] * nx, M);
                const double th = TWO_PI * (double)a / (double)M;
                acc += C[2 * f] * cos(th) - C[2 * f + 1] * sin(th);
            }
        u[q] = acc;
    }
}

/* The same sum in nested order: first over kw for every (kk, mt), then over
 * kk.  Angles are reduced exactly in integers before scaling. */
void oracle_field_nested(int nk, int nw, int nx, int nt, const double *C, double *u)
{
    const int nc = 2 * nw - 1;
    double *G = (double *)malloc(sizeof(double) * 2 * (size_t)nk * nt);
    double *ct = (double *)malloc(sizeof(double) * (size_t)nt);
    double *st = (double *)malloc(sizeof(double) * (size_t)nt);
    double *cx = (double *)malloc(sizeof(double) * (size_t)nx);
    double *sx = (double *)malloc(sizeof(double) * (size_t)nx);
    for (int n = 0; n < nt; ++n) { ct[n] = cos(TWO_PI * n / nt); st[n] = sin(TWO_PI * n / nt); }
    for (int n = 0; n < nx; ++n) { cx[n] = cos(TWO_PI * n / nx); sx[n] = sin(TWO_PI * n / nx); }
#pragma omp parallel for schedule(static)
    for (int kk = 0; kk < nk; ++kk)
        for (int mt = 0; mt < nt; ++mt) {
            double gr = 0.0, gi = 0.0;
            for (int kw = -(nw - 1); kw <= nw - 1; ++kw) {
                const size_t f = (size_t)kk * nc + (kw + nw - 1);
                const int a = (int)posmod((long long)kw * mt, nt);
                gr += C[2 * f] * ct[a] - C[2 * f + 1] * st[a];
                gi += C[2 * f] * st[a] + C[2 * f + 1] * ct[a];
            }
            G[2 * ((size_t)kk * nt + mt)] = gr;
            G[2 * ((size_t)kk * nt + mt) + 1] = gi;
        }
#pragma omp parallel for schedule(static)
    for (int mx = 0; mx < nx; ++mx)
        for (int mt = 0; mt < nt; ++mt) {
            double acc = 0.0;
            for (int kk = 0; kk < nk; ++kk) {
                const int a = (int)posmod((long long)kk * mx, nx);
                const double *g = G + 2 * ((size_t)kk * nt + mt);
                acc += g[0] * cx[a] - g[1] * sx[a];
            }
            u[(size_t)mx * nt + mt] = acc;
        }
    free(G); free(ct); free(st); free(cx); free(sx);
}

/* ------------------------------------------------------------------------ */
/* 3rd-order SRM for a 1-D stochastic process u(t) (Section 3, the form of   */
/* Shields and Kim), read as:                                                */
/*  - Frequencies w_k = k dw, 0 <= k < N (one-sided).                        */
/*  - Pairs: i + j = k with i >= j >= 0 and i, j < W, each unordered pair    */
/*    once, the self pair i = j included (the printed index bounds are       */
/*    garbled; the process has no difference interactions).                 */
/*  - Phase of frequency k: the wave's phase of line (0, k) (key = seed,    */
/*    word k mod 4 of counter (0, floor(k / 4), 0, 0));                      */
/*    biphase beta(i, j): key = beta seed, counter (max, min, 1, 0).         */
/*  - rho_k, b_p^2 = rho_k b2_raw, Sigma_k, pure part sqrt(1 - Sigma_k) as   */
/*    for the wave (the pure-spectrum equation with b_p^2).                  */
/*  - u(t_m) = 2 [ sum_k sqrt(S_p,k dw) cos(w_k t_m + phi_k)                 */
/*             + sum_k sum_{i+j=k} sqrt(S_k dw) b_p cos(w_k t_m + phi_i      */
/*               + phi_j + beta) ],  t_m = m dt, dw dt = 2 pi / NT.          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n, W;
    double dw;
    const double *S;        /* [n] one-sided power spectrum */
    const double *b2;       /* [W][W] raw squared bicoherence, i, j >= 0 */
    const uint32_t *beta;   /* [W][W] fixed-point biphase */
    double cap;
} oracle_process;

void oracle_process_phases(int n, uint64_t seed, uint32_t *U)
{
    for (int k = 0; k < n; ++k) U[k] = phase_word(0, k, seed);
}

void oracle_process_biphase(int W, int mode, uint64_t beta_seed, uint32_t *beta)
{
    for (int i = 0; i < W; ++i)
        for (int j = 0; j < W; ++j) {
            const int hi = i >= j ? i : j, lo = i >= j ? j : i;
            beta[(size_t)i * W + j] = mode == 0 ? philox_word0((uint32_t)hi, (uint32_t)lo, 1u, beta_seed) : 0u;
        }
}

/* Raw bicoherence sum over the pairs of frequency k, cap factor, Sigma and
 * pair count; returns 2 if Sigma_k >= 1. */
int oracle_process_terms(const oracle_process *p, int k, double *sigma_raw, double *rho, double *sigma,
                         long *npairs)
{
    double sr = 0.0;
    long cnt = 0;
    for (int j = 0; 2 * j <= k; ++j) {
        const int i = k - j;
        if (i >= p->W) continue;
        sr += p->b2[(size_t)i * p->W + j];
        ++cnt;
    }
    double r = 1.0;
    if (p->cap > 0.0 && sr > p->cap) r = p->cap / sr;
    if (sigma_raw) *sigma_raw = sr;
    if (rho) *rho = r;
    if (sigma) *sigma = r * sr;
    if (npairs) *npairs = cnt;
    return (r * sr >= 1.0) ? 2 : 0;
}

/* Coefficients C_k = 2 sqrt(S_k dw) [sqrt(1 - Sigma_k) e^{i phi_k} + sum b_p
 * e^{i(phi_i + phi_j + beta)}], interleaved re/im, [n]. */
int oracle_process_coefficients(const oracle_process *p, const uint32_t *U, double *C)
{
    int status = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(max : status)
    for (int k = 0; k < p->n; ++k) {
        double rho, sigma;
        const int st = oracle_process_terms(p, k, NULL, &rho, &sigma, NULL);
        if (st) { status = st; C[2 * k] = NAN; C[2 * k + 1] = NAN; continue; }
        const double amp = 2.0 * sqrt(p->S[k] * p->dw);
        const double phik = TWO_PI * (double)U[k] / 4294967296.0;
        double re = sqrt(1.0 - sigma) * cos(phik);
        double im = sqrt(1.0 - sigma) * sin(phik);
        for (int j = 0; 2 * j <= k; ++j) {
            const int i = k - j;
            if (i >= p->W) continue;
            const size_t e = (size_t)i * p->W + j;
            const double bp = sqrt(rho * p->b2[e]);
            const uint32_t ang = U[i] + U[j] + p->beta[e];     /* exact mod 2^32 */
            const double th = TWO_PI * (double)ang / 4294967296.0;
            re += bp * cos(th);
            im += bp * sin(th);
        }
        C[2 * k] = amp * re;
        C[2 * k + 1] = amp * im;
    }
    return status;
}

/* u(t_m) = sum_k Re[C_k exp(2 pi i k m / nt)], direct cosine sum, [nt]. */
void oracle_process_field(int n, int nt, const double *C, double *u)
{
#pragma omp parallel for schedule(static)
    for (int m = 0; m < nt; ++m) {
        double acc = 0.0;
        for (int k = 0; k < n; ++k) {
            const double th = TWO_PI * (double)posmod((long long)k * m, nt) / (double)nt;
            acc += C[2 * k] * cos(th) - C[2 * k + 1] * sin(th);
        }
        u[m] = acc;
    }
}

/* Threads the OpenMP runtime will use (for reporting). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
