/*
 * srm3 -- 3rd-order Spectral Representation Method for skewed non-Gaussian
 * 1-D stochastic waves u(x, t) on one MI355X (gfx950).
 *
 * Method: Vandanapu & Shields, "Simulation of non-Gaussian wind field as a
 * 3rd-order stochastic wave", Section 4.1 (direct double cosine sum) and
 * Section 4.3 (FFT form: per-line coefficients B(+/-) followed by a 2-D
 * inverse DFT).  The library builds, for every wavenumber-frequency line
 * k = (k_kappa, k_omega), the coefficient
 *
 *   C_k = 2 sqrt(S_k dk dw) [ sqrt(1 - Sigma_k) e^{i phi_k}
 *                             + sum_{p={i,j}, i+j=k} b_p e^{i(phi_i + phi_j + beta_p)} ]
 *
 * (pure amplitude of Eq. pure with b_p^2, plus the pair sum of biamplitude x
 * phase factor), then evaluates u(m_x dx, m_t dt) = Re sum_k C_k
 * exp(2 pi i (k_kappa m_x / n_x + k_omega m_t / n_t)) with dk dx = 2 pi / n_x,
 * dw dt = 2 pi / n_t (Section 4.3 interval relations).
 *
 * Conventions shared by every entry point
 *  - Lines: 0 <= k_kappa < n_kappa, -n_omega < k_omega < n_omega (one line per
 *    signed frequency; kappa >= 0 half plane, Section 2).  Arrays over lines
 *    are row-major [n_kappa][2 n_omega - 1]; column c holds k_omega = c - (n_omega - 1).
 *  - Pairs: unordered {i, j} with i + j = k in both components, both partners
 *    inside the bicoherence support |i_omega|, |j_omega| < support_w, self pair
 *    included, each pair counted once.
 *  - Phases: phi_k = 2 pi U / 2^32 with U a word of Philox4x32-10 (Salmon et
 *    al., SC'11) under key = realization seed (low word first): one call
 *    serves four consecutive frequencies, U = word r of counter
 *    (k_kappa, (uint32)q, 0, 0) with k_omega = 4 q + r, 0 <= r < 4.  Seeded
 *    biphases use key = beta_seed, counter = (max(i_w, j_w), min(i_w, j_w), 1, 0)
 *    and word 0.
 *  - Streams: every device action is enqueued on the caller's hipStream_t
 *    (passed as void*; NULL = the default stream).  Calls return before the
 *    work finishes.  One plan may be driven by one stream at a time.
 *  - Errors: no exception crosses the ABI.  Arguments are validated before any
 *    device work; a failing call returns a non-zero srm3_status and leaves a
 *    message for srm3_last_error() (thread-local).
 *  - Ownership: host inputs are copied during the call and may be freed when
 *    it returns.  The plan owns every device buffer it allocates.  Output
 *    buffers are device memory owned by the caller.
 */
#ifndef SRM3_H
#define SRM3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct srm3_plan_s *srm3_plan_t;

typedef enum {
    SRM3_OK = 0,
    SRM3_E_INVALID = 1,        /* bad argument (null pointer, size, NaN, negative S, asymmetric table) */
    SRM3_E_PURE_NEGATIVE = 2,  /* some line has Sigma_k >= 1: pure spectrum not positive (Section 5) */
    SRM3_E_NOMEM = 3,          /* device or host allocation failed */
    SRM3_E_DEVICE = 4,         /* a HIP runtime call or kernel launch failed */
    SRM3_E_UNSUPPORTED = 5     /* valid but outside the library's limits (see srm3_plan) */
} srm3_status;

typedef enum { SRM3_FP64 = 0, SRM3_FP32 = 1 } srm3_precision;

typedef enum {
    SRM3_BISPEC_NONE = 0,      /* b == 0: the 2nd-order (Gaussian) SRM of Section 3 */
    SRM3_BISPEC_SEPARABLE = 1, /* b^2_raw(i_w, j_w) = g2[i_w] * g2[j_w] */
    SRM3_BISPEC_DENSE = 2,     /* b^2_raw given as a full symmetric table */
    SRM3_BISPEC_WIND = 3,      /* the wind bispectrum of Section 5 (Eq. bispectrum) times alpha, beta = 0,
                                  through the partial bicoherence of Section 4.1 (see below) */
    SRM3_BISPEC_PRODUCT = 4,   /* a prescribed bispectrum B(i, j) = F_k G_i G_j H(i_w, j_w) through the
                                  partial bicoherence, beta = atan2(Im B, Re B) (see below) */
    SRM3_BISPEC_HASHED = 5     /* b^2_raw and beta of every 4-index pair generated inside the kernel
                                  from a counter-based hash, no table (see below) */
} srm3_bispec_kind;

typedef enum {
    SRM3_BETA_SEEDED = 0,      /* beta drawn uniformly on [0, 2 pi) from beta_seed */
    SRM3_BETA_ZERO = 1,        /* beta == 0 (real positive bispectrum, as in Section 5) */
    SRM3_BETA_TABLE = 2        /* beta given as a symmetric fixed-point table */
} srm3_beta_mode;

/* Discretisation (Section 4.1 grid definitions, Section 4.3 interval relations). */
typedef struct {
    int32_t n_kappa;   /* wavenumber lines, >= 1 */
    int32_t n_omega;   /* frequency lines per sign, >= 1 (2 n_omega - 1 signed lines) */
    double d_kappa;    /* wavenumber step [rad/m], > 0 */
    double d_omega;    /* frequency step [rad/s], > 0 */
    int32_t n_x;       /* field points in x: power of two, n_kappa <= n_x <= 16384
                          (<= 8192 for SRM3_FP64) */
    int32_t n_t;       /* field points in t: power of two, 2 n_omega - 1 <= n_t <= 16384
                          (<= 8192 for SRM3_FP64) */
} srm3_grid;

/* Power spectrum sampled on the lines (Section 4.1): host FP64
 * [n_kappa][2 n_omega - 1], finite and >= 0. */
typedef struct {
    const double *S;
} srm3_spectrum;

/* Bicoherence and biphase over the frequency indices of a pair (the raw
 * squared bicoherence b^2_raw(i_w, j_w) before the per-line cap).  Indices run
 * over |i_w|, |j_w| < support_w, stored at [i_w + support_w - 1]. */
typedef struct {
    int32_t kind;            /* srm3_bispec_kind */
    const double *g2;        /* SEPARABLE: host [2W-1], finite, >= 0 */
    const double *b2;        /* DENSE: host [2W-1][2W-1], symmetric, finite, >= 0 */
    const uint32_t *beta;    /* BETA_TABLE: host [2W-1][2W-1] symmetric, 2^32 == 2 pi */
    int32_t support_w;       /* W, 1 <= W <= n_omega */
    double cap;              /* > 0: per line, b^2_p = min(1, cap / sum_{P(k)} b^2_raw) b^2_raw;
                                <= 0: no rescale */
    int32_t beta_mode;       /* srm3_beta_mode */
    uint64_t beta_seed;      /* BETA_SEEDED: Philox key */
    /* kappa-dependent bicoherence through per-line factors (optional, host
     * [n_kappa][2 n_omega - 1], NULL = 1): a pair {i, j} -> k has
     * b^2_raw = line_c[k]^2 line_r[i]^2 line_r[j]^2 b^2_raw(i_w, j_w).
     * line_c >= 0, line_r > 0, finite.  Not with SRM3_BISPEC_WIND. */
    const double *line_c;
    const double *line_r;
    double alpha;            /* SRM3_BISPEC_WIND: scale of the bispectrum, > 0 */
    /* SRM3_BISPEC_PRODUCT: host complex arrays (interleaved re, im): F and G
     * [n_kappa][2 n_omega - 1], H [2W-1][2W-1] symmetric (NULL = 1). */
    const double *prod_f;
    const double *prod_g;
    const double *prod_h;
} srm3_bispectrum;

/* SRM3_BISPEC_PRODUCT.  A prescribed bispectrum of product form
 * B(i, j) = F_k G_i G_j H(i_w, j_w), k = i + j (complex), enters as in
 * Section 4.1: b_p = |B| sqrt(dk dw) / sqrt(S_p,i S_p,j S_k) and
 * beta_p = atan2(Im B, Re B), with S_p = S (1 - Sigma) solved as for
 * SRM3_BISPEC_WIND (least fixed point, optional cap).  Equivalently
 * b_p e^{i beta_p} = c_k rho_i rho_j H(i_w, j_w) with the complex line factors
 * c_k = F_k sqrt(dk dw / S_k) and rho_i = G_i / sqrt(S_p,i) (zero where S is
 * zero); the library applies rho to the phase factors, c to a line's pair
 * sum and H as the weight table.  The wind bispectrum is the case
 * F_k = alpha 2 sqrt(S_k) / (3 sqrt(3 |w_k| kappa_k)), G = sqrt(S), H = 1.
 * support_w limits the pairs; g2, b2, beta and alpha are ignored.  Plan-time
 * sums: 2-D FFTs when H is NULL, else O(M (4W-3)(2W-1)) per sweep.  The
 * factors depend on S, so such a plan keeps its spectrum: srm3_set_spectrum
 * and per-request spectra (batches, server) return SRM3_E_UNSUPPORTED. */

/* SRM3_BISPEC_WIND.  B = alpha 2 sqrt(S_i S_j S_k) / (3 sqrt(3 |w_i + w_j| (kappa_i + kappa_j)))
 * (Section 5; |.| since the kappa >= 0 half plane holds negative frequencies;
 * zero where singular, k_kappa = 0 or k_omega = 0, or where an S is 0), and
 * b_p = |B| sqrt(dk dw) / sqrt(S_p,i S_p,j S_k) with the pure spectrum
 * S_p = S (1 - Sigma) (Section 4.1).  This factorises into line factors,
 * c_k = alpha 2 / (3 sqrt 3) / sqrt(|k_omega| k_kappa) and r_i = sqrt(S_i / S_p,i),
 * and Sigma solves a fixed point (Sigma_k = min(cap, c_k^2 sum_{P(k)} r_i^2 r_j^2)),
 * found at plan time by sweeps from Sigma = 0 (each a 2-D FFT
 * autoconvolution on the host).  support_w limits the pairs as usual; g2, b2
 * and beta are ignored.  SRM3_E_PURE_NEGATIVE if no admissible pure spectrum
 * exists without a cap.  The factors do not depend on the values of S (only on
 * where it is zero), so srm3_set_spectrum and per-request spectra with the
 * same zero lines keep them. */

/* SRM3_BISPEC_HASHED.  A bispectrum that depends on all four indices of a
 * pair, generated just in time: for the canonical member (i, j) of an
 * unordered pair (i_kappa > j_kappa, or equal and i_w >= j_w), with
 * m = floor(i_w / 8) and t = i_w - 8 m, Philox4x32-10 with key = beta_seed and
 * counter (i_kappa, (uint32)m, j_kappa, (uint32)(i_w + j_w)) holds the pair's
 * 16 bits h in word floor(t / 2) (high half for even t, low half for odd t):
 * u = h >> 8, v = h & 255, b_p = sqrt(alpha) u / 2^8 (so b^2_raw =
 * alpha (u / 2^8)^2) and beta = 2 pi v / 2^8.  One generator call thus serves
 * the eight pairs of a line whose i_w share m.  The per-line raw sums are computed on the device when the plan is built
 * (O(pairs)), then the cap applies as usual.  Direct pair sum only (the
 * weights depend on kappa); not in batches or the server (SRM3_E_UNSUPPORTED);
 * g2, b2, beta tables and line factors are ignored. */

/* The line factors and Sigma that SRM3_BISPEC_WIND derives (host only, FP64,
 * no device work): S host [n_kappa][2 n_omega - 1]; line_c, line_r, sigma:
 * caller-owned host arrays of the same shape (sigma may be NULL); sweeps
 * (may be NULL) receives the number of fixed-point sweeps.  Errors as for
 * srm3_plan with that kind. */
srm3_status srm3_wind_factors(const srm3_grid *grid, const double *S, double alpha, double cap, int32_t support_w,
                              double *line_c, double *line_r, double *sigma, int32_t *sweeps);

/* The complex line factors c and rho (interleaved, [n_kappa][2 n_omega - 1][2])
 * and Sigma that SRM3_BISPEC_PRODUCT derives (host only, FP64); F, G, H as in
 * srm3_bispectrum.  Errors as for srm3_plan with that kind. */
srm3_status srm3_product_factors(const srm3_grid *grid, const double *S, const double *F, const double *G,
                                 const double *H, int32_t support_w, double cap, double *line_c, double *line_rho,
                                 double *sigma, int32_t *sweeps);

/* Build a plan: validates every input, computes on the host in FP64 the
 * per-line raw bicoherence sums, the cap factor rho_k, Sigma_k and the two
 * amplitudes A_pure = 2 sqrt(S dk dw (1 - Sigma)) and A_pair = 2 sqrt(S dk dw
 * rho) (Eq. pure, Section 4.3), the complex pair weight table
 * W[i_w][j_w] = sqrt(b^2_raw) e^{i beta} and the transform twiddles, and
 * uploads them on `hip_stream` (the call synchronises that stream before it
 * returns).  bispectrum may be NULL (== SRM3_BISPEC_NONE).
 * Returns SRM3_E_PURE_NEGATIVE if any line has Sigma_k >= 1 and
 * SRM3_E_UNSUPPORTED for sizes outside the limits of srm3_grid. */
srm3_status srm3_plan(const srm3_grid *grid, const srm3_spectrum *spectrum,
                      const srm3_bispectrum *bispectrum, int32_t precision,
                      void *hip_stream, srm3_plan_t *out_plan);

/* Generate `batch` realizations (Section 4.3): phases from seeds[b] (host
 * array), pair sums, coefficients, 2-D inverse DFT.  out_dev: device buffer of
 * batch * n_x * n_t values of the plan's precision (float or double), layout
 * [b][m_x][m_t].  The plan's workspace grows on first use of a larger batch
 * (that call allocates device memory). */
srm3_status srm3_generate(srm3_plan_t plan, const uint64_t *seeds, int32_t batch,
                          void *out_dev, void *hip_stream);

/* Allocation-free generation, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same work and result as srm3_generate, with the workspace
 * taken from a fixed device array of the library instead of the plan's own
 * buffer.  The array holds 64 MiB on each GPU the library runs on and stays allocated until the process ends; the call makes no
 * device allocation and records no profiling events.  Nothing in it needs to
 * start at zero.  Every call on one GPU shares that GPU's array and leaves its
 * contents behind: calls that overlap on one GPU (two streams, two threads)
 * race, so callers serialise them.  Requires the plan's device to be current.
 * Errors: those of srm3_generate, and SRM3_E_UNSUPPORTED when the workspace of
 * `batch` realizations (srm3_workspace_bytes, rounded to 256 bytes) exceeds the
 * array, with the sizes in srm3_last_error(). */
srm3_status srm3_generate_noalloc(srm3_plan_t plan, const uint64_t *seeds, int32_t batch,
                                  void *out_dev, void *hip_stream);

/* Coefficients only: C_dev receives batch * n_kappa * (2 n_omega - 1) complex
 * values (interleaved re, im; float or double) laid out [b][k_kappa][c]. */
srm3_status srm3_coefficients(srm3_plan_t plan, const uint64_t *seeds, int32_t batch,
                              void *C_dev, void *hip_stream);

/* Transform only (Section 4.3, last step): field from caller-supplied device
 * coefficients laid out as for srm3_coefficients. */
srm3_status srm3_transform(srm3_plan_t plan, const void *C_dev, int32_t batch,
                           void *out_dev, void *hip_stream);

/* Device workspace bytes that srm3_generate needs for `batch` realizations. */
srm3_status srm3_workspace_bytes(srm3_plan_t plan, int32_t batch, size_t *bytes);

/* Fill the plan's whole device workspace for `batch` realizations (grown as
 * srm3_generate would grow it, so that call may allocate) with the 32-bit
 * pattern `word`, by a kernel on hip_stream.  For tests and tooling: with a
 * NaN pattern, a later generation shows that no kernel lets a value it did not
 * write reach the field.  Errors: SRM3_E_INVALID (NULL plan, batch < 0),
 * SRM3_E_UNSUPPORTED (batch > 65535), SRM3_E_NOMEM, SRM3_E_DEVICE. */
srm3_status srm3_workspace_fill(srm3_plan_t plan, int32_t batch, uint32_t word, void *hip_stream);

/* Number of unordered pair terms of one realization (sum over lines of |P(k)|). */
srm3_status srm3_pair_terms(srm3_plan_t plan, double *terms);

/* Output rows per wavefront of the plan's pair-sum tile (R: each wave owns
 * 64 frequency columns x R kappa rows); the kernel is instantiated per R. */
srm3_status srm3_rows_per_wave(srm3_plan_t plan, int32_t *rows);

/* Pair-sum algorithm of a plan (used by every entry point that takes the plan:
 * generation, coefficients, batches, the server).
 *   SRM3_ALGO_DIRECT     enumerates the unordered pairs of every line (the
 *                        coefficient sum of Section 4.1 / 4.3 as written).
 *   SRM3_ALGO_KAPPA_FFT  the same sum, reorganised: the weights depend on the
 *                        frequency indices only, so the kappa part of the
 *                        ordered pair sum is a linear convolution of phase
 *                        columns; it runs as a DFT along kappa (length
 *                        M >= 2 N_kappa - 1), a weighted frequency
 *                        autoconvolution per kappa frequency, and the inverse
 *                        DFT.  Same result up to rounding; O(M W^2) terms per
 *                        realization instead of O(N_kappa^2 W^2).
 *   SRM3_ALGO_FFT2D      for rank-one weights only (separable b^2 and
 *                        beta = 0, e.g. SRM3_BISPEC_WIND): W = g_i g_j, so the
 *                        whole pair sum is a 2-D linear autoconvolution of
 *                        g z: the DFT along kappa, then per kappa frequency a
 *                        forward FFT of length L >= 2(2W - 1) - 1 along the
 *                        frequency, a squaring and the inverse FFT, then the
 *                        inverse DFT along kappa.  Same result up to rounding;
 *                        O(M L log L) work per realization.
 *   SRM3_ALGO_MFMA       the direct form's unordered pairs (same terms) on the
 *                        matrix cores: for each kappa split the sum over the
 *                        partner frequency is a dense product of a block of
 *                        phase rows with a block of weighted phases, evaluated
 *                        with 16x16x4 MFMAs (FP32: v_mfma_f32_16x16x4_f32 with
 *                        two-sum flushes; FP64: v_mfma_f64_16x16x4_f64).  Same
 *                        result up to rounding.  Output rows go in groups of
 *                        32 kappa rows: grids with few rows (a 1-D process has
 *                        one) leave most of each product idle and are better
 *                        served by SRM3_ALGO_KAPPA_FFT.  Runs through
 *                        srm3_generate, srm3_coefficients, srm3_transform,
 *                        uneven batches (whose persistent launch then takes
 *                        matrix-core work items: a batch's direct-form plans
 *                        must be all SRM3_ALGO_DIRECT or all SRM3_ALGO_MFMA)
 *                        and servers created with pair_kernel SRM3_ALGO_MFMA.
 * Switching to SRM3_ALGO_KAPPA_FFT builds its sheared weight table on the
 * device (stream-ordered on hip_stream).  Errors: SRM3_E_INVALID (bad plan or
 * algorithm), SRM3_E_UNSUPPORTED (N_kappa > 2048; SRM3_ALGO_FFT2D: weights
 * not rank-one, or L above 16384, 8192 in FP64; any algorithm but
 * SRM3_ALGO_DIRECT for a bispectrum generated per pair, SRM3_BISPEC_HASHED),
 * SRM3_E_NOMEM, SRM3_E_DEVICE. */
enum { SRM3_ALGO_DIRECT = 0, SRM3_ALGO_KAPPA_FFT = 1, SRM3_ALGO_FFT2D = 2, SRM3_ALGO_MFMA = 3 };
srm3_status srm3_plan_set_algorithm(srm3_plan_t plan, int32_t algorithm, void *hip_stream);

/* Tile shape of the matrix-core pair sum (SRM3_ALGO_MFMA) used by
 * srm3_generate / srm3_coefficients on this plan: each wave owns `rows` kappa
 * rows x `cols` frequency columns of outputs (srm3_mfma_shape tells them for a
 * precision): shape 0 (the default) 32 x 32, shape 1 32 x 16, shape 2
 * 16 x 32, in FP32 and FP64.  The smaller tiles leave more waves resident per
 * SIMD and fit grids with few rows or columns better; every shape sums the same
 * pair terms, so results agree up to rounding.  Uneven batches created with
 * SRM3_BATCH_AUTOTUNE pick their shape by timing.  Errors: SRM3_E_INVALID (NULL
 * plan, shape outside 0..2). */
srm3_status srm3_plan_set_mfma_shape(srm3_plan_t plan, int32_t shape);
srm3_status srm3_mfma_shape(int32_t precision, int32_t shape, int32_t *rows, int32_t *cols);

/* Complex multiply-accumulate terms the plan's current pair-sum algorithm
 * evaluates per realization (SRM3_ALGO_DIRECT and SRM3_ALGO_MFMA: the pair
 * terms). */
srm3_status srm3_algorithm_terms(srm3_plan_t plan, double *terms);

/* Per-kernel device time, measured with HIP events recorded on the launch
 * stream around every launch while profiling is on.  Kernel ids:
 * 0 phases, 1 pair sum, 2 assemble + t-transform, 3 x-transform. */
typedef struct {
    double ms[4];          /* summed elapsed time per kernel id */
    int64_t launches[4];   /* launches per kernel id */
} srm3_profile;

srm3_status srm3_profile_enable(srm3_plan_t plan, int32_t enable); /* clears the record */
srm3_status srm3_profile_read(srm3_plan_t plan, srm3_profile *out); /* waits for the events */

/* ---- the 1-D stochastic process u(t) (Section 3, the 3rd-order SRM of a
 * process in the form of Shields and Kim) ----
 * Frequencies w_k = k d_omega, 0 <= k < n_omega (one-sided); pairs {i, j} with
 * i + j = k, i >= j >= 0, both < support_w, each once (self pair included);
 *   C_k = 2 sqrt(S_k dw) [ sqrt(1 - Sigma_k) e^{i phi_k}
 *                          + sum_{i+j=k} b_p e^{i(phi_i + phi_j + beta_p)} ],
 *   u(m dt) = Re sum_k C_k exp(2 pi i k m / n_t),  dw dt = 2 pi / n_t.
 * Cap, Sigma_k, the pure amplitude and the phase/biphase counters are those of
 * the wave with k_kappa = 0 and k_omega = k.  A process plan is the wave's plan
 * on one kappa line (d_kappa = 1, n_x = 1) with no spectrum at negative
 * frequencies and no pair with a negative partner, and every plan entry point
 * takes it: srm3_generate writes [b][n_t] (n_x = 1), srm3_coefficients
 * [b][2 n_omega - 1] (column n_omega - 1 + k; the negative columns are zero).
 * Its pair sum defaults to the frequency autoconvolution of
 * SRM3_ALGO_KAPPA_FFT (a DFT of length 1 along kappa), with the realizations of
 * a call as the rows of one launch; SRM3_ALGO_DIRECT also works. */
typedef struct {
    int32_t n_omega;   /* frequencies, >= 1 */
    double d_omega;    /* > 0 */
    int32_t n_t;       /* time points: power of two, 2 n_omega - 1 <= n_t <= 16384 (8192 for FP64) */
} srm3_process_grid;

/* S: host FP64 [n_omega] one-sided, finite, >= 0.  bispectrum (may be NULL)
 * as for srm3_plan but over 0 <= i, j < support_w only: g2 [W], b2 [W][W],
 * beta table [W][W] (symmetric).  Errors as for srm3_plan. */
srm3_status srm3_process_plan(const srm3_process_grid *grid, const double *S, const srm3_bispectrum *bispectrum,
                              int32_t precision, void *hip_stream, srm3_plan_t *out_plan);

/* Replace the plan's spectrum (same grid and bicoherence table): host FP64
 * [n_kappa][2 n_omega - 1] (a process plan: [n_omega] one-sided), validated
 * like srm3_plan; synchronises the stream. */
srm3_status srm3_set_spectrum(srm3_plan_t plan, const srm3_spectrum *spectrum, void *hip_stream);

/* Parameters of the wind-field spectrum of Section 5 (workload normalisation):
 * S(kappa, omega) = 200 u*^2 (z/U) / (1 + 50 f z/U)^(5/3) * (a/pi) / (a^2 + kappa^2),
 * f = |omega| / 2 pi, a = lam |omega| / (2 pi U), S(., 0) = 0. */
typedef struct {
    double u_star;   /* shear velocity [m/s], >= 0 */
    double z;        /* height [m], > 0 */
    double U;        /* mean wind speed [m/s], > 0 */
    double lam;      /* Davenport coherence decay, > 0 */
} srm3_kaimal_davenport;

/* Evaluate that spectrum on the lines of `grid` into device memory S_dev
 * (FP64 [n_kappa][2 n_omega - 1], caller-owned), stream-ordered.  Used to give
 * each request of a batch or server its own spectrum without host traffic. */
srm3_status srm3_spectrum_kaimal_davenport(const srm3_grid *grid, const srm3_kaimal_davenport *params,
                                           double *S_dev, void *hip_stream);

/* Release every device buffer of the plan.  NULL is a no-op.  Batches and
 * servers that use the plan must be destroyed first. */
void srm3_destroy(srm3_plan_t plan);

/* ---- uneven batches: many realizations of mixed grids in one persistent launch ----
 * One generation request: a realization of `plan` (grid, bicoherence table,
 * spectrum) with its own seed, bicoherence scale and optionally its own
 * spectrum.  With b2_scale = c, b^2_raw -> c b^2_raw for this realization (the
 * per-line cap is applied after scaling).  S_dev (device FP64, may be NULL =
 * the plan's spectrum) must hold finite values >= 0 in the line layout (a
 * process plan: [2 n_omega - 1], zero at negative frequencies) and stay valid
 * while the batch exists.  out_dev: [n_x][n_t] in the plan's precision. */
typedef struct {
    srm3_plan_t plan;
    uint64_t seed;
    double b2_scale;
    const double *S_dev;
    void *out_dev;
} srm3_request;

typedef struct srm3_batch_s *srm3_batch_t;

enum {
    SRM3_BATCH_GRAPH = 1,     /* capture the launch sequence in a hipGraph at the first run, replay after */
    SRM3_BATCH_AUTOTUNE = 2   /* pick rows per wave and persistent grid size by timing at the first run;
                                 choices are cached in $SRM3_TUNE_CACHE (default ~/.cache/srm3_tune.txt) */
};

/* Prepare a batch of n requests sharing one precision (plans may differ).
 * Allocates one workspace slice per request and builds the work list: every
 * (request, row block, column group) item, ordered by request cost and cut
 * into eight queues, one per XCD.  Requests whose plan uses
 * SRM3_ALGO_KAPPA_FFT or SRM3_ALGO_FFT2D run that pair sum per grid (all their
 * realizations at once) instead; plans with zero bicoherence have no pair
 * stage.  Plans with SRM3_ALGO_MFMA put matrix-core items (32 kappa rows x
 * 128 frequencies) into the persistent launch; a batch whose direct-form
 * plans mix SRM3_ALGO_DIRECT and SRM3_ALGO_MFMA is refused
 * (SRM3_E_UNSUPPORTED).  The plan's
 * algorithm is read here: set it before creating the batch (plans with
 * SRM3_BISPEC_HASHED are refused, SRM3_E_UNSUPPORTED).  Host arrays are
 * copied; plans must outlive the batch.  Fails with SRM3_E_PURE_NEGATIVE if a
 * scaled request would make some Sigma_k >= 1. */
srm3_status srm3_batch_create(const srm3_request *reqs, int32_t n, int32_t flags, void *hip_stream,
                              srm3_batch_t *out);
/* Run the batch: phases of every request, one persistent pair-sum launch over
 * all work items, then the transforms per plan.  seeds: host [n] in request
 * order (NULL = the seeds of the requests).  Stream-ordered; the first run
 * also tunes and/or captures when the flags ask for it (that run synchronises). */
srm3_status srm3_batch_run(srm3_batch_t batch, const uint64_t *seeds, void *hip_stream);

typedef struct {
    double pair_terms;      /* unordered pair terms over all requests */
    double run_ms;          /* device time of the last run (HIP events), -1 if none */
    double pairsum_ms;      /* pair-sum launch time of the last non-graph run, else -1 */
    int32_t rows_per_wave;  /* tile shape in use (vector-ALU pair sum) */
    int32_t blocks_per_cu;  /* persistent workgroups per compute unit */
    int32_t work_items;
    int32_t groups;         /* distinct plans */
    int32_t mfma_shape;     /* matrix-core tile shape in use (see srm3_plan_set_mfma_shape), -1 for vector items */
} srm3_batch_stats;
srm3_status srm3_batch_info(srm3_batch_t batch, srm3_batch_stats *out); /* waits for the last run */
void srm3_batch_destroy(srm3_batch_t batch);   /* NULL is a no-op */

/* One-shot uneven generation: create, run, synchronise, destroy. */
srm3_status srm3_generate_uneven(const srm3_request *reqs, int32_t n, void *hip_stream);

/* ---- request server: continuous (iteration-level) batching ----
 * Requests wait in FIFO order until a slot is free and their workspace fits
 * in the server's device arena (admission by HBM footprint; head-of-line
 * requests are never skipped).  Each srm3_server_step() retires finished
 * requests, admits what fits, and enqueues one step of work: pair-sum work
 * items of the resident requests (shortest remaining work first, or
 * round-robin; enough to fill the GPU twice and at least step_pair_terms pair
 * terms) in one persistent launch,
 * then the transforms of the requests whose work has all been issued.  A
 * request whose plan uses SRM3_ALGO_KAPPA_FFT runs its pair sum (the DFT form,
 * workspace from the arena) at admission within the step; a plan with zero
 * bicoherence has no pair stage.  A request admitted between steps joins the
 * next step, sharing the GPU with the requests already running.  A request's
 * result does not depend on what it was batched with. */
typedef struct srm3_server_s *srm3_server_t;

enum {
    SRM3_SERVE_SHORTEST_FIRST = 0,  /* each step serves the requests with the least work left first */
    SRM3_SERVE_ROUND_ROBIN = 1      /* each step takes one item from every request in turn */
};

typedef struct {
    int32_t precision;        /* SRM3_FP32 or SRM3_FP64; every request must match */
    int32_t max_active;       /* resident requests at once (slots), 1..4096 */
    size_t hbm_budget;        /* bytes of the device arena holding request workspaces (allocated once) */
    double step_pair_terms;   /* minimum pair terms per step; <= 0: 2e11 */
    int32_t policy;           /* SRM3_SERVE_SHORTEST_FIRST or SRM3_SERVE_ROUND_ROBIN */
    int32_t pair_kernel;      /* SRM3_ALGO_DIRECT (0: vector ALUs) or SRM3_ALGO_MFMA (matrix cores): the
                                 kernel of the per-step persistent pair-sum launch; direct-form requests
                                 must have plans with this algorithm (else SRM3_E_UNSUPPORTED) */
    int32_t mfma_shape;       /* matrix-core tile shape of those launches (0..2, see srm3_plan_set_mfma_shape) */
} srm3_server_config;

typedef struct {
    int32_t queued, active, finishing, completed;  /* requests in each state after the call */
    int32_t launched;                              /* 1 if this call enqueued a step */
    int64_t steps;                                 /* steps enqueued so far */
} srm3_server_state;

srm3_status srm3_server_create(const srm3_server_config *cfg, void *hip_stream, srm3_server_t *out);
/* Queue a request.  If `spectrum` is given, the request's spectrum is
 * evaluated on the device at admission into its own arena space (req->S_dev
 * must then be NULL; SRM3_E_UNSUPPORTED for a process plan).  The plan's
 * pair-sum algorithm is read here; the plan must not change algorithm while
 * the request is in flight.  Plans with SRM3_BISPEC_HASHED are refused
 * (SRM3_E_UNSUPPORTED).  out_dev must stay valid until the ticket completes.
 * SRM3_E_NOMEM if the request could never fit the arena. */
srm3_status srm3_server_submit(srm3_server_t srv, const srm3_request *req,
                               const srm3_kaimal_davenport *spectrum, int64_t *ticket);
/* One scheduling iteration (non-blocking: does nothing while two steps are in flight). */
srm3_status srm3_server_step(srm3_server_t srv, srm3_server_state *state);
/* Tickets whose fields are complete, oldest first; *n receives the count. */
srm3_status srm3_server_poll(srm3_server_t srv, int64_t *tickets, int32_t max, int32_t *n);
/* Wait for all enqueued work and free the server (queued requests are dropped). */
void srm3_server_destroy(srm3_server_t srv);

/* Message describing the last failure on the calling thread ("" if none). */
const char *srm3_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SRM3_H */
