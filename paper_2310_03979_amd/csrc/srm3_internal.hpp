// Internal declarations of the srm3 HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "srm3.h"

namespace srm3 {

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11):
// ten rounds of two 32x32 -> 64-bit multiplies mixed with a Weyl key schedule.
// Only the first output word is used.  Host and device share this definition.
// ---------------------------------------------------------------------------
__host__ __device__ inline uint32_t philox_word0(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint64_t key)
{
    uint32_t k0 = static_cast<uint32_t>(key), k1 = static_cast<uint32_t>(key >> 32);
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
        c1 = static_cast<uint32_t>(p1);
        c3 = static_cast<uint32_t>(p0);
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c0;
}

// The first two output words of the same generator.
__host__ __device__ inline void philox_words01(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t key,
                                               uint32_t *w0, uint32_t *w1)
{
    uint32_t k0 = static_cast<uint32_t>(key), k1 = static_cast<uint32_t>(key >> 32);
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
        c1 = static_cast<uint32_t>(p1);
        c3 = static_cast<uint32_t>(p0);
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    *w0 = c0;
    *w1 = c1;
}

// All four output words of the same generator.
__host__ __device__ inline void philox_words4(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t key,
                                              uint32_t (&w)[4])
{
    uint32_t k0 = static_cast<uint32_t>(key), k1 = static_cast<uint32_t>(key >> 32);
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
        c1 = static_cast<uint32_t>(p1);
        c3 = static_cast<uint32_t>(p0);
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    w[0] = c0;
    w[1] = c1;
    w[2] = c2;
    w[3] = c3;
}

template <typename T> struct vec;
template <> struct vec<float> { using v2 = float2; using v4 = float4; };
template <> struct vec<double> { using v2 = double2; using v4 = double4; };
// elements of the a operand per (support column, row): 3 planes in FP32,
// 3 interleaved values padded to 4 in FP64
inline size_t a_slots(int precision) { return precision == SRM3_FP64 ? 4 : 3; }

constexpr int kMaxSeedsPerLaunch = 256;   // 2 KB of kernel arguments
struct SeedChunk {
    uint64_t s[kMaxSeedsPerLaunch];
};

// Geometry shared by the kernels of one plan.
struct Geometry {
    int nk, nw, W;      // lines n_kappa x (2 nw - 1); pair support |omega| < W
    int nc, ncw;        // 2 nw - 1, 2 W - 1
    int nx, nt;         // field
    int R;              // output rows per wave in the pair sum
    int nkp;            // n_kappa rounded up to a multiple of R
};

// Device workspace of one generate call (views into the plan's buffer).
struct Workspace {
    void *zrow;   // [B][nk][nc] complex phase factors, row-major over lines
    void *zcol;   // a operand (re + im, re, im) per support column, kappa-contiguous:
                  // FP32 [B][3][ncw][nkp] planes, FP64 [B][ncw][nkp][4] (4th slot unused)
    void *tsum;   // [B][nk][nc] complex pair sums
    void *g;      // [B][nk][nt] complex, after the t-transform
};

size_t workspace_bytes(const Geometry &g, int precision, int batch);
Workspace carve_workspace(const Geometry &g, int precision, int batch, void *base);

// Inputs of the FP64 amplitude computation done on the device (see
// assemble_line): plan spectrum, unit-scale raw pair sums, optional
// per-realization b^2 scales and spectra (device arrays indexed by the
// realization within a launch).
struct AmpRef {
    const double *S;
    const double *sig;
    const double *scale_b;
    const double *const *S_b;
    double dkdw;
    double cap;
    int pairs = 1;   // 0: zero bicoherence, the pair sums are not computed (Gaussian field);
                     // 2: the pair sums hold the whole self pair (hashed bispectra)
    const double *lc = nullptr;   // per-line complex pair factor c_k, interleaved (NULL = 1)
    const double *lr = nullptr;   // per-line complex phase factor rho_k, interleaved (NULL = 1);
                                  // the pure part divides it out
    const void *tab = nullptr;    // per-line (A_pure, A_pair) of the plan's spectrum at unit scale,
                                  // rounded to the plan's type (NULL: evaluated per line in FP64)
};

// Kernel launchers (stream-ordered, return the launch status).
hipError_t launch_phases(const Geometry &g, int precision, const uint64_t *seeds, const uint64_t *seeds_dev,
                         int batch, const Workspace &ws, const double *lr, hipStream_t st);
hipError_t launch_pairsum(const Geometry &g, int precision, const void *wtab, int batch,
                          const Workspace &ws, hipStream_t st);
// The same pair sum on the matrix cores: dense products over the partner
// frequency for each kappa split.  A wave owns rt x ct tiles of 16 x 16
// outputs; `shape` picks one of kMfmaShapes per precision (0: the default).
struct MfmaShape {
    int rt, ct;
};
constexpr int kMfmaShapes = 3;
MfmaShape mfma_shape(int precision, int shape);
hipError_t launch_pairsum_mfma(const Geometry &g, int precision, int shape, const void *wtab, int batch,
                               const Workspace &ws, hipStream_t st);
// Bispectrum generated per pair inside the kernel (hashed b^2 and beta).  With
// ws == nullptr it writes the per-line raw sums sum b^2_raw to sig (FP64).
hipError_t launch_pairsum_hash(const Geometry &g, int precision, uint64_t key, double scale, int batch,
                               const Workspace *ws, double *sig, hipStream_t st);
// Persistent pair sum over a device work list (all requests share R).
// mfma: items of the matrix-core pair sum (see mfma_rows_per_group).
hipError_t launch_pairsum_persistent(int precision, int R, const void *reqs, const void *items, const int *q_begin,
                                     int *q_next, int nblocks, hipStream_t st, bool mfma = false, int shape = 0);
// Output rows and columns of one matrix-core work item (a block of waves).
int mfma_rows_per_group(int precision, int shape);
int mfma_cols_per_group(int precision, int shape);
size_t persistent_req_bytes();
size_t persistent_item_bytes();
void fill_persistent_req(void *dst, const Geometry &g, const void *zrow, const void *zcol, void *tsum,
                         const void *wtab);
void fill_persistent_item(void *dst, int req, int kb, int cg);
int waves_per_block();
// 32-bit fill of device memory by a kernel (graph-safe, unlike hipMemsetAsync)
hipError_t launch_fill_u32(void *p, size_t words, uint32_t v, hipStream_t st);
constexpr int kXcds = 8;
// mode 0: assemble C from pair sums and phases; mode 1: read C from `cin`;
// mode 2 (zero bicoherence): C = A_pure e^{i phi} with the phases drawn here
// from the host `seeds` (no phase rows are read).
// rout (n_x == n_kappa == 1 only, else ignored): write the real field [B][n_t]
// directly; the x-transform is then skipped.
// Pass schedule of the register-blocked Stockham FFT of length N (a power of
// two, 1 <= N <= 16384): radix-16 passes while a factor 16 is left, then one
// pass of radix 2, 4 or 8.  Pass p has radix R[p] and span Ns[p] (product of
// the earlier radices); its twiddles e^{+2 pi i r k / (R Ns)}, r = 1 .. R - 1,
// k < Ns, sit at off[p] + (r - 1) Ns + k of the plan's table (N - 1 entries).
struct FftSched {
    int N, npass;
    int R[6], Ns[6], off[6];
};
inline FftSched fft_schedule(int N)
{
    FftSched s{};
    s.N = N;
    int ns = 1, off = 0;
    while (ns * 16 <= N) {
        s.R[s.npass] = 16;
        s.Ns[s.npass] = ns;
        s.off[s.npass] = off;
        off += 15 * ns;
        ns *= 16;
        ++s.npass;
    }
    if (ns < N) {
        s.R[s.npass] = N / ns;
        s.Ns[s.npass] = ns;
        s.off[s.npass] = off;
        ++s.npass;
    }
    return s;
}

// Per-line amplitudes (A_pure, A_pair) of a plan at unit scale, in the plan's
// type, exactly as the assembly evaluates them in FP64 and rounds them.
hipError_t launch_amp_table(int precision, long n, const double *S, const double *sig, double dkdw, double cap,
                            void *out, hipStream_t st);
hipError_t launch_tfft(const Geometry &g, int precision, int mode, const void *cin, const AmpRef &amp,
                       const void *wtab, const void *tw, int batch, const Workspace &ws, hipStream_t st,
                       void *rout = nullptr, const uint64_t *seeds = nullptr);
hipError_t launch_assemble(const Geometry &g, int precision, const AmpRef &amp, const void *wtab, int batch,
                           const Workspace &ws, void *cout, hipStream_t st);
hipError_t launch_xfft(const Geometry &g, int precision, const void *tw, int batch, const Workspace &ws,
                       void *out, void *const *out_b, hipStream_t st);
hipError_t launch_wtable(int precision, int W, int b2_kind, const double *g2, const double *b2, int beta_mode,
                        const uint32_t *beta_tab, uint64_t beta_seed, void *wt, hipStream_t st);
hipError_t launch_spectrum(int nk, int nw, double dk, double dw, double u_star, double z, double U, double lam,
                           double *S, hipStream_t st);

// Pair sum through an FFT along kappa (see the kernels for the derivation).
struct KfftGeom {
    int M = 0;        // DFT length along kappa, power of two >= 2 n_kappa - 1
    int nca = 0;      // output columns that a support pair reaches
    int c_lo = 0;     // first of them (column index, k_omega + n_omega - 1)
    int kw0 = 0;      // its k_omega
    int wh_rows = 0;  // rows of the sheared weight table, zero rows included
    int one_sided = 0;  // 1: outputs and partners at k_omega >= 0 only (the 1-D process)
    int L = 0;          // > 0: rank-one weights, the frequency autoconvolution runs as FFTs of length L
};
// Device tables of the kappa-DFT pair sum: the sheared half weight table and
// kappa twiddles; for rank-one weights W = g_i g_j instead the factor g [2W-1]
// and the twiddles of the length-L frequency transform.
struct KfftTables {
    const void *wh = nullptr;
    const void *tw_k = nullptr;
    const void *gw = nullptr;
    const void *tw_l = nullptr;
};
struct KfftWorkspace {
    void *Z = nullptr;   // [B][M][2W - 1] complex
    void *Y = nullptr;   // [B][M][nca] complex
};
KfftGeom kfft_geometry(const Geometry &g, bool one_sided);
size_t kfft_workspace_bytes(const Geometry &g, const KfftGeom &k, int precision, int batch);
KfftWorkspace carve_kfft(const Geometry &g, const KfftGeom &k, int precision, int batch, void *base);
bool kfft_supported(const Geometry &g, const KfftGeom &k, int precision, std::string *why);
hipError_t launch_wsh(int precision, const void *wt, const Geometry &g, const KfftGeom &k, void *wh, hipStream_t st);
// tw: e^{+2 pi i n / M}, n < M
hipError_t launch_kfft_pairsum(int precision, const Geometry &g, const KfftGeom &k, const KfftTables &t, int batch,
                               const Workspace &ws, const KfftWorkspace &kw, hipStream_t st);
double kfft_terms(const Geometry &g, const KfftGeom &k);

int pairsum_rows_per_wave(int nk, int precision);
hipError_t prepare_transforms(int precision);

// ---- host-side shared pieces (defined in srm3_api.hip) ----
struct DevBuf {
    void *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release();
    hipError_t alloc(size_t bytes);
};

// Kappa-dependent bicoherence (plan time, host FP64).  Per-line raw pair sums
// Q_k = sum_{P(k)} r_i^2 r_j^2 b2(i_w, j_w) (r may be NULL = 1; b2 separable
// from g2 or dense), and the line factors of the wind bispectrum through the
// partial-bicoherence recursion.
void line_pair_sums(int nk, int nw, int W, const double *r, int kind, const double *g2, const double *b2,
                    std::vector<double> &Q);
srm3_status wind_factors(int nk, int nw, int W, const double *S, double alpha, double cap, std::vector<double> &c,
                         std::vector<double> &r, int *sweeps, double *max_sig);
srm3_status product_factors(int nk, int nw, int W, const double *S, const double *F, const double *G,
                            const double *H, double dk, double dw, double cap, std::vector<double> &c,
                            std::vector<double> &rho, int *sweeps, double *max_sig,
                            std::vector<double> *sigma_out = nullptr);

srm3_status fail(srm3_status s, const char *fmt, ...);
srm3_status dev_err(hipError_t e, const char *what);
srm3_status upload_bytes(DevBuf &buf, const void *data, size_t bytes, hipStream_t st);
// Largest Sigma_k over the lines at a given b^2 scale.
double max_sigma(double max_sig, double cap, double scale);
// Rows per wave for a grid with nk wavenumber lines (R_pref <= 0: default).
int rows_for(int nk, int precision, int R_pref);
// Relative cost of pair-sum work item (row block kb, column group cg).
double item_cost(const Geometry &g, int R, int kb, int cg);
double mfma_item_cost(const Geometry &g, int kb, int cg, int precision, int shape);

}  // namespace srm3

struct srm3_plan_s {
    srm3::Geometry g{};
    int precision = SRM3_FP64;
    double dk = 0, dw = 0, cap = 0, max_sig = 0;
    double pair_terms = 0;
    int device = 0;
    srm3::DevBuf wtab, S, sig, tw_t, tw_x, ws;
    srm3::DevBuf amp_t;   // per-line (A_pure, A_pair) at unit scale (plans without line factors)
    srm3::DevBuf lc, lr;     // per-line complex bicoherence factors c, rho (interleaved FP64), or empty
    int ws_batch = 0;
    bool gaussian = false;   // zero bicoherence: no pair sum (2nd-order SRM)
    bool process = false;    // the 1-D process: one kappa line, one-sided spectrum and pairs
    bool hashed = false;     // bispectrum generated per pair in the kernel (SRM3_BISPEC_HASHED)
    bool fixed_spectrum = false;   // line factors derived from S (SRM3_BISPEC_PRODUCT): S may not change
    uint64_t hash_key = 0;
    double hash_scale = 0;
    // pair-sum algorithm; the kappa-FFT form keeps its tables and workspace here
    int algo = SRM3_ALGO_DIRECT;
    int mfma_shape = 0;   // tile shape of the matrix-core pair sum
    srm3::KfftGeom kg{};
    srm3::DevBuf wsh, tw_k, kws;
    srm3::DevBuf gw, tw_l;   // rank-one weights (SRM3_ALGO_FFT2D): sqrt(g2) and length-L twiddles
    std::vector<double> g2_host;   // separable factor of a plan with beta == 0, else empty
    int kws_batch = 0;
    // profiling
    bool prof = false;
    struct Rec {
        int kernel;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
};

namespace srm3 {
AmpRef plan_amp(srm3_plan_t p);
KfftTables plan_ktab(srm3_plan_t p);
}  // namespace srm3
