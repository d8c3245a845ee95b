// C-ABI of the srm3 library: plan construction (host, FP64), generation
// launch sequences, uneven batches (persistent launch, hipGraph, autotuner),
// error reporting and event-based kernel timing.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "srm3_internal.hpp"

using namespace srm3;

namespace srm3 {

thread_local char g_err[512] = "";

srm3_status fail(srm3_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

srm3_status dev_err(hipError_t e, const char *what)
{
    return fail(SRM3_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void DevBuf::release()
{
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
}

hipError_t DevBuf::alloc(size_t bytes)
{
    release();
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipSuccess) n = bytes;
    else p = nullptr;
    return e;
}

srm3_status upload_bytes(DevBuf &buf, const void *data, size_t bytes, hipStream_t st)
{
    hipError_t e = buf.alloc(bytes);
    if (e != hipSuccess) return fail(SRM3_E_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    e = hipMemcpyAsync(buf.p, data, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return dev_err(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return dev_err(e, "hipStreamSynchronize");
    return SRM3_OK;
}

KfftTables plan_ktab(srm3_plan_t p)
{
    KfftTables t;
    t.wh = p->wsh.p;
    t.tw_k = p->tw_k.p;
    if (p->kg.L > 0) {
        t.gw = p->gw.p;
        t.tw_l = p->tw_l.p;
    }
    return t;
}

AmpRef plan_amp(srm3_plan_t p)
{
    return AmpRef{static_cast<const double *>(p->S.p), static_cast<const double *>(p->sig.p), nullptr, nullptr,
                  p->dk * p->dw, p->cap, p->gaussian ? 0 : (p->hashed ? 2 : 1), static_cast<const double *>(p->lc.p),
                  static_cast<const double *>(p->lr.p), p->amp_t.p};
}

// The plan's per-line amplitudes at unit scale (plans without line factors);
// recomputed whenever the spectrum changes.
srm3_status refresh_amp_table(srm3_plan_t p, hipStream_t st)
{
    if (p->lc.p || p->lr.p) return SRM3_OK;
    const long n = static_cast<long>(p->g.nk) * p->g.nc;
    const size_t bytes = static_cast<size_t>(n) * (p->precision == SRM3_FP64 ? 16 : 8);
    if (!p->amp_t.p) {
        hipError_t e = p->amp_t.alloc(bytes);
        if (e != hipSuccess) return fail(SRM3_E_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    hipError_t e = launch_amp_table(p->precision, n, static_cast<const double *>(p->S.p),
                                    static_cast<const double *>(p->sig.p), p->dk * p->dw, p->cap, p->amp_t.p, st);
    if (e != hipSuccess) return dev_err(e, "amplitude-table kernel");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return dev_err(e, "hipStreamSynchronize");
    return SRM3_OK;
}

double max_sigma(double max_sig, double cap, double scale)
{
    const double s = scale * max_sig;
    return (cap > 0 && s > cap) ? cap : s;
}

int rows_for(int nk, int precision, int R_pref)
{
    int r = R_pref > 0 ? R_pref : pairsum_rows_per_wave(nk, precision);
    const int cap = precision == SRM3_FP64 ? 8 : 16;
    if (r > cap) r = cap;
    while (r > 2 && r > nk) r /= 2;
    return r;
}

}  // namespace srm3

namespace {

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

namespace {

template <typename T>
std::vector<unsigned char> to_bytes(const std::vector<double> &v)
{
    std::vector<unsigned char> out(v.size() * sizeof(T));
    T *p = reinterpret_cast<T *>(out.data());
    for (size_t i = 0; i < v.size(); ++i) p[i] = static_cast<T>(v[i]);
    return out;
}

srm3_status upload(DevBuf &buf, const std::vector<double> &v, int precision, hipStream_t st)
{
    std::vector<unsigned char> bytes = precision == SRM3_FP64 ? to_bytes<double>(v) : to_bytes<float>(v);
    return upload_bytes(buf, bytes.data(), bytes.size(), st);
}

// Twiddles of the register-blocked FFT's passes (fft_schedule): for pass p,
// e^{+2 pi i r k / (R Ns)} at off[p] + (r - 1) Ns + k, interleaved (at least
// one entry, so that N = 1 still has a table).
std::vector<double> pass_twiddles(int N)
{
    const FftSched s = fft_schedule(N);
    std::vector<double> v(2 * static_cast<size_t>(std::max(1, N - 1)), 0.0);
    for (int p = 0; p < s.npass; ++p) {
        const int R = s.R[p], Ns = s.Ns[p];
        for (int r = 1; r < R; ++r)
            for (int k = 0; k < Ns; ++k) {
                const long double a = 2.0L * 3.14159265358979323846264338327950288L * (r * k) / (R * Ns);
                const size_t i = static_cast<size_t>(s.off[p] + (r - 1) * Ns + k);
                v[2 * i] = static_cast<double>(cosl(a));
                v[2 * i + 1] = static_cast<double>(sinl(a));
            }
    }
    return v;
}

// exp(+2 pi i n / N), n < N, interleaved
std::vector<double> twiddles(int N)
{
    std::vector<double> v(2 * static_cast<size_t>(N));
    for (int n = 0; n < N; ++n) {
        const long double a = 2.0L * 3.14159265358979323846264338327950288L * n / N;
        v[2 * n] = static_cast<double>(cosl(a));
        v[2 * n + 1] = static_cast<double>(sinl(a));
    }
    return v;
}

srm3_status event_pair(srm3_plan_t p, int kernel, hipStream_t st, bool begin)
{
    if (!p->prof) return SRM3_OK;
    hipEvent_t ev;
    if (!p->pool.empty()) {
        ev = p->pool.back();
        p->pool.pop_back();
    } else {
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) return dev_err(e, "hipEventCreate");
    }
    hipError_t e = hipEventRecord(ev, st);
    if (e != hipSuccess) return dev_err(e, "hipEventRecord");
    if (begin) {
        p->recs.push_back({kernel, ev, nullptr});
    } else {
        p->recs.back().b = ev;
    }
    return SRM3_OK;
}

// The pair-sum algorithms that go through a DFT along kappa (own workspace and tables).
bool kfft_family(int algo) { return algo == SRM3_ALGO_KAPPA_FFT || algo == SRM3_ALGO_FFT2D; }

srm3_status ensure_workspace(srm3_plan_t p, int batch, hipStream_t st)
{
    if (batch > p->ws_batch) {
        const size_t bytes = workspace_bytes(p->g, p->precision, batch);
        hipError_t e = p->ws.alloc(bytes);
        if (e != hipSuccess) {
            p->ws_batch = 0;
            return fail(SRM3_E_NOMEM, "workspace hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        }
        p->ws_batch = batch;
    }
    if (kfft_family(p->algo) && batch > p->kws_batch) {
        const size_t bytes = kfft_workspace_bytes(p->g, p->kg, p->precision, batch);
        hipError_t e = p->kws.alloc(bytes);
        if (e != hipSuccess) {
            p->kws_batch = 0;
            return fail(SRM3_E_NOMEM, "kappa-FFT workspace hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        }
        p->kws_batch = batch;
    }
    return SRM3_OK;
}

srm3_status check_batch(srm3_plan_t p, const void *seeds, int32_t batch, const void *out)
{
    if (!p) return fail(SRM3_E_INVALID, "plan is NULL");
    if (batch < 0) return fail(SRM3_E_INVALID, "batch %d < 0", batch);
    if (batch > 0 && (!seeds || !out)) return fail(SRM3_E_INVALID, "seeds/output pointer is NULL");
    const long long lines = static_cast<long long>(p->g.nk) * p->g.nc;
    if (static_cast<long long>(batch) * p->g.nkp * p->g.nc > (1LL << 31) ||
        static_cast<long long>(batch) * lines > (1LL << 31) || batch > 65535)
        return fail(SRM3_E_UNSUPPORTED, "batch %d too large for this grid", batch);
    return SRM3_OK;
}

srm3_status run_front_kfft(srm3_plan_t p, const uint64_t *seeds, int32_t batch, const Workspace &ws,
                           const KfftWorkspace &kw, hipStream_t st)
{
    srm3_status s;
    if ((s = event_pair(p, 0, st, true))) return s;
    Workspace wp = ws;
    if (p->gaussian || p->hashed || kfft_family(p->algo)) wp.zcol = nullptr;   // no a operand planes needed
    hipError_t e = launch_phases(p->g, p->precision, seeds, nullptr, batch, wp, static_cast<const double *>(p->lr.p), st);
    if (e != hipSuccess) return dev_err(e, "phase kernel");
    if ((s = event_pair(p, 0, st, false))) return s;
    if (p->gaussian) return SRM3_OK;   // zero bicoherence: the pair sums are not used
    if ((s = event_pair(p, 1, st, true))) return s;
    if (p->hashed) {
        e = launch_pairsum_hash(p->g, p->precision, p->hash_key, p->hash_scale, batch, &ws, nullptr, st);
        if (e != hipSuccess) return dev_err(e, "hashed pair-sum kernel");
    } else if (kfft_family(p->algo)) {
        e = launch_kfft_pairsum(p->precision, p->g, p->kg, plan_ktab(p), batch, ws, kw, st);
        if (e != hipSuccess) return dev_err(e, "kappa-FFT pair-sum kernels");
    } else if (p->algo == SRM3_ALGO_MFMA) {
        e = launch_pairsum_mfma(p->g, p->precision, p->mfma_shape, p->wtab.p, batch, ws, st);
        if (e != hipSuccess) return dev_err(e, "matrix-core pair-sum kernel");
    } else {
        e = launch_pairsum(p->g, p->precision, p->wtab.p, batch, ws, st);
        if (e != hipSuccess) return dev_err(e, "pair-sum kernel");
    }
    if ((s = event_pair(p, 1, st, false))) return s;
    return SRM3_OK;
}

// phases and pair sums with the plan's own kappa-FFT workspace
srm3_status run_front(srm3_plan_t p, const uint64_t *seeds, int32_t batch, const Workspace &ws, hipStream_t st)
{
    KfftWorkspace kw;
    if (kfft_family(p->algo)) kw = carve_kfft(p->g, p->kg, p->precision, batch, p->kws.p);
    return run_front_kfft(p, seeds, batch, ws, kw, st);
}

srm3_status run_back(srm3_plan_t p, int mode, const void *cin, int32_t batch, const Workspace &ws, void *out,
                     hipStream_t st, const uint64_t *seeds = nullptr)
{
    srm3_status s;
    if ((s = event_pair(p, 2, st, true))) return s;
    const bool direct_out = p->g.nx == 1 && p->g.nk == 1;   // the x-transform is the real part
    hipError_t e = launch_tfft(p->g, p->precision, mode, cin, plan_amp(p), p->wtab.p, p->tw_t.p, batch, ws, st,
                               direct_out ? out : nullptr, seeds);
    if (e != hipSuccess) return dev_err(e, "t-transform kernel");
    if ((s = event_pair(p, 2, st, false))) return s;
    if (direct_out) return SRM3_OK;
    if ((s = event_pair(p, 3, st, true))) return s;
    e = launch_xfft(p->g, p->precision, p->tw_x.p, batch, ws, out, nullptr, st);
    if (e != hipSuccess) return dev_err(e, "x-transform kernel");
    if ((s = event_pair(p, 3, st, false))) return s;
    return SRM3_OK;
}

srm3_status check_spectrum(const double *S, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!(S[i] >= 0) || !std::isfinite(S[i])) return fail(SRM3_E_INVALID, "S[%zu] must be finite and >= 0", i);
    return SRM3_OK;
}

}  // namespace

extern "C" {

const char *srm3_last_error(void) { return g_err; }

srm3_status srm3_plan(const srm3_grid *grid, const srm3_spectrum *spectrum, const srm3_bispectrum *bispectrum,
                      int32_t precision, void *hip_stream, srm3_plan_t *out_plan)
{
    g_err[0] = 0;
    if (!out_plan) return fail(SRM3_E_INVALID, "out_plan is NULL");
    *out_plan = nullptr;
    if (!grid || !spectrum || !spectrum->S) return fail(SRM3_E_INVALID, "grid/spectrum is NULL");
    if (precision != SRM3_FP64 && precision != SRM3_FP32) return fail(SRM3_E_INVALID, "precision %d", precision);
    const int nk = grid->n_kappa, nw = grid->n_omega, nx = grid->n_x, nt = grid->n_t;
    if (nk < 1 || nw < 1) return fail(SRM3_E_INVALID, "n_kappa=%d n_omega=%d must be >= 1", nk, nw);
    if (!(grid->d_kappa > 0) || !(grid->d_omega > 0) || !std::isfinite(grid->d_kappa) ||
        !std::isfinite(grid->d_omega))
        return fail(SRM3_E_INVALID, "d_kappa/d_omega must be finite and > 0");
    if (!is_pow2(nx) || !is_pow2(nt)) return fail(SRM3_E_UNSUPPORTED, "n_x=%d n_t=%d must be powers of two", nx, nt);
    const int nc = 2 * nw - 1;
    if (nx < nk || nt < nc)
        return fail(SRM3_E_INVALID, "field %dx%d smaller than the line grid (need n_x >= %d, n_t >= %d)", nx, nt,
                    nk, nc);
    const int tmax = precision == SRM3_FP64 ? 8192 : 16384;   // one transform fits 128 KB of LDS
    if (nt > tmax || nx > tmax)
        return fail(SRM3_E_UNSUPPORTED, "n_t=%d / n_x=%d above the library's limit %d", nt, nx, tmax);
    if (static_cast<long long>(nk) * nc > (1LL << 30)) return fail(SRM3_E_UNSUPPORTED, "line grid too large");

    // ---- bicoherence description ----
    srm3_bispectrum none{};
    none.kind = SRM3_BISPEC_NONE;
    none.support_w = 1;
    none.beta_mode = SRM3_BETA_ZERO;
    srm3_bispectrum bs = bispectrum ? *bispectrum : none;
    const int W = bs.kind == SRM3_BISPEC_NONE ? (bs.support_w >= 1 ? bs.support_w : 1) : bs.support_w;
    if (W < 1 || W > nw) return fail(SRM3_E_INVALID, "support_w=%d must be in [1, n_omega=%d]", W, nw);
    const int ncw = 2 * W - 1;
    if (bs.kind != SRM3_BISPEC_NONE && bs.kind != SRM3_BISPEC_SEPARABLE && bs.kind != SRM3_BISPEC_DENSE &&
        bs.kind != SRM3_BISPEC_WIND && bs.kind != SRM3_BISPEC_PRODUCT && bs.kind != SRM3_BISPEC_HASHED)
        return fail(SRM3_E_INVALID, "bispectrum kind %d", bs.kind);
    const bool hashed = bs.kind == SRM3_BISPEC_HASHED;
    const uint64_t hash_key = bs.beta_seed;
    const double hash_scale = bs.alpha;
    if (hashed) {
        // generated per pair in the kernel; the unit table only serves the pair count
        if (bs.line_c || bs.line_r) return fail(SRM3_E_INVALID, "line factors do not apply to a hashed bispectrum");
        if (!(bs.alpha > 0) || !std::isfinite(bs.alpha)) return fail(SRM3_E_INVALID, "alpha (scale) must be finite and > 0");
        bs.kind = SRM3_BISPEC_SEPARABLE;
        bs.beta_mode = SRM3_BETA_ZERO;
    }
    if (bs.kind == SRM3_BISPEC_NONE) bs.line_c = bs.line_r = nullptr;
    const size_t nlines0 = static_cast<size_t>(nk) * nc;
    // complex per-line factors c (pair sum) and rho (phase factor), interleaved
    std::vector<double> lcx, lrx, hw2, hcx;
    const std::vector<double> ones(static_cast<size_t>(ncw), 1.0);
    auto real_to_complex = [&](const double *f, std::vector<double> &out) {
        out.assign(2 * nlines0, 0.0);
        for (size_t l = 0; l < nlines0; ++l) out[2 * l] = f[l];
    };
    if (bs.kind == SRM3_BISPEC_WIND || bs.kind == SRM3_BISPEC_PRODUCT) {
        if (bs.line_c || bs.line_r) return fail(SRM3_E_INVALID, "line factors are derived from the bispectrum");
        if (!(bs.cap < 1.0) || !std::isfinite(bs.cap)) return fail(SRM3_E_INVALID, "cap must be < 1");
        srm3_status sw = check_spectrum(spectrum->S, nlines0);
        if (sw) return sw;
        if (bs.kind == SRM3_BISPEC_WIND) {
            // the wind bispectrum becomes real line factors over a unit separable table
            if (!(bs.alpha > 0) || !std::isfinite(bs.alpha)) return fail(SRM3_E_INVALID, "alpha must be finite and > 0");
            std::vector<double> c, r;
            if ((sw = wind_factors(nk, nw, W, spectrum->S, bs.alpha, bs.cap, c, r, nullptr, nullptr))) return sw;
            real_to_complex(c.data(), lcx);
            real_to_complex(r.data(), lrx);
        } else {
            // a prescribed product bispectrum: complex line factors, H as the weight table
            if (!bs.prod_f || !bs.prod_g) return fail(SRM3_E_INVALID, "prod_f / prod_g is NULL");
            for (size_t l = 0; l < 2 * nlines0; ++l)
                if (!std::isfinite(bs.prod_f[l]) || !std::isfinite(bs.prod_g[l]))
                    return fail(SRM3_E_INVALID, "F and G must be finite");
            if (bs.prod_h) {
                const size_t n2 = static_cast<size_t>(ncw) * ncw;
                for (int i = 0; i < ncw; ++i)
                    for (int j = 0; j < ncw; ++j) {
                        const size_t a = 2 * (static_cast<size_t>(i) * ncw + j), b = 2 * (static_cast<size_t>(j) * ncw + i);
                        if (!std::isfinite(bs.prod_h[a]) || !std::isfinite(bs.prod_h[a + 1]))
                            return fail(SRM3_E_INVALID, "H must be finite");
                        if (bs.prod_h[a] != bs.prod_h[b] || bs.prod_h[a + 1] != bs.prod_h[b + 1])
                            return fail(SRM3_E_INVALID, "H is not symmetric at [%d][%d]", i, j);
                    }
                hw2.resize(n2);
                for (size_t e = 0; e < n2; ++e)
                    hw2[e] = bs.prod_h[2 * e] * bs.prod_h[2 * e] + bs.prod_h[2 * e + 1] * bs.prod_h[2 * e + 1];
                hcx.assign(bs.prod_h, bs.prod_h + 2 * n2);
            }
            if ((sw = product_factors(nk, nw, W, spectrum->S, bs.prod_f, bs.prod_g, bs.prod_h, grid->d_kappa,
                                      grid->d_omega, bs.cap, lcx, lrx, nullptr, nullptr)))
                return sw;
        }
        if (bs.kind == SRM3_BISPEC_PRODUCT && bs.prod_h) {
            bs.kind = SRM3_BISPEC_DENSE;      // |H|^2 for the plan-time sums; H itself is the weight table
            bs.b2 = hw2.data();
        } else {
            bs.kind = SRM3_BISPEC_SEPARABLE;
            bs.g2 = ones.data();
        }
        bs.beta_mode = SRM3_BETA_ZERO;
    } else {
        for (const double *f : {bs.line_c, bs.line_r}) {
            if (!f) continue;
            for (size_t l = 0; l < nlines0; ++l)
                if (!(f[l] >= 0) || !std::isfinite(f[l]) || (f == bs.line_r && !(f[l] > 0)))
                    return fail(SRM3_E_INVALID, "line factor [%zu] must be finite (line_c >= 0, line_r > 0)", l);
        }
        if (bs.line_c) real_to_complex(bs.line_c, lcx);
        if (bs.line_r) real_to_complex(bs.line_r, lrx);
    }
    if (hashed) bs.g2 = ones.data();
    const bool factors = !lcx.empty() || !lrx.empty();
    if (bs.kind == SRM3_BISPEC_SEPARABLE && !bs.g2) return fail(SRM3_E_INVALID, "g2 is NULL");
    if (bs.kind == SRM3_BISPEC_DENSE && !bs.b2) return fail(SRM3_E_INVALID, "b2 is NULL");
    if (bs.beta_mode != SRM3_BETA_SEEDED && bs.beta_mode != SRM3_BETA_ZERO && bs.beta_mode != SRM3_BETA_TABLE)
        return fail(SRM3_E_INVALID, "beta_mode %d", bs.beta_mode);
    if (bs.kind != SRM3_BISPEC_NONE && bs.beta_mode == SRM3_BETA_TABLE && !bs.beta)
        return fail(SRM3_E_INVALID, "beta table is NULL");
    if (!std::isfinite(bs.cap)) return fail(SRM3_E_INVALID, "cap is not finite");

    // validate the bicoherence description (the weight table itself is built on the device)
    if (bs.kind == SRM3_BISPEC_SEPARABLE) {
        for (int i = 0; i < ncw; ++i)
            if (!(bs.g2[i] >= 0) || !std::isfinite(bs.g2[i]))
                return fail(SRM3_E_INVALID, "g2[%d] must be finite and >= 0", i);
    } else if (bs.kind == SRM3_BISPEC_DENSE) {
        for (int i = 0; i < ncw; ++i)
            for (int j = 0; j < ncw; ++j) {
                const double v = bs.b2[static_cast<size_t>(i) * ncw + j];
                if (!(v >= 0) || !std::isfinite(v))
                    return fail(SRM3_E_INVALID, "b2[%d][%d] must be finite and >= 0", i, j);
                if (v != bs.b2[static_cast<size_t>(j) * ncw + i])
                    return fail(SRM3_E_INVALID, "b2 is not symmetric at [%d][%d]", i, j);
            }
    }
    if (bs.kind != SRM3_BISPEC_NONE && bs.beta_mode == SRM3_BETA_TABLE) {
        for (int i = 0; i < ncw; ++i)
            for (int j = 0; j < i; ++j)
                if (bs.beta[static_cast<size_t>(i) * ncw + j] != bs.beta[static_cast<size_t>(j) * ncw + i])
                    return fail(SRM3_E_INVALID, "beta table is not symmetric at [%d][%d]", i, j);
    }
    auto b2at = [&](int i, int j) -> double {
        if (bs.kind == SRM3_BISPEC_SEPARABLE) return bs.g2[i] * bs.g2[j];
        if (bs.kind == SRM3_BISPEC_DENSE) return bs.b2[static_cast<size_t>(i) * ncw + j];
        return 0.0;
    };

    const double *S = spectrum->S;
    const size_t nlines = static_cast<size_t>(nk) * nc;
    srm3_status s = check_spectrum(S, nlines);
    if (s) return s;

    // ---- per-line unit-scale raw pair sums (ordered frequency splits + self pair), FP64 ----
    // D[kw] = sum_{iw} b2(iw, kw - iw) over the support; a line with k_kappa
    // = kk has (kk + 1) kappa splits, so its ordered sum is (kk+1) D[kw] and
    // its unordered sum half of that plus half the self pair.
    std::vector<double> D(nc, 0.0);
    std::vector<long> nsplit(nc, 0);
    for (int kw = -(nw - 1); kw <= nw - 1; ++kw) {
        double acc = 0.0;
        for (int iw = -(W - 1); iw <= W - 1; ++iw) {
            const int jw = kw - iw;
            if (jw <= -W || jw >= W) continue;
            acc += b2at(iw + W - 1, jw + W - 1);
            ++nsplit[kw + nw - 1];
        }
        D[kw + nw - 1] = acc;
    }
    std::vector<double> sig(nlines);
    double pair_terms = 0.0, max_sig = 0.0;
    for (int kk = 0; kk < nk; ++kk)
        for (int c = 0; c < nc; ++c) {
            const int kw = c - (nw - 1);
            double diag = 0.0;
            int self = 0;
            if ((kk % 2) == 0 && (kw % 2) == 0 && kw / 2 > -W && kw / 2 < W) {
                diag = b2at(kw / 2 + W - 1, kw / 2 + W - 1);
                self = 1;
            }
            pair_terms += 0.5 * (static_cast<double>(kk + 1) * nsplit[c] + self);
            const double v = 0.5 * ((kk + 1) * D[c] + diag);
            sig[static_cast<size_t>(kk) * nc + c] = v;
            max_sig = std::max(max_sig, v);
        }
    if (factors) {
        // kappa-dependent bicoherence: weighted 2-D autoconvolution of r^2 on the host
        if (bs.kind == SRM3_BISPEC_DENSE) {
            int Mk = 1;
            while (Mk < 2 * nk - 1) Mk *= 2;
            if (static_cast<double>(Mk) * (4.0 * W - 3) * ncw > 4e9)
                return fail(SRM3_E_UNSUPPORTED, "line factors with a dense table: grid too large for the plan-time sums");
        }
        std::vector<double> Q, rmag;
        if (!lrx.empty()) {
            rmag.resize(nlines);
            for (size_t l = 0; l < nlines; ++l) rmag[l] = std::hypot(lrx[2 * l], lrx[2 * l + 1]);
        }
        line_pair_sums(nk, nw, W, rmag.empty() ? nullptr : rmag.data(), bs.kind, bs.g2, bs.b2, Q);
        max_sig = 0.0;
        for (size_t l = 0; l < nlines; ++l) {
            const double c2 = lcx.empty() ? 1.0 : lcx[2 * l] * lcx[2 * l] + lcx[2 * l + 1] * lcx[2 * l + 1];
            sig[l] = c2 * Q[l];
            max_sig = std::max(max_sig, sig[l]);
        }
    }
    if (!hashed && max_sigma(max_sig, bs.cap, 1.0) >= 1.0)
        return fail(SRM3_E_PURE_NEGATIVE, "a line has sum of b^2 = %.6g >= 1: pure spectrum not positive",
                    max_sigma(max_sig, bs.cap, 1.0));

    std::unique_ptr<srm3_plan_s> p(new (std::nothrow) srm3_plan_s);
    if (!p) return fail(SRM3_E_NOMEM, "host allocation failed");
    p->precision = precision;
    p->dk = grid->d_kappa;
    p->dw = grid->d_omega;
    p->cap = bs.cap;
    p->max_sig = max_sig;
    p->gaussian = bs.kind == SRM3_BISPEC_NONE;
    if (bs.kind == SRM3_BISPEC_SEPARABLE && bs.beta_mode == SRM3_BETA_ZERO)
        p->g2_host.assign(bs.g2, bs.g2 + ncw);   // rank-one weights: the 2-D FFT pair sum applies
    p->pair_terms = p->gaussian ? 0.0 : pair_terms;
    p->hashed = hashed;
    p->fixed_spectrum = bispectrum && bispectrum->kind == SRM3_BISPEC_PRODUCT;
    p->hash_key = hash_key;
    p->hash_scale = hash_scale;
    Geometry &g = p->g;
    g.nk = nk;
    g.nw = nw;
    g.W = W;
    g.nc = nc;
    g.ncw = ncw;
    g.nx = nx;
    g.nt = nt;
    g.R = pairsum_rows_per_wave(nk, precision);
    g.nkp = ((nk + g.R - 1) / g.R) * g.R;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) return dev_err(e, "hipGetDevice");
    e = prepare_transforms(precision);
    if (e != hipSuccess) return dev_err(e, "hipFuncSetAttribute");

    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    {
        // complex weight table W = sqrt(b2) e^{i beta}, built on the device
        DevBuf g2d, b2d, betad;
        if (bs.kind == SRM3_BISPEC_SEPARABLE && (s = upload_bytes(g2d, bs.g2, ncw * sizeof(double), st))) return s;
        if (bs.kind == SRM3_BISPEC_DENSE &&
            (s = upload_bytes(b2d, bs.b2, static_cast<size_t>(ncw) * ncw * sizeof(double), st)))
            return s;
        if (bs.kind != SRM3_BISPEC_NONE && bs.beta_mode == SRM3_BETA_TABLE &&
            (s = upload_bytes(betad, bs.beta, static_cast<size_t>(ncw) * ncw * sizeof(uint32_t), st)))
            return s;
        const size_t wbytes = static_cast<size_t>(ncw) * ncw * 2 * (precision == SRM3_FP64 ? 8 : 4);
        e = p->wtab.alloc(wbytes);
        if (e != hipSuccess) return fail(SRM3_E_NOMEM, "hipMalloc(%zu): %s", wbytes, hipGetErrorString(e));
        e = launch_wtable(precision, W, bs.kind, static_cast<const double *>(g2d.p),
                          static_cast<const double *>(b2d.p), bs.beta_mode, static_cast<const uint32_t *>(betad.p),
                          bs.beta_seed, p->wtab.p, st);
        if (e != hipSuccess) return dev_err(e, "weight-table kernel");
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return dev_err(e, "hipStreamSynchronize");
    }
    if ((s = upload_bytes(p->S, S, nlines * sizeof(double), st))) return s;
    if ((s = upload_bytes(p->sig, sig.data(), nlines * sizeof(double), st))) return s;
    if (!lcx.empty() && (s = upload_bytes(p->lc, lcx.data(), lcx.size() * sizeof(double), st))) return s;
    if (!lrx.empty() && (s = upload_bytes(p->lr, lrx.data(), lrx.size() * sizeof(double), st))) return s;
    if (!hcx.empty() && (s = upload(p->wtab, hcx, precision, st))) return s;   // the prescribed H as the weights
    if ((s = upload(p->tw_t, pass_twiddles(nt), precision, st))) return s;
    if ((s = upload(p->tw_x, pass_twiddles(nx), precision, st))) return s;
    if (hashed) {
        // per-line raw sums of the generated bicoherence, on the device, then the cap check
        e = launch_pairsum_hash(g, precision, hash_key, hash_scale, 1, nullptr, static_cast<double *>(p->sig.p), st);
        if (e != hipSuccess) return dev_err(e, "hashed bispectrum sums");
        if ((e = hipMemcpyAsync(sig.data(), p->sig.p, nlines * sizeof(double), hipMemcpyDeviceToHost, st)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return dev_err(e, "copy of the raw sums");
        p->max_sig = *std::max_element(sig.begin(), sig.end());
        if (max_sigma(p->max_sig, bs.cap, 1.0) >= 1.0)
            return fail(SRM3_E_PURE_NEGATIVE, "a line has sum of b^2 = %.6g >= 1: pure spectrum not positive",
                        max_sigma(p->max_sig, bs.cap, 1.0));
    }
    if ((s = refresh_amp_table(p.get(), st))) return s;
    *out_plan = p.release();
    return SRM3_OK;
}

srm3_status srm3_wind_factors(const srm3_grid *grid, const double *S, double alpha, double cap, int32_t support_w,
                              double *line_c, double *line_r, double *sigma, int32_t *sweeps)
{
    g_err[0] = 0;
    if (!grid || !S || !line_c || !line_r) return fail(SRM3_E_INVALID, "NULL argument");
    const int nk = grid->n_kappa, nw = grid->n_omega;
    if (nk < 1 || nw < 1) return fail(SRM3_E_INVALID, "n_kappa=%d n_omega=%d must be >= 1", nk, nw);
    if (support_w < 1 || support_w > nw) return fail(SRM3_E_INVALID, "support_w=%d must be in [1, n_omega]", support_w);
    if (!(alpha > 0) || !std::isfinite(alpha)) return fail(SRM3_E_INVALID, "alpha must be finite and > 0");
    if (!(cap < 1.0) || !std::isfinite(cap)) return fail(SRM3_E_INVALID, "cap must be < 1");
    const size_t nl = static_cast<size_t>(nk) * (2 * nw - 1);
    srm3_status s = check_spectrum(S, nl);
    if (s) return s;
    std::vector<double> c, r;
    int it = 0;
    if ((s = wind_factors(nk, nw, support_w, S, alpha, cap, c, r, &it, nullptr))) return s;
    for (size_t l = 0; l < nl; ++l) {
        line_c[l] = c[l];
        line_r[l] = r[l];
        if (sigma) sigma[l] = r[l] > 0.0 ? 1.0 - 1.0 / (r[l] * r[l]) : 0.0;
    }
    if (sweeps) *sweeps = it;
    return SRM3_OK;
}

srm3_status srm3_product_factors(const srm3_grid *grid, const double *S, const double *F, const double *G,
                                 const double *H, int32_t support_w, double cap, double *line_c, double *line_rho,
                                 double *sigma, int32_t *sweeps)
{
    g_err[0] = 0;
    if (!grid || !S || !F || !G || !line_c || !line_rho) return fail(SRM3_E_INVALID, "NULL argument");
    const int nk = grid->n_kappa, nw = grid->n_omega;
    if (nk < 1 || nw < 1) return fail(SRM3_E_INVALID, "n_kappa=%d n_omega=%d must be >= 1", nk, nw);
    if (support_w < 1 || support_w > nw) return fail(SRM3_E_INVALID, "support_w=%d must be in [1, n_omega]", support_w);
    if (!(grid->d_kappa > 0) || !(grid->d_omega > 0)) return fail(SRM3_E_INVALID, "d_kappa/d_omega must be > 0");
    if (!(cap < 1.0) || !std::isfinite(cap)) return fail(SRM3_E_INVALID, "cap must be < 1");
    const size_t nl = static_cast<size_t>(nk) * (2 * nw - 1);
    srm3_status s = check_spectrum(S, nl);
    if (s) return s;
    std::vector<double> c, rho, sig;
    int it = 0;
    if ((s = product_factors(nk, nw, support_w, S, F, G, H, grid->d_kappa, grid->d_omega, cap, c, rho, &it, nullptr,
                             &sig)))
        return s;
    for (size_t l = 0; l < 2 * nl; ++l) {
        line_c[l] = c[l];
        line_rho[l] = rho[l];
    }
    if (sigma)
        for (size_t l = 0; l < nl; ++l) sigma[l] = sig[l];
    if (sweeps) *sweeps = it;
    return SRM3_OK;
}

srm3_status srm3_process_plan(const srm3_process_grid *grid, const double *S, const srm3_bispectrum *bispectrum,
                              int32_t precision, void *hip_stream, srm3_plan_t *out_plan)
{
    g_err[0] = 0;
    if (!out_plan) return fail(SRM3_E_INVALID, "out_plan is NULL");
    *out_plan = nullptr;
    if (!grid || !S) return fail(SRM3_E_INVALID, "grid/S is NULL");
    const int n = grid->n_omega;
    if (n < 1) return fail(SRM3_E_INVALID, "n_omega=%d must be >= 1", n);
    // the wave with one kappa line (d_kappa = 1 leaves the amplitude 2 sqrt(S dw)),
    // no spectrum at negative frequencies and no pair with a negative partner
    srm3_grid wg{};
    wg.n_kappa = 1;
    wg.n_omega = n;
    wg.d_kappa = 1.0;
    wg.d_omega = grid->d_omega;
    wg.n_x = 1;
    wg.n_t = grid->n_t;
    std::vector<double> Sw(2 * static_cast<size_t>(n) - 1, 0.0);
    for (int k = 0; k < n; ++k) Sw[n - 1 + k] = S[k];
    const srm3_spectrum spec{Sw.data()};
    srm3_bispectrum wb{};
    std::vector<double> g2w, b2w;
    std::vector<uint32_t> betaw;
    long long process_pairs = 0;
    if (bispectrum && (bispectrum->kind == SRM3_BISPEC_WIND || bispectrum->kind == SRM3_BISPEC_PRODUCT ||
                       bispectrum->kind == SRM3_BISPEC_HASHED ||
                       bispectrum->line_c || bispectrum->line_r))
        return fail(SRM3_E_UNSUPPORTED, "process plans take frequency-only bicoherence");
    if (bispectrum && bispectrum->kind != SRM3_BISPEC_NONE) {
        const srm3_bispectrum &q = *bispectrum;
        const int W = q.support_w;
        if (W < 1 || W > n) return fail(SRM3_E_INVALID, "support_w=%d must be in [1, n_omega=%d]", W, n);
        const size_t nw2 = 2 * static_cast<size_t>(W) - 1;
        wb = q;
        if (q.kind == SRM3_BISPEC_SEPARABLE) {
            if (!q.g2) return fail(SRM3_E_INVALID, "g2 is NULL");
            g2w.assign(nw2, 0.0);
            for (int i = 0; i < W; ++i) g2w[W - 1 + i] = q.g2[i];
            wb.g2 = g2w.data();
        } else if (q.kind == SRM3_BISPEC_DENSE) {
            if (!q.b2) return fail(SRM3_E_INVALID, "b2 is NULL");
            b2w.assign(nw2 * nw2, 0.0);
            for (int i = 0; i < W; ++i)
                for (int j = 0; j < W; ++j) b2w[(W - 1 + i) * nw2 + (W - 1 + j)] = q.b2[static_cast<size_t>(i) * W + j];
            wb.b2 = b2w.data();
        }
        if (q.beta_mode == SRM3_BETA_TABLE && q.beta) {
            betaw.assign(nw2 * nw2, 0u);
            for (int i = 0; i < W; ++i)
                for (int j = 0; j < W; ++j)
                    betaw[(W - 1 + i) * nw2 + (W - 1 + j)] = q.beta[static_cast<size_t>(i) * W + j];
            wb.beta = betaw.data();
        }
        // pairs i + j = k, i >= j >= 0, i < W, outputs k < n
        for (int k = 0; k < n; ++k) process_pairs += std::max(0, k / 2 - std::max(0, k - W + 1) + 1);
    } else if (bispectrum) {
        wb = *bispectrum;
    }
    srm3_plan_t p = nullptr;
    srm3_status s = srm3_plan(&wg, &spec, bispectrum ? &wb : nullptr, precision, hip_stream, &p);
    if (s) return s;
    p->process = true;
    if (!p->gaussian) {
        p->pair_terms = static_cast<double>(process_pairs);
        if ((s = srm3_plan_set_algorithm(p, SRM3_ALGO_KAPPA_FFT, hip_stream))) {
            srm3_destroy(p);
            return s;
        }
    }
    *out_plan = p;
    return SRM3_OK;
}

srm3_status srm3_set_spectrum(srm3_plan_t plan, const srm3_spectrum *spectrum, void *hip_stream)
{
    g_err[0] = 0;
    if (!plan || !spectrum || !spectrum->S) return fail(SRM3_E_INVALID, "plan/spectrum is NULL");
    if (plan->fixed_spectrum)
        return fail(SRM3_E_UNSUPPORTED, "a product bispectrum's line factors were derived from the plan's spectrum");
    const size_t n = static_cast<size_t>(plan->g.nk) * plan->g.nc;
    const double *src = spectrum->S;
    std::vector<double> Sw;
    if (plan->process) {
        // one-sided [n_omega] -> the line layout, zero at negative frequencies
        const int nw = plan->g.nw;
        srm3_status s = check_spectrum(spectrum->S, static_cast<size_t>(nw));
        if (s) return s;
        Sw.assign(n, 0.0);
        for (int k = 0; k < nw; ++k) Sw[nw - 1 + k] = spectrum->S[k];
        src = Sw.data();
    }
    srm3_status s = check_spectrum(src, n);
    if (s) return s;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipMemcpyAsync(plan->S.p, src, n * sizeof(double), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return dev_err(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return dev_err(e, "hipStreamSynchronize");
    return refresh_amp_table(plan, st);
}

srm3_status srm3_spectrum_kaimal_davenport(const srm3_grid *grid, const srm3_kaimal_davenport *params,
                                           double *S_dev, void *hip_stream)
{
    g_err[0] = 0;
    if (!grid || !params || !S_dev) return fail(SRM3_E_INVALID, "NULL argument");
    if (grid->n_kappa < 1 || grid->n_omega < 1 || !(grid->d_kappa > 0) || !(grid->d_omega > 0))
        return fail(SRM3_E_INVALID, "bad grid");
    if (!(params->U > 0) || !(params->z > 0) || !(params->u_star >= 0) || !(params->lam > 0) ||
        !std::isfinite(params->U) || !std::isfinite(params->z) || !std::isfinite(params->u_star) ||
        !std::isfinite(params->lam))
        return fail(SRM3_E_INVALID, "spectrum parameters must be finite (U, z, lambda > 0, u* >= 0)");
    hipError_t e = launch_spectrum(grid->n_kappa, grid->n_omega, grid->d_kappa, grid->d_omega, params->u_star,
                                   params->z, params->U, params->lam, S_dev, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return dev_err(e, "spectrum kernel");
    return SRM3_OK;
}

void srm3_destroy(srm3_plan_t plan)
{
    if (!plan) return;
    (void)hipDeviceSynchronize();
    for (auto &r : plan->recs) {
        if (r.a) (void)hipEventDestroy(r.a);
        if (r.b) (void)hipEventDestroy(r.b);
    }
    for (auto ev : plan->pool) (void)hipEventDestroy(ev);
    delete plan;
}

srm3_status srm3_workspace_bytes(srm3_plan_t plan, int32_t batch, size_t *bytes)
{
    if (!plan || !bytes || batch < 0) return fail(SRM3_E_INVALID, "bad argument");
    *bytes = workspace_bytes(plan->g, plan->precision, batch);
    if (kfft_family(plan->algo)) *bytes += kfft_workspace_bytes(plan->g, plan->kg, plan->precision, batch);
    return SRM3_OK;
}

srm3_status srm3_workspace_fill(srm3_plan_t plan, int32_t batch, uint32_t word, void *hip_stream)
{
    g_err[0] = 0;
    if (!plan || batch < 0) return fail(SRM3_E_INVALID, "bad argument");
    if (batch == 0) return SRM3_OK;
    if (batch > 65535) return fail(SRM3_E_UNSUPPORTED, "batch %d too large", batch);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    srm3_status s = ensure_workspace(plan, batch, st);
    if (s) return s;
    hipError_t e = launch_fill_u32(plan->ws.p, plan->ws.n / 4, word, st);
    if (e == hipSuccess && kfft_family(plan->algo)) e = launch_fill_u32(plan->kws.p, plan->kws.n / 4, word, st);
    if (e != hipSuccess) return dev_err(e, "fill kernel");
    return SRM3_OK;
}

srm3_status srm3_pair_terms(srm3_plan_t plan, double *terms)
{
    if (!plan || !terms) return fail(SRM3_E_INVALID, "bad argument");
    *terms = plan->pair_terms;
    return SRM3_OK;
}

srm3_status srm3_rows_per_wave(srm3_plan_t plan, int32_t *rows)
{
    if (!plan || !rows) return fail(SRM3_E_INVALID, "bad argument");
    *rows = plan->g.R;
    return SRM3_OK;
}

srm3_status srm3_plan_set_algorithm(srm3_plan_t plan, int32_t algorithm, void *hip_stream)
{
    g_err[0] = 0;
    if (!plan) return fail(SRM3_E_INVALID, "plan is NULL");
    if (algorithm == SRM3_ALGO_DIRECT) {
        plan->algo = SRM3_ALGO_DIRECT;
        return SRM3_OK;
    }
    if (algorithm != SRM3_ALGO_KAPPA_FFT && algorithm != SRM3_ALGO_FFT2D && algorithm != SRM3_ALGO_MFMA)
        return fail(SRM3_E_INVALID, "algorithm %d", algorithm);
    if (plan->hashed)
        return fail(SRM3_E_UNSUPPORTED, "a bispectrum generated per pair has kappa-dependent weights: direct form only");
    if (algorithm == SRM3_ALGO_MFMA) {
        plan->algo = SRM3_ALGO_MFMA;
        return SRM3_OK;
    }
    if (plan->algo == algorithm) return SRM3_OK;
    KfftGeom k = kfft_geometry(plan->g, plan->process);
    std::string why;
    if (!kfft_supported(plan->g, k, plan->precision, &why))
        return fail(SRM3_E_UNSUPPORTED, "kappa-FFT pair sum: %s", why.c_str());
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    srm3_status s;
    if (algorithm == SRM3_ALGO_FFT2D) {
        if (plan->g2_host.empty())
            return fail(SRM3_E_UNSUPPORTED, "the 2-D FFT pair sum needs rank-one weights (separable b^2, beta = 0)");
        int L = 1;
        while (L < 2 * plan->g.ncw - 1) L *= 2;
        const int lmax = plan->precision == SRM3_FP64 ? 8192 : 16384;   // one row transform in 128 KB of LDS
        if (L > lmax) return fail(SRM3_E_UNSUPPORTED, "2-D FFT pair sum: frequency transform %d above %d", L, lmax);
        k.L = L;
        std::vector<double> g(plan->g2_host.size());
        for (size_t i = 0; i < g.size(); ++i) g[i] = std::sqrt(plan->g2_host[i]);
        if ((s = upload(plan->gw, g, plan->precision, st))) return s;
        if ((s = upload(plan->tw_l, twiddles(L), plan->precision, st))) return s;
    } else {
        const size_t e2 = plan->precision == SRM3_FP64 ? 16 : 8;
        hipError_t e = plan->wsh.alloc(static_cast<size_t>(k.wh_rows) * k.nca * e2);
        if (e != hipSuccess) return fail(SRM3_E_NOMEM, "weight table hipMalloc: %s", hipGetErrorString(e));
        if ((e = launch_wsh(plan->precision, plan->wtab.p, plan->g, k, plan->wsh.p, st)) != hipSuccess)
            return dev_err(e, "sheared weight table kernel");
    }
    if ((s = upload(plan->tw_k, twiddles(k.M), plan->precision, st))) return s;
    plan->kg = k;
    plan->kws_batch = 0;
    plan->algo = algorithm;
    return SRM3_OK;
}

srm3_status srm3_plan_set_mfma_shape(srm3_plan_t plan, int32_t shape)
{
    g_err[0] = 0;
    if (!plan) return fail(SRM3_E_INVALID, "plan is NULL");
    if (shape < 0 || shape >= kMfmaShapes) return fail(SRM3_E_INVALID, "matrix-core tile shape %d", shape);
    plan->mfma_shape = shape;
    return SRM3_OK;
}

srm3_status srm3_mfma_shape(int32_t precision, int32_t shape, int32_t *rows, int32_t *cols)
{
    if (shape < 0 || shape >= kMfmaShapes || !rows || !cols ||
        (precision != SRM3_FP32 && precision != SRM3_FP64))
        return fail(SRM3_E_INVALID, "bad argument");
    const MfmaShape m = mfma_shape(precision, shape);
    *rows = 16 * m.rt;
    *cols = 16 * m.ct;
    return SRM3_OK;
}

srm3_status srm3_algorithm_terms(srm3_plan_t plan, double *terms)
{
    if (!plan || !terms) return fail(SRM3_E_INVALID, "bad argument");
    *terms = kfft_family(plan->algo) ? kfft_terms(plan->g, plan->kg) : plan->pair_terms;
    return SRM3_OK;
}

srm3_status srm3_generate(srm3_plan_t plan, const uint64_t *seeds, int32_t batch, void *out_dev, void *hip_stream)
{
    g_err[0] = 0;
    srm3_status s = check_batch(plan, seeds, batch, out_dev);
    if (s) return s;
    if (batch == 0) return SRM3_OK;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if ((s = ensure_workspace(plan, batch, st))) return s;
    const Workspace ws = carve_workspace(plan->g, plan->precision, batch, plan->ws.p);
    // zero bicoherence: the t-transform draws the phases itself (no phase rows)
    if (plan->gaussian && !plan->lr.p) return run_back(plan, 2, nullptr, batch, ws, out_dev, st, seeds);
    if ((s = run_front(plan, seeds, batch, ws, st))) return s;
    return run_back(plan, 0, nullptr, batch, ws, out_dev, st);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free generation: the workspace lives in a fixed device array of
// this library (one copy per GPU, kept until the process ends) instead of the
// plan's own buffer, so that callers that cannot allocate device memory (code
// under stream capture, serving loops, harnesses that forbid it) can generate.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per GPU
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of the scratch array, looked up once per
// device with that device current (the array's host-side name is not a device
// address).
srm3_status scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return dev_err(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(SRM3_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return dev_err(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SRM3_OK;
}

// Profiling records events (and may create them): off for the duration of an
// allocation-free call.
struct ProfPause {
    srm3_plan_t p;
    bool was;
    explicit ProfPause(srm3_plan_t plan) : p(plan), was(plan->prof) { p->prof = false; }
    ~ProfPause() { p->prof = was; }
};

}  // namespace

extern "C" {

srm3_status srm3_generate_noalloc(srm3_plan_t plan, const uint64_t *seeds, int32_t batch, void *out_dev,
                                  void *hip_stream)
{
    g_err[0] = 0;
    srm3_status s = check_batch(plan, seeds, batch, out_dev);
    if (s) return s;
    if (batch == 0) return SRM3_OK;
    auto al = [](size_t x) { return (x + 255) & ~static_cast<size_t>(255); };
    const size_t main_bytes = al(workspace_bytes(plan->g, plan->precision, batch));
    const size_t need = main_bytes + (kfft_family(plan->algo) ? kfft_workspace_bytes(plan->g, plan->kg,
                                                                                     plan->precision, batch) : 0);
    if (need > kScratchBytes)
        return fail(SRM3_E_UNSUPPORTED, "allocation-free generation of %d realizations needs %zu bytes of "
                    "workspace; the library's scratch array holds %zu", batch, need, kScratchBytes);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return dev_err(e, "hipGetDevice");
    if (dev != plan->device)
        return fail(SRM3_E_INVALID, "current device %d is not the plan's device %d", dev, plan->device);
    void *base = nullptr;
    if ((s = scratch_address(&base))) return s;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    ProfPause pause(plan);
    const Workspace ws = carve_workspace(plan->g, plan->precision, batch, base);
    if (kfft_family(plan->algo)) {
        // the kappa-DFT stage takes its workspace from the scratch too
        const KfftWorkspace kw = carve_kfft(plan->g, plan->kg, plan->precision, batch,
                                            static_cast<char *>(base) + main_bytes);
        if ((s = run_front_kfft(plan, seeds, batch, ws, kw, st))) return s;
    } else if (plan->gaussian && !plan->lr.p) {
        return run_back(plan, 2, nullptr, batch, ws, out_dev, st, seeds);
    } else if ((s = run_front(plan, seeds, batch, ws, st))) {
        return s;
    }
    return run_back(plan, 0, nullptr, batch, ws, out_dev, st);
}

srm3_status srm3_coefficients(srm3_plan_t plan, const uint64_t *seeds, int32_t batch, void *C_dev, void *hip_stream)
{
    g_err[0] = 0;
    srm3_status s = check_batch(plan, seeds, batch, C_dev);
    if (s) return s;
    if (batch == 0) return SRM3_OK;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if ((s = ensure_workspace(plan, batch, st))) return s;
    const Workspace ws = carve_workspace(plan->g, plan->precision, batch, plan->ws.p);
    if ((s = run_front(plan, seeds, batch, ws, st))) return s;
    hipError_t e = launch_assemble(plan->g, plan->precision, plan_amp(plan), plan->wtab.p, batch, ws, C_dev, st);
    if (e != hipSuccess) return dev_err(e, "assemble kernel");
    return SRM3_OK;
}

srm3_status srm3_transform(srm3_plan_t plan, const void *C_dev, int32_t batch, void *out_dev, void *hip_stream)
{
    g_err[0] = 0;
    srm3_status s = check_batch(plan, C_dev, batch, out_dev);
    if (s) return s;
    if (batch == 0) return SRM3_OK;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if ((s = ensure_workspace(plan, batch, st))) return s;
    const Workspace ws = carve_workspace(plan->g, plan->precision, batch, plan->ws.p);
    return run_back(plan, 1, C_dev, batch, ws, out_dev, st);
}

srm3_status srm3_profile_enable(srm3_plan_t plan, int32_t enable)
{
    if (!plan) return fail(SRM3_E_INVALID, "plan is NULL");
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return dev_err(e, "hipDeviceSynchronize");
    for (auto &r : plan->recs) {
        if (r.a) plan->pool.push_back(r.a);
        if (r.b) plan->pool.push_back(r.b);
    }
    plan->recs.clear();
    plan->prof = enable != 0;
    return SRM3_OK;
}

srm3_status srm3_profile_read(srm3_plan_t plan, srm3_profile *out)
{
    if (!plan || !out) return fail(SRM3_E_INVALID, "bad argument");
    std::memset(out, 0, sizeof *out);
    for (auto &r : plan->recs) {
        if (!r.a || !r.b) continue;
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return dev_err(e, "hipEventSynchronize");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return dev_err(e, "hipEventElapsedTime");
        out->ms[r.kernel] += ms;
        out->launches[r.kernel] += 1;
    }
    return SRM3_OK;
}

}  // extern "C"

// ===========================================================================
// Uneven batches: requests with mixed plans in one persistent pair-sum launch
// ===========================================================================
struct srm3_batch_s {
    int precision = 0;
    int n = 0;
    int flags = 0;
    std::vector<srm3_request> req;     // caller order
    struct Group {
        srm3_plan_t plan;
        std::vector<int> members;      // caller indices, slot = position
        Geometry g;                    // with the batch's R
        size_t ws_off = 0;
        int first = 0;                 // offset of the group in the device arrays
        int mode = 0;                  // 0: items of the persistent launch; 1: the plan's kappa-DFT
                                       // pair sum over the group; 2: zero bicoherence, no pair sum
        size_t kws_off = 0;            // kappa-DFT workspace of the group (mode 1)
    };
    std::vector<Group> groups;
    int R = 0;                         // rows per wave of the persistent launch
    bool mfma = false;                 // its items are those of the matrix-core pair sum
    int mfma_shape = 0;                // and their tile shape
    int blocks_per_cu = 2;
    int n_cu = 256;
    DevBuf ws, seeds, scales, sptr, outs, preq, pitem, qbegin, qnext;
    int n_items = 0;
    uint64_t *seeds_host = nullptr;    // pinned staging
    hipEvent_t copy_done = nullptr;
    bool copy_pending = false;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    double pair_terms = 0;
    bool tuned = false;
    bool ran = false, ps_timed = false;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;     // pair sum (direct runs)
    hipEvent_t run_a = nullptr, run_b = nullptr;   // whole run
};

namespace {

// Relative cost of one work item: kappa steps times the widest partner range
// of its column tiles.
double item_cost_impl(const Geometry &g, int R, int kb, int cg)
{
    const int wpb = waves_per_block();
    const int nct = (g.nc + 63) / 64;
    int widest = 0;
    for (int w = 0; w < wpb; ++w) {
        const int ct = cg * wpb + w;
        if (ct >= nct) break;
        const int kw_lo = ct * 64 - (g.nw - 1);
        const int kw_hi = std::min(ct * 64 + 63, g.nc - 1) - (g.nw - 1);
        const int lo = std::max(-(g.W - 1), kw_lo - (g.W - 1));
        const int hi = std::min(g.W - 1, kw_hi + (g.W - 1));
        widest = std::max(widest, hi - lo + 1);
    }
    return static_cast<double>(kb * R / 2 + R / 2) * widest;
}

// Relative cost of a matrix-core item (row group kb, column group cg): its
// kappa splits times the widest partner range of its waves' column tiles.
double mfma_item_cost_impl(const Geometry &g, int kb, int cg, int precision, int shape)
{
    const int rows = mfma_rows_per_group(precision, shape), cols = mfma_cols_per_group(precision, shape);
    const int wcols = cols / waves_per_block();
    int widest = 0;
    for (int c0 = cg * cols; c0 < std::min(g.nc, (cg + 1) * cols); c0 += wcols) {
        const int kw_lo = c0 - (g.nw - 1);
        const int kw_hi = std::min(c0 + wcols - 1, g.nc - 1) - (g.nw - 1);
        const int lo = std::max(-(g.W - 1), kw_lo - (g.W - 1));
        const int hi = std::min(g.W - 1, kw_hi + (g.W - 1));
        widest = std::max(widest, hi - lo + 1);
    }
    const int kk_max = std::min(kb * rows + rows - 1, g.nk - 1);
    return static_cast<double>(kk_max / 2 + 1) * widest;
}

// (Re)build layouts and work queues for rows-per-wave R and grid size.
srm3_status batch_layout(srm3_batch_t b, int R, hipStream_t st)
{
    b->R = R;
    size_t off = 0;
    auto al = [](size_t x) { return (x + 255) & ~static_cast<size_t>(255); };
    int first = 0;
    for (auto &gr : b->groups) {
        gr.g = gr.plan->g;
        gr.mode = gr.plan->gaussian ? 2 : (kfft_family(gr.plan->algo) ? 1 : 0);
        if (gr.mode == 0) {
            gr.g.R = rows_for(gr.g.nk, b->precision, R);
            gr.g.nkp = ((gr.g.nk + gr.g.R - 1) / gr.g.R) * gr.g.R;
            if (gr.g.R != R)
                return fail(SRM3_E_UNSUPPORTED, "a %dx%d grid needs rows per wave %d != %d of the batch", gr.g.nk,
                            gr.g.nw, gr.g.R, R);
        }
        const int nb = static_cast<int>(gr.members.size());
        gr.ws_off = off;
        gr.first = first;
        off += al(workspace_bytes(gr.g, b->precision, nb));
        if (gr.mode == 1) {
            gr.kws_off = off;
            off += al(kfft_workspace_bytes(gr.g, gr.plan->kg, b->precision, nb));
        }
        first += nb;
    }
    if (b->ws.n < off) {
        hipError_t e = b->ws.alloc(off);
        if (e != hipSuccess) return fail(SRM3_E_NOMEM, "batch workspace hipMalloc(%zu): %s", off, hipGetErrorString(e));
    }
    // per-request descriptors (device order = group order) and work items
    const size_t rb = persistent_req_bytes(), ib = persistent_item_bytes();
    std::vector<unsigned char> reqs(rb * b->n);
    struct It {
        int req, kb, cg;
        double cost;
    };
    std::vector<std::vector<It>> per_req(b->n);
    std::vector<double> req_cost(b->n, 0.0);
    const size_t e = b->precision == SRM3_FP64 ? 8 : 4;
    for (auto &gr : b->groups) {
        const Workspace ws = carve_workspace(gr.g, b->precision, static_cast<int>(gr.members.size()),
                                             static_cast<char *>(b->ws.p) + gr.ws_off);
        const size_t lines = static_cast<size_t>(gr.g.nk) * gr.g.nc;
        const size_t plane3 = a_slots(b->precision) * gr.g.ncw * gr.g.nkp;
        const int mr = mfma_rows_per_group(b->precision, b->mfma_shape);
        const int mc = mfma_cols_per_group(b->precision, b->mfma_shape);
        const int nrb = b->mfma ? (gr.g.nk + mr - 1) / mr : gr.g.nkp / gr.g.R;
        const int ncg = b->mfma ? (gr.g.nc + mc - 1) / mc
                                : ((gr.g.nc + 63) / 64 + waves_per_block() - 1) / waves_per_block();
        if (gr.mode != 0) continue;   // no items in the persistent launch
        for (size_t slot = 0; slot < gr.members.size(); ++slot) {
            const int d = gr.first + static_cast<int>(slot);
            fill_persistent_req(reqs.data() + rb * d, gr.g, static_cast<char *>(ws.zrow) + slot * lines * 2 * e,
                                static_cast<char *>(ws.zcol) + slot * plane3 * e,
                                static_cast<char *>(ws.tsum) + slot * lines * 2 * e, gr.plan->wtab.p);
            for (int kb = nrb - 1; kb >= 0; --kb)
                for (int cg = 0; cg < ncg; ++cg) {
                    const double c = b->mfma ? mfma_item_cost_impl(gr.g, kb, cg, b->precision, b->mfma_shape)
                                             : item_cost_impl(gr.g, gr.g.R, kb, cg);
                    per_req[d].push_back({d, kb, cg, c});
                    req_cost[d] += c;
                }
        }
    }
    // Order: requests by descending cost, items of a request heaviest first;
    // cut into kXcds contiguous runs of equal cost (one queue per XCD).
    std::vector<int> order(b->n);
    for (int i = 0; i < b->n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return req_cost[x] > req_cost[y]; });
    std::vector<It> all;
    double total = 0.0;
    for (int d : order) {
        auto &v = per_req[d];
        std::stable_sort(v.begin(), v.end(), [](const It &x, const It &y) { return x.cost > y.cost; });
        for (auto &it : v) {
            all.push_back(it);
            total += it.cost;
        }
    }
    std::vector<int> qbegin(kXcds + 1, 0);
    double acc = 0.0;
    int q = 1;
    for (size_t i = 0; i < all.size(); ++i) {
        while (q < kXcds && acc >= total * q / kXcds) qbegin[q++] = static_cast<int>(i);
        acc += all[i].cost;
    }
    while (q <= kXcds) qbegin[q++] = static_cast<int>(all.size());
    std::vector<unsigned char> items(ib * std::max<size_t>(1, all.size()));
    for (size_t i = 0; i < all.size(); ++i) fill_persistent_item(items.data() + ib * i, all[i].req, all[i].kb, all[i].cg);
    b->n_items = static_cast<int>(all.size());
    srm3_status s;
    if ((s = upload_bytes(b->preq, reqs.data(), reqs.size(), st))) return s;
    if ((s = upload_bytes(b->pitem, items.data(), items.size(), st))) return s;
    if ((s = upload_bytes(b->qbegin, qbegin.data(), qbegin.size() * sizeof(int), st))) return s;
    if (!b->qnext.p) {
        hipError_t er = b->qnext.alloc(kXcds * sizeof(int));
        if (er != hipSuccess) return fail(SRM3_E_NOMEM, "hipMalloc: %s", hipGetErrorString(er));
    }
    return SRM3_OK;
}

// The launch sequence of one run (stream-ordered; capturable).
srm3_status batch_launch(srm3_batch_t b, hipStream_t st, bool time_pairsum)
{
    for (auto &gr : b->groups) {
        Workspace ws = carve_workspace(gr.g, b->precision, static_cast<int>(gr.members.size()),
                                       static_cast<char *>(b->ws.p) + gr.ws_off);
        if (gr.mode != 0) ws.zcol = nullptr;   // no a operand planes needed
        hipError_t e = launch_phases(gr.g, b->precision, nullptr, static_cast<const uint64_t *>(b->seeds.p) + gr.first,
                                     static_cast<int>(gr.members.size()), ws,
                                     static_cast<const double *>(gr.plan->lr.p), st);
        if (e != hipSuccess) return dev_err(e, "phase kernel");
    }
    if (time_pairsum) (void)hipEventRecord(b->ev_a, st);
    hipError_t e;
    for (auto &gr : b->groups) {
        if (gr.mode != 1) continue;
        const int nb = static_cast<int>(gr.members.size());
        const Workspace ws = carve_workspace(gr.g, b->precision, nb, static_cast<char *>(b->ws.p) + gr.ws_off);
        const KfftWorkspace kw = carve_kfft(gr.g, gr.plan->kg, b->precision, nb,
                                            static_cast<char *>(b->ws.p) + gr.kws_off);
        e = launch_kfft_pairsum(b->precision, gr.g, gr.plan->kg, plan_ktab(gr.plan), nb, ws, kw, st);
        if (e != hipSuccess) return dev_err(e, "kappa-DFT pair-sum kernels");
    }
    if (b->n_items > 0) {
        e = launch_pairsum_persistent(b->precision, b->R, b->preq.p, b->pitem.p,
                                      static_cast<const int *>(b->qbegin.p), static_cast<int *>(b->qnext.p),
                                      b->n_cu * b->blocks_per_cu, st, b->mfma, b->mfma_shape);
        if (e != hipSuccess) return dev_err(e, "persistent pair-sum kernel");
    }
    if (time_pairsum) (void)hipEventRecord(b->ev_b, st);
    for (auto &gr : b->groups) {
        const int nb = static_cast<int>(gr.members.size());
        const Workspace ws = carve_workspace(gr.g, b->precision, nb, static_cast<char *>(b->ws.p) + gr.ws_off);
        AmpRef amp = plan_amp(gr.plan);
        amp.scale_b = static_cast<const double *>(b->scales.p) + gr.first;
        amp.S_b = static_cast<const double *const *>(b->sptr.p) + gr.first;
        amp.tab = nullptr;   // per-realization scales and spectra: amplitudes per line
        e = launch_tfft(gr.g, b->precision, 0, nullptr, amp, gr.plan->wtab.p, gr.plan->tw_t.p, nb, ws, st);
        if (e != hipSuccess) return dev_err(e, "t-transform kernel");
        e = launch_xfft(gr.g, b->precision, gr.plan->tw_x.p, nb, ws, nullptr,
                        static_cast<void *const *>(b->outs.p) + gr.first, st);
        if (e != hipSuccess) return dev_err(e, "x-transform kernel");
    }
    return SRM3_OK;
}

srm3_status batch_copy_seeds(srm3_batch_t b, const uint64_t *seeds, hipStream_t st)
{
    if (b->copy_pending) {
        hipError_t e = hipEventSynchronize(b->copy_done);
        if (e != hipSuccess) return dev_err(e, "hipEventSynchronize");
    }
    for (auto &gr : b->groups)
        for (size_t slot = 0; slot < gr.members.size(); ++slot)
            b->seeds_host[gr.first + slot] = seeds ? seeds[gr.members[slot]] : b->req[gr.members[slot]].seed;
    hipError_t e = hipMemcpyAsync(b->seeds.p, b->seeds_host, b->n * sizeof(uint64_t), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return dev_err(e, "hipMemcpyAsync");
    e = hipEventRecord(b->copy_done, st);
    if (e != hipSuccess) return dev_err(e, "hipEventRecord");
    b->copy_pending = true;
    return SRM3_OK;
}

std::string tune_cache_path()
{
    const char *p = std::getenv("SRM3_TUNE_CACHE");
    if (p && *p) return p;
    const char *h = std::getenv("HOME");
    return std::string(h ? h : "/tmp") + "/.cache/srm3_tune.txt";
}

std::string batch_signature(srm3_batch_t b)
{
    std::map<std::string, int> count;
    for (auto &gr : b->groups) {
        std::ostringstream k;
        k << gr.plan->g.nk << 'x' << gr.plan->g.nw << 'w' << gr.plan->g.W;
        count[k.str()] += static_cast<int>(gr.members.size());
    }
    std::ostringstream o;
    o << (b->precision == SRM3_FP64 ? "fp64" : "fp32") << (b->mfma ? ";mfma" : "") << ";cu" << b->n_cu;
    for (auto &kv : count) o << ';' << kv.first << '*' << kv.second;
    return o.str();
}

// Cache lines: signature, rows per wave, workgroups per CU, matrix-core tile
// shape (a missing shape reads as 0).
bool tune_lookup(const std::string &sig, int *R, int *bpc, int *shape)
{
    std::ifstream f(tune_cache_path());
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream ls(line);
        std::string s;
        int r, c, m = 0;
        if (ls >> s >> r >> c && s == sig) {
            if (!(ls >> m) || m < 0 || m >= kMfmaShapes) m = 0;
            *R = r;
            *bpc = c;
            *shape = m;
            found = true;
        }
    }
    return found;
}

void tune_store(const std::string &sig, int R, int bpc, int shape)
{
    const std::string path = tune_cache_path();
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) (void)mkdir(path.substr(0, slash).c_str(), 0755);
    std::ofstream f(path, std::ios::app);
    if (f) f << sig << ' ' << R << ' ' << bpc << ' ' << shape << '\n';
}

}  // namespace

namespace srm3 {
double item_cost(const Geometry &g, int R, int kb, int cg) { return item_cost_impl(g, R, kb, cg); }
double mfma_item_cost(const Geometry &g, int kb, int cg, int precision, int shape)
{
    return mfma_item_cost_impl(g, kb, cg, precision, shape);
}
}  // namespace srm3

extern "C" {

srm3_status srm3_batch_create(const srm3_request *reqs, int32_t n, int32_t flags, void *hip_stream,
                              srm3_batch_t *out)
{
    g_err[0] = 0;
    if (!out) return fail(SRM3_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!reqs || n <= 0) return fail(SRM3_E_INVALID, "no requests");
    const int precision = reqs[0].plan ? reqs[0].plan->precision : -1;
    bool has_mfma = false, has_vector = false;
    for (int i = 0; i < n; ++i) {
        const srm3_request &r = reqs[i];
        if (!r.plan || !r.out_dev) return fail(SRM3_E_INVALID, "request %d: NULL plan or output", i);
        if (r.plan->hashed)
            return fail(SRM3_E_UNSUPPORTED, "request %d: bispectra generated per pair run through srm3_generate", i);
        if (r.plan->algo == SRM3_ALGO_MFMA && !r.plan->gaussian) has_mfma = true;
        if (r.plan->algo == SRM3_ALGO_DIRECT && !r.plan->gaussian) has_vector = true;
        if (has_mfma && has_vector)
            return fail(SRM3_E_UNSUPPORTED,
                        "request %d: a batch's direct-form plans use one pair-sum kernel (all vector or all matrix-core)", i);
        if (r.plan->fixed_spectrum && r.S_dev)
            return fail(SRM3_E_UNSUPPORTED, "request %d: a product bispectrum's plan keeps its own spectrum", i);
        if (r.plan->precision != precision)
            return fail(SRM3_E_INVALID, "request %d: all requests of a batch share one precision", i);
        if (!(r.b2_scale > 0) || !std::isfinite(r.b2_scale))
            return fail(SRM3_E_INVALID, "request %d: b2_scale must be finite and > 0", i);
        if (max_sigma(r.plan->max_sig, r.plan->cap, r.b2_scale) >= 1.0)
            return fail(SRM3_E_PURE_NEGATIVE, "request %d: scaled sum of b^2 reaches 1", i);
    }
    std::unique_ptr<srm3_batch_s> b(new (std::nothrow) srm3_batch_s);
    if (!b) return fail(SRM3_E_NOMEM, "host allocation failed");
    b->precision = precision;
    b->n = n;
    b->flags = flags;
    b->mfma = has_mfma;
    if (has_mfma) b->blocks_per_cu = 3;   // the matrix-core kernel runs 3 waves per SIMD
    b->req.assign(reqs, reqs + n);
    std::map<srm3_plan_t, int> gi;
    for (int i = 0; i < n; ++i) {
        auto it = gi.find(reqs[i].plan);
        if (it == gi.end()) {
            gi[reqs[i].plan] = static_cast<int>(b->groups.size());
            b->groups.push_back({reqs[i].plan, {i}, reqs[i].plan->g, 0, 0});
        } else {
            b->groups[it->second].members.push_back(i);
        }
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        b->n_cu = prop.multiProcessorCount;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    // the largest rows per wave every grid of the persistent launch supports
    int R = precision == SRM3_FP64 ? 8 : 16;
    for (auto &gr : b->groups)
        if (!gr.plan->gaussian && !kfft_family(gr.plan->algo))
            R = std::min(R, rows_for(gr.plan->g.nk, precision, 0));
    srm3_status s = batch_layout(b.get(), R, st);
    if (s) return s;
    for (auto &gr : b->groups) b->pair_terms += gr.plan->pair_terms * gr.members.size();
    // per-request device arrays in group order
    std::vector<double> scales(n);
    std::vector<const double *> sptr(n);
    std::vector<void *> outs(n);
    for (auto &gr : b->groups)
        for (size_t slot = 0; slot < gr.members.size(); ++slot) {
            const srm3_request &r = reqs[gr.members[slot]];
            scales[gr.first + slot] = r.b2_scale;
            sptr[gr.first + slot] = r.S_dev;
            outs[gr.first + slot] = r.out_dev;
        }
    if ((s = upload_bytes(b->scales, scales.data(), n * sizeof(double), st))) return s;
    if ((s = upload_bytes(b->sptr, sptr.data(), n * sizeof(void *), st))) return s;
    if ((s = upload_bytes(b->outs, outs.data(), n * sizeof(void *), st))) return s;
    hipError_t e = b->seeds.alloc(n * sizeof(uint64_t));
    if (e != hipSuccess) return fail(SRM3_E_NOMEM, "hipMalloc: %s", hipGetErrorString(e));
    e = hipHostMalloc(reinterpret_cast<void **>(&b->seeds_host), n * sizeof(uint64_t), hipHostMallocDefault);
    if (e != hipSuccess) return fail(SRM3_E_NOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
    if ((e = hipEventCreateWithFlags(&b->copy_done, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreate(&b->ev_a)) != hipSuccess || (e = hipEventCreate(&b->ev_b)) != hipSuccess ||
        (e = hipEventCreate(&b->run_a)) != hipSuccess || (e = hipEventCreate(&b->run_b)) != hipSuccess)
        return dev_err(e, "hipEventCreate");
    *out = b.release();
    return SRM3_OK;
}

// Time the candidate tile shapes on a stride sample of the batch (requests
// sorted by cost) and keep the fastest; the choice is cached by signature.
// Vector-ALU batches: rows per wave {R_max, R_max / 2} x workgroups per CU
// {1, 2, 3, 4}.  Matrix-core batches: the tile shapes (32 x 32, 32 x 16 and
// 16 x 32 outputs per wave) x workgroups per CU {2, 3, 4, 5} (the smaller
// tiles leave room for more resident waves).
static srm3_status batch_autotune(srm3_batch_t b, hipStream_t st)
{
    const std::string sig = batch_signature(b);
    int R = b->R, bpc = b->blocks_per_cu, shape = b->mfma_shape;
    if (tune_lookup(sig, &R, &bpc, &shape)) {
        b->blocks_per_cu = bpc;
        if (R == b->R && shape == b->mfma_shape) return SRM3_OK;
        b->mfma_shape = shape;
        return batch_layout(b, R, st);
    }
    // Sample every 4th request in cost order (all of them for small batches):
    // about a quarter of the work, with the same mix of grid sizes.  A
    // candidate replaces the default only if it beats it by 3 % on the sample
    // (the sample's queues are shorter than the batch's, so small wins there
    // need not carry over).
    std::vector<int> order(b->n);
    for (int i = 0; i < b->n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->req[x].plan->pair_terms > b->req[y].plan->pair_terms; });
    const int stride = b->n >= 64 ? 4 : 1;
    std::vector<srm3_request> sub;
    for (int i = stride / 2; i < b->n; i += stride) sub.push_back(b->req[order[i]]);
    if (sub.empty()) sub.push_back(b->req[order[0]]);
    srm3_batch_t t = nullptr;
    srm3_status s = srm3_batch_create(sub.data(), static_cast<int32_t>(sub.size()), 0, st, &t);
    if (s) return s;
    const int Rmax = t->R;
    const int defC = t->blocks_per_cu;
    float best = 1e30f, base = 1e30f;
    int bestR = Rmax, bestC = defC, bestM = 0;
    bool first = true;
    auto trial = [&](int r, int m, int c) -> srm3_status {
        if (r != t->R || m != t->mfma_shape) {
            t->mfma_shape = m;
            srm3_status e = batch_layout(t, r, st);
            if (e) return e;
        }
        t->blocks_per_cu = c;
        float ms = 0.f;
        const int reps = first ? 2 : 1;   // the first launch also warms up
        first = false;
        for (int rep = 0; rep < reps; ++rep) {
            srm3_status e = batch_copy_seeds(t, nullptr, st);
            if (!e) e = batch_launch(t, st, true);
            if (e) return e;
            hipError_t he = hipStreamSynchronize(st);
            if (he != hipSuccess) return dev_err(he, "hipStreamSynchronize");
            (void)hipEventElapsedTime(&ms, t->ev_a, t->ev_b);
        }
        if (r == Rmax && m == 0 && c == defC) base = ms;
        if (ms < best) {
            best = ms;
            bestR = r;
            bestC = c;
            bestM = m;
        }
        return SRM3_OK;
    };
    s = trial(Rmax, 0, defC);   // the default first
    if (t->mfma) {
        for (int m = 0; m < kMfmaShapes && !s; ++m)
            for (int c : {2, 3, 4, 5})
                if (!(m == 0 && c == defC) && (s = trial(Rmax, m, c))) break;
    } else {
        for (int r : {Rmax, Rmax / 2}) {
            if (r < 2 || s) continue;
            for (int c : {1, 2, 3, 4})
                if (!(r == Rmax && c == defC) && (s = trial(r, 0, c))) break;
        }
    }
    srm3_batch_destroy(t);
    if (s) return s;
    if (!(best < 0.97f * base)) {
        bestR = Rmax;
        bestC = defC;
        bestM = 0;
    }
    b->mfma_shape = bestM;
    if ((bestR != b->R || b->mfma) && (s = batch_layout(b, bestR, st))) return s;
    b->blocks_per_cu = bestC;
    tune_store(sig, bestR, bestC, bestM);
    return SRM3_OK;
}

srm3_status srm3_batch_run(srm3_batch_t b, const uint64_t *seeds, void *hip_stream)
{
    g_err[0] = 0;
    if (!b) return fail(SRM3_E_INVALID, "batch is NULL");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    srm3_status s;
    if ((b->flags & SRM3_BATCH_AUTOTUNE) && !b->tuned) {
        if ((s = batch_autotune(b, st))) return s;
        b->tuned = true;
    }
    if ((s = batch_copy_seeds(b, seeds, st))) return s;
    b->ran = true;
    if (b->flags & SRM3_BATCH_GRAPH) {
        if (!b->exec) {
            hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return dev_err(e, "hipStreamCreate");
            e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return dev_err(e, "hipStreamBeginCapture");
            s = batch_launch(b, b->cap_stream, false);
            hipGraph_t graph = nullptr;
            hipError_t e2 = hipStreamEndCapture(b->cap_stream, &graph);
            if (s) return s;
            if (e2 != hipSuccess) return dev_err(e2, "hipStreamEndCapture");
            e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                b->exec = nullptr;
                return dev_err(e, "hipGraphInstantiate");
            }
        }
        (void)hipEventRecord(b->run_a, st);
        hipError_t e = hipGraphLaunch(b->exec, st);
        if (e != hipSuccess) return dev_err(e, "hipGraphLaunch");
        (void)hipEventRecord(b->run_b, st);
        b->ps_timed = false;
        return SRM3_OK;
    }
    (void)hipEventRecord(b->run_a, st);
    if ((s = batch_launch(b, st, true))) return s;
    (void)hipEventRecord(b->run_b, st);
    b->ps_timed = true;
    return SRM3_OK;
}

srm3_status srm3_batch_info(srm3_batch_t b, srm3_batch_stats *out)
{
    if (!b || !out) return fail(SRM3_E_INVALID, "bad argument");
    out->pair_terms = b->pair_terms;
    out->rows_per_wave = b->R;
    out->blocks_per_cu = b->blocks_per_cu;
    out->mfma_shape = b->mfma ? b->mfma_shape : -1;
    out->work_items = b->n_items;
    out->groups = static_cast<int32_t>(b->groups.size());
    out->run_ms = -1.0;
    out->pairsum_ms = -1.0;
    float ms = 0.f;
    if (b->ran) {
        hipError_t e = hipEventSynchronize(b->run_b);
        if (e != hipSuccess) return dev_err(e, "hipEventSynchronize");
        if (hipEventElapsedTime(&ms, b->run_a, b->run_b) == hipSuccess) out->run_ms = ms;
        if (b->ps_timed && hipEventElapsedTime(&ms, b->ev_a, b->ev_b) == hipSuccess) out->pairsum_ms = ms;
    }
    return SRM3_OK;
}

void srm3_batch_destroy(srm3_batch_t b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->seeds_host) (void)hipHostFree(b->seeds_host);
    if (b->copy_done) (void)hipEventDestroy(b->copy_done);
    for (hipEvent_t ev : {b->ev_a, b->ev_b, b->run_a, b->run_b})
        if (ev) (void)hipEventDestroy(ev);
    delete b;
}

srm3_status srm3_generate_uneven(const srm3_request *reqs, int32_t n, void *hip_stream)
{
    srm3_batch_t b = nullptr;
    srm3_status s = srm3_batch_create(reqs, n, 0, hip_stream, &b);
    if (s) return s;
    s = srm3_batch_run(b, nullptr, hip_stream);
    if (!s) {
        hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(hip_stream));
        if (e != hipSuccess) s = dev_err(e, "hipStreamSynchronize");
    }
    srm3_batch_destroy(b);
    return s;
}

}  // extern "C"
