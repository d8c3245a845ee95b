// C-ABI of the srm3 library: plan construction (host, FP64), generation
// launch sequences, error reporting and event-based kernel timing.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "srm3_internal.hpp"

using namespace srm3;

namespace {

thread_local char g_err[512] = "";

srm3_status fail(srm3_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

struct DevBuf {
    void *p = nullptr;
    size_t n = 0;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    hipError_t alloc(size_t bytes)
    {
        release();
        if (bytes == 0) bytes = 256;
        hipError_t e = hipMalloc(&p, bytes);
        if (e == hipSuccess) n = bytes;
        else p = nullptr;
        return e;
    }
};

}  // namespace

struct srm3_plan_s {
    Geometry g{};
    int precision = SRM3_FP64;
    double dk = 0, dw = 0;
    double pair_terms = 0;
    int device = 0;
    DevBuf wtab, amp_pure, amp_pair, tw_t, tw_x, ws;
    int ws_batch = 0;
    // profiling
    bool prof = false;
    struct Rec {
        int kernel;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
};

namespace {

srm3_status dev_err(hipError_t e, const char *what)
{
    return fail(SRM3_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

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
    std::vector<unsigned char> bytes =
        precision == SRM3_FP64 ? to_bytes<double>(v) : to_bytes<float>(v);
    hipError_t e = buf.alloc(bytes.size());
    if (e != hipSuccess) return fail(SRM3_E_NOMEM, "hipMalloc(%zu): %s", bytes.size(), hipGetErrorString(e));
    e = hipMemcpyAsync(buf.p, bytes.data(), bytes.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return dev_err(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return dev_err(e, "hipStreamSynchronize");
    return SRM3_OK;
}

// exp(+2 pi i n / N), n < N, interleaved
std::vector<double> twiddles(int N)
{
    std::vector<double> v(2 * static_cast<size_t>(N));
    for (int n = 0; n < N; ++n) {
        // reduce to the first octant-free form through long double for accuracy
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

srm3_status ensure_workspace(srm3_plan_t p, int batch)
{
    if (batch <= p->ws_batch) return SRM3_OK;
    const size_t bytes = workspace_bytes(p->g, p->precision, batch);
    hipError_t e = p->ws.alloc(bytes);
    if (e != hipSuccess) {
        p->ws_batch = 0;
        return fail(SRM3_E_NOMEM, "workspace hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    p->ws_batch = batch;
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

srm3_status run_front(srm3_plan_t p, const uint64_t *seeds, int32_t batch, const Workspace &ws,
                      hipStream_t st)
{
    srm3_status s;
    if ((s = event_pair(p, 0, st, true))) return s;
    hipError_t e = launch_phases(p->g, p->precision, seeds, batch, ws, st);
    if (e != hipSuccess) return dev_err(e, "phase kernel");
    if ((s = event_pair(p, 0, st, false))) return s;
    if ((s = event_pair(p, 1, st, true))) return s;
    e = launch_pairsum(p->g, p->precision, p->wtab.p, batch, ws, st);
    if (e != hipSuccess) return dev_err(e, "pair-sum kernel");
    if ((s = event_pair(p, 1, st, false))) return s;
    return SRM3_OK;
}

srm3_status run_back(srm3_plan_t p, int mode, const void *cin, int32_t batch, const Workspace &ws,
                     void *out, hipStream_t st)
{
    srm3_status s;
    if ((s = event_pair(p, 2, st, true))) return s;
    hipError_t e = launch_tfft(p->g, p->precision, mode, cin, p->amp_pure.p, p->amp_pair.p, p->wtab.p,
                               p->tw_t.p, batch, ws, st);
    if (e != hipSuccess) return dev_err(e, "t-transform kernel");
    if ((s = event_pair(p, 2, st, false))) return s;
    if ((s = event_pair(p, 3, st, true))) return s;
    e = launch_xfft(p->g, p->precision, p->tw_x.p, batch, ws, out, st);
    if (e != hipSuccess) return dev_err(e, "x-transform kernel");
    if ((s = event_pair(p, 3, st, false))) return s;
    return SRM3_OK;
}

}  // namespace

extern "C" {

const char *srm3_last_error(void) { return g_err; }

srm3_status srm3_plan(const srm3_grid *grid, const srm3_spectrum *spectrum,
                      const srm3_bispectrum *bispectrum, int32_t precision, void *hip_stream,
                      srm3_plan_t *out_plan)
{
    g_err[0] = 0;
    if (!out_plan) return fail(SRM3_E_INVALID, "out_plan is NULL");
    *out_plan = nullptr;
    if (!grid || !spectrum || !spectrum->S) return fail(SRM3_E_INVALID, "grid/spectrum is NULL");
    if (precision != SRM3_FP64 && precision != SRM3_FP32)
        return fail(SRM3_E_INVALID, "precision %d", precision);
    const int nk = grid->n_kappa, nw = grid->n_omega, nx = grid->n_x, nt = grid->n_t;
    if (nk < 1 || nw < 1) return fail(SRM3_E_INVALID, "n_kappa=%d n_omega=%d must be >= 1", nk, nw);
    if (!(grid->d_kappa > 0) || !(grid->d_omega > 0) || !std::isfinite(grid->d_kappa) ||
        !std::isfinite(grid->d_omega))
        return fail(SRM3_E_INVALID, "d_kappa/d_omega must be finite and > 0");
    if (!is_pow2(nx) || !is_pow2(nt))
        return fail(SRM3_E_UNSUPPORTED, "n_x=%d n_t=%d must be powers of two", nx, nt);
    const int nc = 2 * nw - 1;
    if (nx < nk || nt < nc)
        return fail(SRM3_E_INVALID, "field %dx%d smaller than the line grid (need n_x >= %d, n_t >= %d)",
                    nx, nt, nk, nc);
    const int tmax = precision == SRM3_FP64 ? 8192 : 16384;   // one transform fits 128 KB of LDS
    if (nt > tmax || nx > tmax)
        return fail(SRM3_E_UNSUPPORTED, "n_t=%d / n_x=%d above this build's limit %d", nt, nx, tmax);
    if (static_cast<long long>(nk) * nc > (1LL << 30))
        return fail(SRM3_E_UNSUPPORTED, "line grid too large");

    // ---- bicoherence description ----
    srm3_bispectrum none{};
    none.kind = SRM3_BISPEC_NONE;
    none.support_w = 1;
    none.beta_mode = SRM3_BETA_ZERO;
    const srm3_bispectrum &bs = bispectrum ? *bispectrum : none;
    const int W = bs.kind == SRM3_BISPEC_NONE ? (bs.support_w >= 1 ? bs.support_w : 1) : bs.support_w;
    if (W < 1 || W > nw) return fail(SRM3_E_INVALID, "support_w=%d must be in [1, n_omega=%d]", W, nw);
    const int ncw = 2 * W - 1;
    if (bs.kind != SRM3_BISPEC_NONE && bs.kind != SRM3_BISPEC_SEPARABLE && bs.kind != SRM3_BISPEC_DENSE)
        return fail(SRM3_E_INVALID, "bispectrum kind %d", bs.kind);
    if (bs.kind == SRM3_BISPEC_SEPARABLE && !bs.g2) return fail(SRM3_E_INVALID, "g2 is NULL");
    if (bs.kind == SRM3_BISPEC_DENSE && !bs.b2) return fail(SRM3_E_INVALID, "b2 is NULL");
    if (bs.beta_mode != SRM3_BETA_SEEDED && bs.beta_mode != SRM3_BETA_ZERO && bs.beta_mode != SRM3_BETA_TABLE)
        return fail(SRM3_E_INVALID, "beta_mode %d", bs.beta_mode);
    if (bs.kind != SRM3_BISPEC_NONE && bs.beta_mode == SRM3_BETA_TABLE && !bs.beta)
        return fail(SRM3_E_INVALID, "beta table is NULL");
    if (!std::isfinite(bs.cap)) return fail(SRM3_E_INVALID, "cap is not finite");

    // raw squared bicoherence table over the support
    std::vector<double> b2(static_cast<size_t>(ncw) * ncw, 0.0);
    if (bs.kind == SRM3_BISPEC_SEPARABLE) {
        for (int i = 0; i < ncw; ++i)
            if (!(bs.g2[i] >= 0) || !std::isfinite(bs.g2[i]))
                return fail(SRM3_E_INVALID, "g2[%d] must be finite and >= 0", i);
        for (int i = 0; i < ncw; ++i)
            for (int j = 0; j < ncw; ++j) b2[static_cast<size_t>(i) * ncw + j] = bs.g2[i] * bs.g2[j];
    } else if (bs.kind == SRM3_BISPEC_DENSE) {
        for (int i = 0; i < ncw; ++i)
            for (int j = 0; j < ncw; ++j) {
                const double v = bs.b2[static_cast<size_t>(i) * ncw + j];
                if (!(v >= 0) || !std::isfinite(v))
                    return fail(SRM3_E_INVALID, "b2[%d][%d] must be finite and >= 0", i, j);
                if (v != bs.b2[static_cast<size_t>(j) * ncw + i])
                    return fail(SRM3_E_INVALID, "b2 is not symmetric at [%d][%d]", i, j);
                b2[static_cast<size_t>(i) * ncw + j] = v;
            }
    }
    // biphase (fixed point)
    std::vector<uint32_t> beta(static_cast<size_t>(ncw) * ncw, 0u);
    if (bs.kind != SRM3_BISPEC_NONE) {
        if (bs.beta_mode == SRM3_BETA_SEEDED) {
            for (int i = 0; i < ncw; ++i)
                for (int j = 0; j < ncw; ++j) {
                    const int iw = i - (W - 1), jw = j - (W - 1);
                    const int hi = iw >= jw ? iw : jw, lo = iw >= jw ? jw : iw;
                    beta[static_cast<size_t>(i) * ncw + j] =
                        philox_word0(static_cast<uint32_t>(hi), static_cast<uint32_t>(lo), 1u, 0u, bs.beta_seed);
                }
        } else if (bs.beta_mode == SRM3_BETA_TABLE) {
            for (int i = 0; i < ncw; ++i)
                for (int j = 0; j < ncw; ++j) {
                    const uint32_t v = bs.beta[static_cast<size_t>(i) * ncw + j];
                    if (v != bs.beta[static_cast<size_t>(j) * ncw + i])
                        return fail(SRM3_E_INVALID, "beta table is not symmetric at [%d][%d]", i, j);
                    beta[static_cast<size_t>(i) * ncw + j] = v;
                }
        }
    }

    // ---- spectrum ----
    const double *S = spectrum->S;
    const size_t nlines = static_cast<size_t>(nk) * nc;
    for (size_t i = 0; i < nlines; ++i)
        if (!(S[i] >= 0) || !std::isfinite(S[i]))
            return fail(SRM3_E_INVALID, "S[%zu] must be finite and >= 0", i);

    // ---- per-line sums (ordered frequency splits + self pair), FP64 ----
    // D[kw] = sum_{iw} b2(iw, kw - iw) over the support; an output line with
    // k_kappa = kk has (kk + 1) kappa splits, so the ordered sum is (kk+1) D[kw]
    // and the unordered sum half of it plus half the self pair.
    std::vector<double> D(nc, 0.0);
    for (int kw = -(nw - 1); kw <= nw - 1; ++kw) {
        double s = 0.0;
        for (int iw = -(W - 1); iw <= W - 1; ++iw) {
            const int jw = kw - iw;
            if (jw <= -W || jw >= W) continue;
            s += b2[static_cast<size_t>(iw + W - 1) * ncw + (jw + W - 1)];
        }
        D[kw + nw - 1] = s;
    }
    std::vector<double> ap(nlines), ac(nlines);
    double pair_terms = 0.0;
    const double dkdw = grid->d_kappa * grid->d_omega;
    for (int kk = 0; kk < nk; ++kk)
        for (int c = 0; c < nc; ++c) {
            const int kw = c - (nw - 1);
            double diag = 0.0;
            long nsplit = 0;
            for (int iw = -(W - 1); iw <= W - 1; ++iw)
                if (kw - iw > -W && kw - iw < W) ++nsplit;
            int self = 0;
            if ((kk % 2) == 0 && (kw % 2) == 0 && kw / 2 > -W && kw / 2 < W) {
                diag = b2[static_cast<size_t>(kw / 2 + W - 1) * ncw + (kw / 2 + W - 1)];
                self = 1;
            }
            pair_terms += 0.5 * (static_cast<double>(kk + 1) * nsplit + self);
            const double sraw = 0.5 * ((kk + 1) * D[c] + diag);
            double rho = 1.0;
            if (bs.cap > 0 && sraw > bs.cap) rho = bs.cap / sraw;
            const double sigma = rho * sraw;
            if (sigma >= 1.0)
                return fail(SRM3_E_PURE_NEGATIVE,
                            "line (%d, %d): sum of b^2 = %.6g >= 1, pure spectrum not positive", kk, kw, sigma);
            const size_t li = static_cast<size_t>(kk) * nc + c;
            ap[li] = 2.0 * std::sqrt(S[li] * dkdw * (1.0 - sigma));
            ac[li] = 2.0 * std::sqrt(S[li] * dkdw * rho);
        }

    // complex weight table W = sqrt(b2) e^{i beta}
    std::vector<double> wt(2 * static_cast<size_t>(ncw) * ncw);
    for (size_t e = 0; e < static_cast<size_t>(ncw) * ncw; ++e) {
        const long double ang = 2.0L * 3.14159265358979323846264338327950288L * beta[e] / 4294967296.0L;
        const double m = std::sqrt(b2[e]);
        wt[2 * e] = m * static_cast<double>(cosl(ang));
        wt[2 * e + 1] = m * static_cast<double>(sinl(ang));
    }

    std::unique_ptr<srm3_plan_s> p(new (std::nothrow) srm3_plan_s);
    if (!p) return fail(SRM3_E_NOMEM, "host allocation failed");
    p->precision = precision;
    p->dk = grid->d_kappa;
    p->dw = grid->d_omega;
    p->pair_terms = pair_terms;
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

    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    srm3_status s;
    if ((s = upload(p->wtab, wt, precision, st))) return s;
    if ((s = upload(p->amp_pure, ap, precision, st))) return s;
    if ((s = upload(p->amp_pair, ac, precision, st))) return s;
    if ((s = upload(p->tw_t, twiddles(nt), precision, st))) return s;
    if ((s = upload(p->tw_x, twiddles(nx), precision, st))) return s;
    *out_plan = p.release();
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
    return SRM3_OK;
}

srm3_status srm3_pair_terms(srm3_plan_t plan, double *terms)
{
    if (!plan || !terms) return fail(SRM3_E_INVALID, "bad argument");
    *terms = plan->pair_terms;
    return SRM3_OK;
}

srm3_status srm3_generate(srm3_plan_t plan, const uint64_t *seeds, int32_t batch, void *out_dev,
                          void *hip_stream)
{
    g_err[0] = 0;
    srm3_status s = check_batch(plan, seeds, batch, out_dev);
    if (s) return s;
    if (batch == 0) return SRM3_OK;
    if ((s = ensure_workspace(plan, batch))) return s;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const Workspace ws = carve_workspace(plan->g, plan->precision, batch, plan->ws.p);
    if ((s = run_front(plan, seeds, batch, ws, st))) return s;
    return run_back(plan, 0, nullptr, batch, ws, out_dev, st);
}

srm3_status srm3_coefficients(srm3_plan_t plan, const uint64_t *seeds, int32_t batch, void *C_dev,
                              void *hip_stream)
{
    g_err[0] = 0;
    srm3_status s = check_batch(plan, seeds, batch, C_dev);
    if (s) return s;
    if (batch == 0) return SRM3_OK;
    if ((s = ensure_workspace(plan, batch))) return s;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const Workspace ws = carve_workspace(plan->g, plan->precision, batch, plan->ws.p);
    if ((s = run_front(plan, seeds, batch, ws, st))) return s;
    hipError_t e = launch_assemble(plan->g, plan->precision, plan->amp_pure.p, plan->amp_pair.p,
                                   plan->wtab.p, batch, ws, C_dev, st);
    if (e != hipSuccess) return dev_err(e, "assemble kernel");
    return SRM3_OK;
}

srm3_status srm3_transform(srm3_plan_t plan, const void *C_dev, int32_t batch, void *out_dev,
                           void *hip_stream)
{
    g_err[0] = 0;
    srm3_status s = check_batch(plan, C_dev, batch, out_dev);
    if (s) return s;
    if (batch == 0) return SRM3_OK;
    if ((s = ensure_workspace(plan, batch))) return s;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
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
