// Plan-time host code for kappa-dependent bicoherence (FP64, no device work).
//
// Line factors.  A pair {i, j} -> k may carry per-line factors,
//     b2_raw(i, j -> k) = c_k^2 r_i^2 r_j^2 b2(i_w, j_w),
// so its biamplitude is c_k r_i r_j sqrt(b2) e^{i beta}: r scales the phase
// factor of every line before the pair sum, c scales a line's pair sum.  The
// per-line raw sums Q_k = sum_{P(k)} r_i^2 r_j^2 b2(i_w, j_w) are a weighted
// 2-D autoconvolution of y = r^2: through a 2-D FFT when b2 is separable,
// through an FFT along kappa and a direct frequency sum otherwise.
//
// The wind bispectrum (Section 5, Eq. bispectrum, scaled by alpha, beta = 0)
// through the partial bicoherence of Section 4.1 factorises exactly this way:
//     b_p = |B| sqrt(dk dw) / sqrt(S_p,i S_p,j S_k)
//         = [alpha 2 / (3 sqrt 3) / sqrt(|k_w| k_kappa)] * sqrt(S_i / S_p,i) * sqrt(S_j / S_p,j),
// (|omega_i + omega_j| under the root; zero where B is singular, k_kappa = 0 or
// k_w = 0, and on lines with S = 0).  r_i = 1 / sqrt(1 - Sigma_i) depends on
// the partner lines' Sigma, so Sigma solves a fixed point; it is found by
// sweeps Sigma <- min(cap, c^2 Q(r(Sigma))) from Sigma = 0, which increase
// monotonically to the least solution.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "srm3_internal.hpp"

namespace srm3 {

using cd = std::complex<double>;

// In-place radix-2 FFT of length n (power of two), sign -1 forward, +1 inverse
// (unnormalised), strided access; tw holds e^{-2 pi i m / n}, m < n / 2.
static void fft1(cd *a, int n, long stride, int sign, const std::vector<cd> &tw)
{
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i * stride], a[j * stride]);
    }
    for (int len = 2; len <= n; len <<= 1) {
        const int step = n / len;
        for (int i = 0; i < n; i += len)
            for (int k = 0; k < len / 2; ++k) {
                const cd w = sign < 0 ? tw[static_cast<size_t>(k) * step] : std::conj(tw[static_cast<size_t>(k) * step]);
                const cd u = a[(i + k) * stride], v = a[(i + k + len / 2) * stride] * w;
                a[(i + k) * stride] = u + v;
                a[(i + k + len / 2) * stride] = u - v;
            }
    }
}

static std::vector<cd> fft_table(int n)
{
    std::vector<cd> tw(std::max(1, n / 2));
    for (int m = 0; m < n / 2; ++m) tw[m] = std::polar(1.0, -2.0 * M_PI * m / n);
    return tw;
}

static int pow2_at_least(int n)
{
    int p = 1;
    while (p < n) p *= 2;
    return p;
}

void line_pair_sums(int nk, int nw, int W, const double *r, int kind, const double *g2, const double *b2,
                    std::vector<double> &Q)
{
    const int nc = 2 * nw - 1, ncw = 2 * W - 1;
    Q.assign(static_cast<size_t>(nk) * nc, 0.0);
    auto y_at = [&](int kk, int iw) {   // r^2 of line (kk, iw)
        const double v = r ? r[static_cast<size_t>(kk) * nc + iw + nw - 1] : 1.0;
        return v * v;
    };
    const int Mk = pow2_at_least(2 * nk - 1);
    const int Mw = pow2_at_least(2 * ncw - 1);
    std::vector<double> self(static_cast<size_t>(nk) * nc, 0.0);   // self-pair terms
    for (int kk = 0; kk < nk; kk += 2)
        for (int kw = -(nw - 1); kw <= nw - 1; ++kw) {
            if (kw % 2 != 0) continue;
            const int h = kw / 2;
            if (h <= -W || h >= W) continue;
            const double wgt = kind == SRM3_BISPEC_SEPARABLE ? g2[h + W - 1] * g2[h + W - 1]
                                                             : b2[static_cast<size_t>(h + W - 1) * ncw + h + W - 1];
            const double y = y_at(kk / 2, h);
            self[static_cast<size_t>(kk) * nc + kw + nw - 1] = wgt * y * y;
        }
    const std::vector<cd> twk = fft_table(Mk), tww = fft_table(Mw);
    if (kind == SRM3_BISPEC_SEPARABLE) {
        // full 2-D autoconvolution of y g2 over kappa in [0, nk), |i_w| < W
        std::vector<cd> A(static_cast<size_t>(Mk) * Mw, cd(0.0, 0.0));
        for (int kk = 0; kk < nk; ++kk)
            for (int iw = -(W - 1); iw <= W - 1; ++iw)
                A[static_cast<size_t>(kk) * Mw + iw + W - 1] = cd(y_at(kk, iw) * g2[iw + W - 1], 0.0);
        for (int kk = 0; kk < nk; ++kk) fft1(A.data() + static_cast<size_t>(kk) * Mw, Mw, 1, -1, tww);
        for (int c = 0; c < Mw; ++c) fft1(A.data() + c, Mk, Mw, -1, twk);
        for (auto &v : A) v *= v;
        for (int c = 0; c < Mw; ++c) fft1(A.data() + c, Mk, Mw, +1, twk);
        for (int kk = 0; kk < nk; ++kk) fft1(A.data() + static_cast<size_t>(kk) * Mw, Mw, 1, +1, tww);
        const double inv = 1.0 / (static_cast<double>(Mk) * Mw);
        for (int kk = 0; kk < nk; ++kk)
            for (int kw = -(nw - 1); kw <= nw - 1; ++kw) {
                if (kw < -(2 * W - 2) || kw > 2 * W - 2) continue;
                const double ordered = A[static_cast<size_t>(kk) * Mw + kw + 2 * W - 2].real() * inv;
                const size_t l = static_cast<size_t>(kk) * nc + kw + nw - 1;
                Q[l] = std::max(0.0, 0.5 * (ordered + self[l]));
            }
        return;
    }
    // dense b2: transform along kappa, weighted frequency sum per kappa frequency
    std::vector<cd> Z(static_cast<size_t>(Mk) * ncw, cd(0.0, 0.0));
    for (int kk = 0; kk < nk; ++kk)
        for (int iw = -(W - 1); iw <= W - 1; ++iw) Z[static_cast<size_t>(kk) * ncw + iw + W - 1] = cd(y_at(kk, iw), 0.0);
    for (int c = 0; c < ncw; ++c) fft1(Z.data() + c, Mk, ncw, -1, twk);
    const int nout = 4 * W - 3;
    std::vector<cd> O(static_cast<size_t>(Mk) * nout, cd(0.0, 0.0));
    for (int q = 0; q < Mk; ++q)
        for (int kw = -(2 * W - 2); kw <= 2 * W - 2; ++kw) {
            cd acc(0.0, 0.0);
            for (int iw = std::max(-(W - 1), kw - (W - 1)); iw <= std::min(W - 1, kw + W - 1); ++iw) {
                const int jw = kw - iw;
                acc += b2[static_cast<size_t>(iw + W - 1) * ncw + jw + W - 1] *
                       Z[static_cast<size_t>(q) * ncw + iw + W - 1] * Z[static_cast<size_t>(q) * ncw + jw + W - 1];
            }
            O[static_cast<size_t>(q) * nout + kw + 2 * W - 2] = acc;
        }
    for (int c = 0; c < nout; ++c) fft1(O.data() + c, Mk, nout, +1, twk);
    for (int kk = 0; kk < nk; ++kk)
        for (int kw = -(nw - 1); kw <= nw - 1; ++kw) {
            if (kw < -(2 * W - 2) || kw > 2 * W - 2) continue;
            const double ordered = O[static_cast<size_t>(kk) * nout + kw + 2 * W - 2].real() / Mk;
            const size_t l = static_cast<size_t>(kk) * nc + kw + nw - 1;
            Q[l] = std::max(0.0, 0.5 * (ordered + self[l]));
        }
}

srm3_status wind_factors(int nk, int nw, int W, const double *S, double alpha, double cap, std::vector<double> &c,
                         std::vector<double> &r, int *sweeps, double *max_sig)
{
    const int nc = 2 * nw - 1;
    const size_t nl = static_cast<size_t>(nk) * nc;
    c.assign(nl, 0.0);
    r.assign(nl, 0.0);
    const double k0 = alpha * 2.0 / (3.0 * std::sqrt(3.0));
    for (int kk = 1; kk < nk; ++kk)
        for (int kw = -(nw - 1); kw <= nw - 1; ++kw)
            if (kw != 0) c[static_cast<size_t>(kk) * nc + kw + nw - 1] = k0 / std::sqrt(std::fabs(kw) * kk);
    std::vector<double> sigma(nl, 0.0), Q;
    const std::vector<double> ones(2 * W - 1, 1.0);
    int it = 0;
    double ms = 0.0, last_diff = 1.0;
    for (it = 1; it <= 1000; ++it) {
        for (size_t l = 0; l < nl; ++l) r[l] = S[l] > 0.0 ? 1.0 / std::sqrt(1.0 - sigma[l]) : 0.0;
        line_pair_sums(nk, nw, W, r.data(), SRM3_BISPEC_SEPARABLE, ones.data(), nullptr, Q);
        double diff = 0.0;
        ms = 0.0;
        for (size_t l = 0; l < nl; ++l) {
            double s = c[l] * c[l] * Q[l];
            if (S[l] <= 0.0) s = 0.0;
            if (cap > 0.0) s = std::min(s, cap);
            if (!(s < 1.0))
                return fail(SRM3_E_PURE_NEGATIVE,
                            "wind bispectrum (alpha %.4g): the partial-bicoherence recursion has no admissible "
                            "pure spectrum (Sigma reaches 1); give a cap < 1 or a smaller alpha", alpha);
            diff = std::max(diff, std::fabs(s - sigma[l]));
            sigma[l] = s;
            ms = std::max(ms, s);
        }
        // converged, or settled at the rounding floor of the FFT sums
        if (diff <= 1e-14 || (diff <= 1e-12 && diff >= last_diff)) break;
        last_diff = diff;
    }
    if (it > 1000) return fail(SRM3_E_UNSUPPORTED, "wind bispectrum: the recursion did not converge");
    for (size_t l = 0; l < nl; ++l) r[l] = S[l] > 0.0 ? 1.0 / std::sqrt(1.0 - sigma[l]) : 0.0;
    if (sweeps) *sweeps = it;
    if (max_sig) *max_sig = ms;
    return SRM3_OK;
}

}  // namespace srm3

namespace srm3 {

// Prescribed product bispectrum B(i, j) = F_k G_i G_j H(i_w, j_w): complex line
// factors c_k = F_k sqrt(dk dw / S_k), rho_i = G_i / sqrt(S_i (1 - Sigma_i)),
// Sigma_k = min(cap, |c_k|^2 sum_{P(k)} |rho_i|^2 |rho_j|^2 |H|^2) by the same
// monotone sweeps as the wind bispectrum.  c, rho: interleaved complex.
srm3_status product_factors(int nk, int nw, int W, const double *S, const double *F, const double *G,
                            const double *H, double dk, double dw, double cap, std::vector<double> &c,
                            std::vector<double> &rho, int *sweeps, double *max_sig, std::vector<double> *sigma_out)
{
    const int nc = 2 * nw - 1, ncw = 2 * W - 1;
    const size_t nl = static_cast<size_t>(nk) * nc;
    c.assign(2 * nl, 0.0);
    rho.assign(2 * nl, 0.0);
    for (size_t l = 0; l < nl; ++l)
        if (S[l] > 0.0) {
            const double f = std::sqrt(dk * dw / S[l]);
            c[2 * l] = F[2 * l] * f;
            c[2 * l + 1] = F[2 * l + 1] * f;
        }
    std::vector<double> h2;
    const std::vector<double> ones(ncw, 1.0);
    if (H) {
        h2.resize(static_cast<size_t>(ncw) * ncw);
        for (size_t e = 0; e < h2.size(); ++e) h2[e] = H[2 * e] * H[2 * e] + H[2 * e + 1] * H[2 * e + 1];
    }
    std::vector<double> sigma(nl, 0.0), mag(nl, 0.0), Q;
    int it = 0;
    double ms = 0.0, last_diff = 1.0;
    auto set_rho = [&]() {
        for (size_t l = 0; l < nl; ++l) {
            if (S[l] > 0.0) {
                const double f = 1.0 / std::sqrt(S[l] * (1.0 - sigma[l]));
                rho[2 * l] = G[2 * l] * f;
                rho[2 * l + 1] = G[2 * l + 1] * f;
            } else {
                rho[2 * l] = rho[2 * l + 1] = 0.0;
            }
            mag[l] = std::hypot(rho[2 * l], rho[2 * l + 1]);
        }
    };
    for (it = 1; it <= 1000; ++it) {
        set_rho();
        if (H)
            line_pair_sums(nk, nw, W, mag.data(), SRM3_BISPEC_DENSE, nullptr, h2.data(), Q);
        else
            line_pair_sums(nk, nw, W, mag.data(), SRM3_BISPEC_SEPARABLE, ones.data(), nullptr, Q);
        double diff = 0.0;
        ms = 0.0;
        for (size_t l = 0; l < nl; ++l) {
            double s = (c[2 * l] * c[2 * l] + c[2 * l + 1] * c[2 * l + 1]) * Q[l];
            if (S[l] <= 0.0) s = 0.0;
            if (cap > 0.0) s = std::min(s, cap);
            if (!(s < 1.0))
                return fail(SRM3_E_PURE_NEGATIVE,
                            "product bispectrum: the partial-bicoherence recursion has no admissible pure spectrum "
                            "(Sigma reaches 1); give a cap < 1 or a smaller bispectrum");
            diff = std::max(diff, std::fabs(s - sigma[l]));
            sigma[l] = s;
            ms = std::max(ms, s);
        }
        // converged, or settled at the rounding floor of the FFT sums
        if (diff <= 1e-14 || (diff <= 1e-12 && diff >= last_diff)) break;
        last_diff = diff;
    }
    if (it > 1000) return fail(SRM3_E_UNSUPPORTED, "product bispectrum: the recursion did not converge");
    set_rho();
    if (sweeps) *sweeps = it;
    if (max_sig) *max_sig = ms;
    if (sigma_out) *sigma_out = sigma;
    return SRM3_OK;
}

}  // namespace srm3
