"""Pins of the oracle's kappa-dependent bicoherence (CPU only).

* Line factors: b2_raw(i, j -> k) = c_k^2 r_i^2 r_j^2 b2(i_w, j_w).  Pinned by
  the pair sum written out in Python and, for a separable b2, by a 2-D linear
  autoconvolution through numpy's FFT.
* The wind bispectrum of Section 5 (Eq. bispectrum) through the partial
  bicoherence of Section 4.1, whose pure spectrum S_p solves a fixed point:
  - a pure-Python solve in another order (kappa rows ascending, each row
    iterated to its own fixed point) reaches the same S_p;
  - the bicoherence factorises into per-line factors, c_k = alpha 2/(3 sqrt 3)
    sqrt(dk dw / (|w_k| kappa_k)) and r_i = sqrt(S_i / S_p,i) (the form the
    generator uses), and the table form with those factors gives the same
    coefficients;
  - Monte Carlo: with the recursion, the third moment of the field is the
    discrete integral of the prescribed bispectrum, 6 sum_k sum_{P(k)} c_p |B_p|
    (dk dw)^2, whatever S_p is (the recursion exists to make that so); with S
    in place of S_p it would differ by many standard errors.
"""
import math

import numpy as np
import pytest

import srm3_inputs as inp

TWO_PI = 2.0 * math.pi


def _pairs(nk, nw, W, kk, kw):
    for ik in range(kk + 1):
        jk = kk - ik
        for iw in range(-(W - 1), W):
            jw = kw - iw
            if abs(jw) >= W:
                continue
            if ik > jk or (ik == jk and iw >= jw):
                yield ik, iw, jk, jw


def test_line_factors_brute_force(oracle_mod):
    nk, nw, W = 4, 5, 4
    S = inp.random_spectrum(nk, nw, seed=21)
    b2 = inp.random_b2_dense(W, 22, scale=0.2)
    beta = inp.random_beta_table(W, 23)
    rng = np.random.default_rng(24)
    lc = rng.uniform(0.2, 1.5, size=S.shape)
    lr = rng.uniform(0.5, 1.2, size=S.shape)
    P = oracle_mod.Problem(nk, nw, W, 0.3, 0.2, S, b2, beta, 0.6, line_c=lc, line_r=lr)
    U = oracle_mod.phases(nk, nw, 77)
    C = P.coefficients(U=U)
    phi = TWO_PI * U.astype(np.float64) / 2.0 ** 32
    c0 = nw - 1
    for kk in range(nk):
        for kw in range(-(nw - 1), nw):
            prs = list(_pairs(nk, nw, W, kk, kw))
            raw = [lc[kk, kw + c0] ** 2 * lr[ik, iw + c0] ** 2 * lr[jk, jw + c0] ** 2
                   * b2[iw + W - 1, jw + W - 1] for ik, iw, jk, jw in prs]
            tot = sum(raw)
            rho = 0.6 / tot if tot > 0.6 else 1.0
            acc = math.sqrt(1.0 - rho * tot) * np.exp(1j * phi[kk, kw + c0])
            for (ik, iw, jk, jw), r2 in zip(prs, raw):
                bt = TWO_PI * float(beta[iw + W - 1, jw + W - 1]) / 2.0 ** 32
                acc += math.sqrt(rho * r2) * np.exp(1j * (phi[ik, iw + c0] + phi[jk, jw + c0] + bt))
            ref = 2.0 * math.sqrt(S[kk, kw + c0] * 0.3 * 0.2) * acc
            assert abs(C[kk, kw + c0] - ref) <= 1e-12 * max(1.0, abs(ref))


def test_line_factors_separable_autoconvolution(oracle_mod):
    """Separable b2 = g g, beta = 0, no cap: the pair sum of line k is
    c_k * (1/2) [(y * y)_k + y_{k/2}^2] with y = r g e^{i phi}."""
    nk, nw, W = 6, 7, 5
    S = inp.random_spectrum(nk, nw, seed=5)
    g2 = inp.exp_bicoherence_g2(W, 0.5, 4.0, scale=0.02)
    g = np.sqrt(g2)
    rng = np.random.default_rng(6)
    lc = rng.uniform(0.2, 1.0, size=S.shape)
    lr = rng.uniform(0.5, 1.5, size=S.shape)
    P = oracle_mod.Problem(nk, nw, W, 0.1, 0.5, S, np.outer(g2, g2),
                           oracle_mod.biphase(W, None), 0.0, line_c=lc, line_r=lr)
    U = oracle_mod.phases(nk, nw, 9)
    C = P.coefficients(U=U)
    z = np.exp(1j * TWO_PI * U.astype(np.float64) / 2.0 ** 32)
    c0 = nw - 1
    y = np.zeros((nk, 2 * W - 1), dtype=np.complex128)
    y[:, :] = lr[:, c0 - (W - 1):c0 + W] * g[None, :] * z[:, c0 - (W - 1):c0 + W]
    Mk, Mw = 2 * nk, 4 * W
    Y = np.fft.fft2(y, s=(Mk, Mw))
    conv = np.fft.ifft2(Y * Y)[:nk, :4 * W - 3]      # kw = -(2W - 2) .. 2W - 2
    for kk in range(nk):
        for kw in range(-(nw - 1), nw):
            if abs(kw) > 2 * W - 2:
                T = 0.0
            else:
                T = conv[kk, kw + 2 * W - 2]
                if kk % 2 == 0 and kw % 2 == 0 and abs(kw // 2) < W:
                    T += y[kk // 2, kw // 2 + W - 1] ** 2
                T *= 0.5
            tot = P.line_terms(kk, kw)["sigma"]
            ref = 2.0 * math.sqrt(S[kk, kw + c0] * 0.05) * (math.sqrt(1.0 - tot) * z[kk, kw + c0]
                                                            + lc[kk, kw + c0] * T)
            assert abs(C[kk, kw + c0] - ref) <= 1e-11 * max(1.0, abs(ref))


def _wind(oracle_mod, nk=4, nw=5, W=None, alpha=0.3, cap=0.0, seed=3):
    S = inp.random_spectrum(nk, nw, seed=seed)
    return oracle_mod.WindProblem(nk, nw, nw if W is None else W, 0.5, 0.4, S, alpha, cap)


def test_wind_solution_in_another_order(oracle_mod):
    """Gauss-Seidel over kappa rows ascending (the pairs of a line reach rows
    <= its own; only row-internal dependencies are circular), each row iterated
    to its fixed point, in pure Python: the same S_p as the oracle's Jacobi
    sweeps over the whole grid."""
    P = _wind(oracle_mod, nk=4, nw=4, alpha=0.4, cap=0.0)
    P.solve()
    nk, nw, W = P.n_kappa, P.n_omega, P.W
    c0 = nw - 1
    Sp = P.S.copy()
    dk, dw = P.d_kappa, P.d_omega
    for kk in range(nk):
        for _ in range(500):
            new = Sp[kk].copy()
            for kw in range(-(nw - 1), nw):
                tot = 0.0
                for ik, iw, jk, jw in _pairs(nk, nw, W, kk, kw):
                    B = P.bispectrum(ik, iw, jk, jw)
                    if B > 0:
                        tot += B * B * dk * dw / (Sp[ik, iw + c0] * Sp[jk, jw + c0] * P.S[kk, kw + c0])
                new[kw + c0] = P.S[kk, kw + c0] * (1.0 - tot)
            done = np.max(np.abs(new - Sp[kk])) <= 1e-16 * np.max(P.S)
            Sp[kk] = new
            if done:
                break
    assert np.max(np.abs(Sp - P.Sp)) <= 1e-13 * np.max(P.S)
    # the fixed point: Sigma recomputed from S_p gives S_p back
    for kk in range(nk):
        for kw in range(-(nw - 1), nw):
            s = P.line_terms(kk, kw)["sigma"]
            assert P.S[kk, kw + c0] * (1.0 - s) == pytest.approx(P.Sp[kk, kw + c0], rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("cap", [0.0, 0.05])
def test_wind_factorises_into_line_factors(oracle_mod, cap):
    P = _wind(oracle_mod, nk=5, nw=6, W=4, alpha=0.5, cap=cap)
    P.solve()
    nk, nw, W = P.n_kappa, P.n_omega, P.W
    c0 = nw - 1
    kk = np.arange(nk)[:, None].astype(float)
    kw = np.abs(np.arange(-(nw - 1), nw))[None, :].astype(float)
    with np.errstate(divide="ignore"):
        lc = P.alpha * 2.0 / (3.0 * math.sqrt(3.0)) * np.sqrt(
            P.d_kappa * P.d_omega / (kw * P.d_omega * kk * P.d_kappa))
    lc[~np.isfinite(lc)] = 0.0
    lr = np.where(P.S > 0, np.sqrt(np.divide(P.S, P.Sp, where=P.Sp > 0, out=np.ones_like(P.S))), 0.0)
    T = oracle_mod.Problem(nk, nw, W, P.d_kappa, P.d_omega, P.S, np.ones((2 * W - 1, 2 * W - 1)),
                           oracle_mod.biphase(W, None), cap, line_c=lc, line_r=lr)
    a = P.coefficients(seed=11)
    b = T.coefficients(seed=11)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))
    assert lc[0].max() == 0 and lc[:, c0].max() == 0          # singular lines carry no pairs


def test_wind_third_moment_is_the_bispectrum_integral(oracle_mod):
    nk, nw, nx, nt = 3, 4, 4, 8
    P = _wind(oracle_mod, nk=nk, nw=nw, alpha=0.7, cap=0.0, seed=12)
    P.solve()
    c0 = nw - 1
    dkdw = P.d_kappa * P.d_omega
    m3, m3_wrong = 0.0, 0.0
    for kk in range(nk):
        for kw in range(-(nw - 1), nw):
            for ik, iw, jk, jw in _pairs(nk, nw, P.W, kk, kw):
                B = P.bispectrum(ik, iw, jk, jw)
                if B == 0:
                    continue
                c = 1.0 if (ik == jk and iw == jw) else 2.0
                m3 += 6.0 * c * B * dkdw ** 2
                # what the same expansion gives with S in place of S_p in b_p
                m3_wrong += 6.0 * c * B * dkdw ** 2 * math.sqrt(
                    P.Sp[ik, iw + c0] * P.Sp[jk, jw + c0] / (P.S[ik, iw + c0] * P.S[jk, jw + c0]))
    var = 2.0 * float(np.sum(P.S * dkdw))
    R = 16000
    X2, X3 = np.zeros(R), np.zeros(R)
    for r in range(R):
        u = oracle_mod.field(P.coefficients(seed=900 + r), nx, nt)
        X2[r], X3[r] = np.mean(u ** 2), np.mean(u ** 3)
    se3 = X3.std(ddof=1) / math.sqrt(R)
    se2 = X2.std(ddof=1) / math.sqrt(R)
    assert abs(X2.mean() - var) <= 4.5 * se2
    assert abs(X3.mean() - m3) <= 4.5 * se3
    assert abs(m3 - m3_wrong) >= 10 * se3        # the test can tell S_p from S


def _product(oracle_mod, nk, nw, W, seed, scale, cap=0.0, with_h=True):
    rng = np.random.default_rng(seed)
    S = inp.random_spectrum(nk, nw, seed=seed)
    shape = (nk, 2 * nw - 1)
    F = scale * (rng.uniform(0.2, 1.0, shape) * np.exp(1j * rng.uniform(0, 2 * np.pi, shape)))
    G = np.sqrt(S) * rng.uniform(0.5, 1.0, shape) * np.exp(1j * rng.uniform(0, 2 * np.pi, shape))
    H = None
    if with_h:
        A = rng.uniform(0.3, 1.0, (2 * W - 1, 2 * W - 1)) * np.exp(1j * rng.uniform(0, 2 * np.pi, (2 * W - 1, 2 * W - 1)))
        H = 0.5 * (A + A.T)
    return oracle_mod.ProductProblem(nk, nw, W, 0.5, 0.4, S, F, G, H, cap)


def test_product_bispectrum_reduces_to_wind(oracle_mod):
    """The wind bispectrum is the product form with F_k = alpha 2 sqrt(S_k) /
    (3 sqrt(3 |w_k| kappa_k)), G = sqrt(S), H = 1."""
    nk, nw, W = 5, 6, 6
    Wd = _wind(oracle_mod, nk=nk, nw=nw, W=W, alpha=0.5)
    Wd.solve()
    S = Wd.S
    kk = np.arange(nk)[:, None]
    kw = np.abs(np.arange(-(nw - 1), nw))[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        F = 0.5 * 2.0 * np.sqrt(S) / (3.0 * np.sqrt(3.0 * kw * Wd.d_omega * kk * Wd.d_kappa))
    F[~np.isfinite(F)] = 0.0
    P = oracle_mod.ProductProblem(nk, nw, W, Wd.d_kappa, Wd.d_omega, S, F + 0j, np.sqrt(S) + 0j, None, 0.0)
    P.solve()
    assert np.max(np.abs(P.Sp - Wd.Sp)) <= 1e-14 * np.max(S)
    a, b = P.coefficients(seed=8), Wd.coefficients(seed=8)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_product_solution_in_another_order(oracle_mod):
    P = _product(oracle_mod, 4, 4, 4, seed=5, scale=0.4)
    P.solve()
    nk, nw, W = P.n_kappa, P.n_omega, P.W
    c0 = nw - 1
    Sp = P.S.copy()
    dkdw = P.d_kappa * P.d_omega
    for kk in range(nk):
        for _ in range(500):
            new = Sp[kk].copy()
            for kw in range(-(nw - 1), nw):
                tot = 0.0
                for ik, iw, jk, jw in _pairs(nk, nw, W, kk, kw):
                    B = P.bispectrum_c(ik, iw, jk, jw)
                    if P.S[kk, kw + c0] > 0 and Sp[ik, iw + c0] > 0 and Sp[jk, jw + c0] > 0:
                        tot += abs(B) ** 2 * dkdw / (Sp[ik, iw + c0] * Sp[jk, jw + c0] * P.S[kk, kw + c0])
                new[kw + c0] = P.S[kk, kw + c0] * (1.0 - tot)
            done = np.max(np.abs(new - Sp[kk])) <= 1e-16 * np.max(P.S)
            Sp[kk] = new
            if done:
                break
    assert np.max(np.abs(Sp - P.Sp)) <= 1e-13 * np.max(P.S)


def test_product_third_moment_is_the_bispectrum_integral(oracle_mod):
    """With a complex prescribed B the biphase is atan2(Im B, Re B), and the
    third moment is 6 sum_k sum_{P(k)} c_p Re(B_p) (dk dw)^2."""
    nk, nw, nx, nt = 3, 4, 4, 8
    P = _product(oracle_mod, nk, nw, nw, seed=21, scale=0.9)
    P.solve()
    dkdw = P.d_kappa * P.d_omega
    m3, m3_nophase = 0.0, 0.0
    for kk in range(nk):
        for kw in range(-(nw - 1), nw):
            if P.S[kk, kw + nw - 1] <= 0:
                continue
            for ik, iw, jk, jw in _pairs(nk, nw, P.W, kk, kw):
                if P.S[ik, iw + nw - 1] <= 0 or P.S[jk, jw + nw - 1] <= 0:
                    continue
                B = P.bispectrum_c(ik, iw, jk, jw)
                c = 1.0 if (ik == jk and iw == jw) else 2.0
                m3 += 6.0 * c * B.real * dkdw ** 2
                m3_nophase += 6.0 * c * abs(B) * dkdw ** 2
    R = 20000
    X3 = np.zeros(R)
    for r in range(R):
        u = oracle_mod.field(P.coefficients(seed=3000 + r), nx, nt)
        X3[r] = np.mean(u ** 3)
    se3 = X3.std(ddof=1) / math.sqrt(R)
    assert abs(X3.mean() - m3) <= 4.5 * se3
    assert abs(m3 - m3_nophase) >= 10 * se3       # the biphase matters at this size


def test_hashed_bispectrum_brute_force(oracle_mod):
    """A bispectrum drawn per 4-index pair: the pair sum written out in Python
    with the generator called per canonical pair (i, j), k = i + j: with
    t = i_w mod 8, the 16-bit half of word t // 2 (high half for even t) of
    Philox4x32-10 at counter (i_kappa, floor(i_w / 8), j_kappa, k_w), its
    high byte u and low byte v, b2_raw = scale (u / 2^8)^2,
    beta = 2 pi v / 2^8; cap included."""
    nk, nw, W, scale, key, cap = 4, 5, 4, 0.05, 0xABCDEF12345, 0.3
    S = inp.random_spectrum(nk, nw, seed=9)
    P = oracle_mod.HashedProblem(nk, nw, W, 0.3, 0.2, S, scale, key, cap)
    U = oracle_mod.phases(nk, nw, 42)
    C = P.coefficients(U=U)
    phi = TWO_PI * U.astype(np.float64) / 2.0 ** 32
    kw0 = [key & 0xFFFFFFFF, key >> 32]
    c0 = nw - 1
    b2_seen = {}
    for kk in range(nk):
        for kw in range(-(nw - 1), nw):
            prs = list(_pairs(nk, nw, W, kk, kw))
            words = []
            for ik, iw, jk, jw in prs:
                w = int(oracle_mod.philox4x32_10([ik, (iw // 8) & 0xFFFFFFFF, jk, (iw + jw) & 0xFFFFFFFF],
                                                 kw0)[(iw % 8) // 2])
                words.append(w >> 16 if iw % 2 == 0 else w & 0xFFFF)
            b2 = [scale * (float(h >> 8) / 2.0 ** 8) ** 2 for h in words]
            for (ik, iw, jk, jw), v in zip(prs, b2):
                b2_seen.setdefault((iw, jw), set()).add(round(v, 15))
            tot = sum(b2)
            rho = cap / tot if tot > cap else 1.0
            acc = math.sqrt(1.0 - rho * tot) * np.exp(1j * phi[kk, kw + c0])
            for (ik, iw, jk, jw), v, w in zip(prs, b2, words):
                acc += math.sqrt(rho * v) * np.exp(1j * (phi[ik, iw + c0] + phi[jk, jw + c0]
                                                         + TWO_PI * float(w & 0xFF) / 2.0 ** 8))
            ref = 2.0 * math.sqrt(S[kk, kw + c0] * 0.3 * 0.2) * acc
            assert abs(C[kk, kw + c0] - ref) <= 1e-12 * max(1.0, abs(ref))
    # the same frequency pair takes different values at different wavenumbers
    assert max(len(v) for v in b2_seen.values()) > 1
