"""Ensemble invariants of the oracle's fields (Monte Carlo, CPU only).

Closed forms, derived from the phase algebra of the 3rd-order expansion
(Section 4.1): with independent uniform line phases, every monomial of C_k has
positive phase degree, so

    E[u]   = 0
    E[u^2] = 2 sum_k S_k dk dw                                   (any admissible b)
    E[u^3] = 6 sum_k sum_{p={i,j} in P(k)} c_p A_k A_i A_j s_i s_j b_p cos(beta_p)

with A = sqrt(S dk dw), s = sqrt(1 - Sigma), c_p = 2 for i != j and 1 for the
self pair.  The variance is the discrete integral of the power spectrum and the
third moment the discrete integral of the bispectrum (Section 5 validates the
method the same way through the skewness).  Tolerances are CLT bounds from the
sample spread of per-realization grid averages.
"""
import math

import numpy as np
import pytest

import srm3_inputs as inp

NSIG = 4.5


def _closed_forms(P, S, b2, beta, self_weight=1.0):
    nk, nw, W = P.n_kappa, P.n_omega, P.W
    dk, dw = P.d_kappa, P.d_omega
    A = np.sqrt(S * dk * dw)
    s = np.zeros_like(S)
    rho = np.zeros_like(S)
    for kk in range(nk):
        for kw in range(-(nw - 1), nw):
            t = P.line_terms(kk, kw)
            s[kk, kw + nw - 1] = math.sqrt(1.0 - t["sigma"])
            rho[kk, kw + nw - 1] = t["rho"]
    var = 2.0 * float(np.sum(S * dk * dw))
    m3 = 0.0
    for kk in range(nk):
        for kw in range(-(nw - 1), nw):
            ck = kw + nw - 1
            for ik in range(kk + 1):
                jk = kk - ik
                for iw in range(-(W - 1), W):
                    jw = kw - iw
                    if abs(jw) >= W or not ((ik > jk) or (ik == jk and iw >= jw)):
                        continue
                    c = self_weight if (ik == jk and iw == jw) else 2.0
                    bp = math.sqrt(rho[kk, ck] * b2[iw + W - 1, jw + W - 1])
                    bt = 2 * math.pi * float(beta[iw + W - 1, jw + W - 1]) / 4294967296.0
                    m3 += 6.0 * c * A[kk, ck] * A[ik, iw + nw - 1] * A[jk, jw + nw - 1] \
                        * s[ik, iw + nw - 1] * s[jk, jw + nw - 1] * bp * math.cos(bt)
    return var, m3


def _ensemble(oracle_mod, P, nx, nt, R, seed0):
    X1, X2, X3 = np.zeros(R), np.zeros(R), np.zeros(R)
    for r in range(R):
        u = oracle_mod.field(P.coefficients(seed=seed0 + r), nx, nt)
        X1[r], X2[r], X3[r] = u.mean(), np.mean(u ** 2), np.mean(u ** 3)
    return X1, X2, X3


def _se(x):
    return x.std(ddof=1) / math.sqrt(x.size)


@pytest.mark.parametrize("case", ["dense_beta0", "dense_seeded_beta", "selfpair_only"])
def test_ensemble_moments_match_closed_forms(oracle_mod, case):
    if case == "selfpair_only":
        # one kappa row and a diagonal bicoherence: every pair is a self pair
        nk, nw, W, nx, nt = 1, 4, 4, 2, 8
        S = inp.random_spectrum(nk, nw, seed=41)
        b2 = np.diag(np.diag(inp.random_b2_dense(W, seed=42, scale=0.3))) * 2
        beta = oracle_mod.biphase(W, None)
    else:
        nk, nw, W, nx, nt = 4, 4, 4, 8, 8
        S = inp.random_spectrum(nk, nw, seed=41)
        b2 = inp.random_b2_dense(W, seed=42, scale=0.3)
        beta = oracle_mod.biphase(W, None if case == "dense_beta0" else 777)
    P = oracle_mod.Problem(nk, nw, W, 1.0, 1.0, S, b2, beta, 0.9)
    var, m3 = _closed_forms(P, S, b2, beta)
    X1, X2, X3 = _ensemble(oracle_mod, P, nx, nt, 20000, 1_000_000)
    # S(0, 0) = 0: every realization has exactly zero grid mean
    assert np.max(np.abs(X1)) < 1e-12 * math.sqrt(var)
    assert abs(X2.mean() - var) < NSIG * _se(X2)
    assert abs(X3.mean() - m3) < NSIG * _se(X3)
    if case == "dense_beta0":
        assert m3 > 20 * _se(X3)                 # the skewness signal is real
    if case == "selfpair_only":
        # counting the self pair twice (or not at all) is rejected
        _, m3_double = _closed_forms(P, S, b2, beta, self_weight=2.0)
        _, m3_none = _closed_forms(P, S, b2, beta, self_weight=0.0)
        assert abs(X3.mean() - m3_double) > 10 * _se(X3)
        assert abs(X3.mean() - m3_none) > 10 * _se(X3)


def test_c0_variance_is_spectrum_integral(oracle_mod):
    """Per-realization Parseval mean vs the theoretical variance on the 32x64 grid."""
    wl = inp.C0
    P = oracle_mod.Problem.from_workload(wl)
    S = wl.spectrum()
    var = 2.0 * float(np.sum(S * wl.d_kappa * wl.d_omega))
    vals = []
    for r in range(64):
        C = P.coefficients(seed=5000 + r)
        row0 = C[0]
        vals.append(0.5 * np.sum(np.abs(C[1:]) ** 2)
                    + 0.25 * np.sum(np.abs(row0 + np.conj(row0[::-1])) ** 2))
    vals = np.asarray(vals)
    assert abs(vals.mean() - var) < NSIG * _se(vals)
    assert abs(var - 113.63) < 0.01 * 113.63
