"""Pins of the oracle's 1-D stochastic process u(t) (Section 3, the 3rd-order
SRM for a process in the form of Shields and Kim), CPU only.

* the cosine form written out in plain Python on tiny inputs (every pair, the
  pure amplitude, the cap) against the oracle's coefficients + field;
* the process is the wave of Section 4.1 with one wavenumber line, no spectrum
  at negative frequencies and no bicoherence with a negative partner: the
  independently pinned wave oracle gives the same coefficients and field;
* zero bicoherence: C_k = 2 sqrt(S_k dw) e^{i phi_k} and the field is a
  library inverse FFT of it;
* pair counts in closed form;
* ensemble moments against their closed forms (Monte Carlo, CLT bounds).
"""
import math

import numpy as np
import pytest

import srm3_inputs as inp

TWO_PI = 2.0 * math.pi


def _problem(oracle_mod, n, W, seed=1, cap=0.0, beta="table", scale=0.3, dw=0.37):
    S = inp.random_process_spectrum(n, seed)
    b2 = inp.random_b2_quadrant(W, seed + 1, scale=scale)
    if beta == "table":
        bt = inp.random_beta_quadrant(W, seed + 2)
    elif beta == "zero":
        bt = oracle_mod.process_biphase(W, None)
    else:
        bt = oracle_mod.process_biphase(W, 99)
    return oracle_mod.ProcessProblem(n, W, dw, S, b2, bt, cap)


def test_phases_and_biphase_follow_the_generator(oracle_mod):
    U = oracle_mod.process_phases(9, 1234)
    key = [1234 & 0xFFFFFFFF, 1234 >> 32]
    for k in range(9):
        assert U[k] == oracle_mod.philox4x32_10([0, k // 4, 0, 0], key)[k % 4]
    B = oracle_mod.process_biphase(5, 77)
    for i in range(5):
        for j in range(5):
            assert B[i, j] == oracle_mod.philox4x32_10([max(i, j), min(i, j), 1, 0], [77, 0])[0]
    assert np.all(oracle_mod.process_biphase(5, None) == 0)


@pytest.mark.parametrize("cap", [0.0, 0.4])
@pytest.mark.parametrize("n,W", [(7, 5), (6, 6), (9, 3)])
def test_cosine_form_brute_force(oracle_mod, n, W, cap):
    P = _problem(oracle_mod, n, W, seed=n + W, cap=cap, scale=0.12)
    nt, seed = 16, 4242
    U = oracle_mod.process_phases(n, seed)
    phi = TWO_PI * U.astype(np.float64) / 2.0 ** 32
    u = oracle_mod.process_field(P.coefficients(U=U), nt)
    dw = P.d_omega
    dt = TWO_PI / (nt * dw)
    ref = np.zeros(nt)
    for m in range(nt):
        t = m * dt
        acc = 0.0
        for k in range(n):
            pairs = [(k - j, j) for j in range(0, k // 2 + 1) if k - j < W]
            raw = sum(P.b2[i, j] for i, j in pairs)
            rho = cap / raw if (cap > 0 and raw > cap) else 1.0
            sigma = rho * raw
            acc += math.sqrt(P.S[k] * (1.0 - sigma) * dw) * math.cos(k * dw * t + phi[k])
            for i, j in pairs:
                bp = math.sqrt(rho * P.b2[i, j])
                beta = TWO_PI * float(P.beta[i, j]) / 2.0 ** 32
                acc += math.sqrt(P.S[k] * dw) * bp * math.cos(k * dw * t + phi[i] + phi[j] + beta)
        ref[m] = 2.0 * acc
    assert np.max(np.abs(u - ref)) <= 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("beta", ["seeded", "zero"])
def test_restriction_of_the_wave(oracle_mod, beta):
    n, W, nt = 12, 9, 32
    P = _problem(oracle_mod, n, W, seed=3, cap=0.5, beta=beta)
    # the wave with one kappa line: S and b2 vanish on the negative side
    Sw = np.zeros((1, 2 * n - 1))
    Sw[0, n - 1:] = P.S
    b2w = np.zeros((2 * W - 1, 2 * W - 1))
    b2w[W - 1:, W - 1:] = P.b2
    betaw = oracle_mod.biphase(W, None if beta == "zero" else 99)
    assert np.array_equal(betaw[W - 1:, W - 1:], P.beta)
    wave = oracle_mod.Problem(1, n, W, 1.0, P.d_omega, Sw, b2w, betaw, 0.5)
    seed = 31
    Cw = wave.coefficients(seed=seed)
    assert np.array_equal(oracle_mod.phases(1, n, seed)[0, n - 1:], oracle_mod.process_phases(n, seed))
    Cp = P.coefficients(seed=seed)
    assert np.all(Cw[0, :n - 1] == 0)
    assert np.max(np.abs(Cw[0, n - 1:] - Cp)) <= 1e-13 * np.max(np.abs(Cp))
    uw = oracle_mod.field(Cw, 1, nt)[0]
    up = oracle_mod.process_field(Cp, nt)
    assert np.max(np.abs(uw - up)) <= 1e-12 * np.max(np.abs(up))
    for k in range(n):
        assert P.terms(k)["sigma"] == pytest.approx(wave.line_terms(0, k)["sigma"], rel=1e-14, abs=1e-15)


def test_zero_bicoherence_is_the_second_order_form(oracle_mod):
    n, W, nt = 20, 20, 64
    S = inp.random_process_spectrum(n, 5)
    P = oracle_mod.ProcessProblem(n, W, 0.2, S, np.zeros((W, W)), oracle_mod.process_biphase(W, 1), 0.0)
    U = oracle_mod.process_phases(n, 8)
    C = P.coefficients(U=U)
    ref = 2.0 * np.sqrt(S * 0.2) * np.exp(1j * TWO_PI * U.astype(np.float64) / 2.0 ** 32)
    assert np.max(np.abs(C - ref)) <= 1e-15 * np.max(np.abs(ref))
    X = np.zeros(nt, dtype=np.complex128)
    X[:n] = C
    u_fft = (np.fft.ifft(X) * nt).real
    assert np.max(np.abs(oracle_mod.process_field(C, nt) - u_fft)) <= 1e-12 * np.max(np.abs(u_fft))


@pytest.mark.parametrize("n,W", [(10, 10), (10, 4), (5, 1)])
def test_pair_counts(oracle_mod, n, W):
    P = _problem(oracle_mod, n, W)
    for k in range(n):
        expect = max(0, k // 2 - max(0, k - W + 1) + 1)
        assert P.terms(k)["npairs"] == expect


NSIG = 4.5


def _se(x):
    return x.std(ddof=1) / math.sqrt(x.size)


@pytest.mark.parametrize("beta", ["zero", "seeded"])
def test_ensemble_moments_match_closed_forms(oracle_mod, beta):
    """E[u] = 0, E[u^2] = 2 sum S dw, E[u^3] = 6 sum_k sum_{p} c_p A_k A_i A_j
    s_i s_j b_p cos(beta_p) (A = sqrt(S dw), s = sqrt(1 - Sigma), c_p = 2 off
    the diagonal, 1 for the self pair): the discrete integrals of the power
    spectrum and the bispectrum."""
    n, W, nt, R = 8, 8, 16, 3000
    P = _problem(oracle_mod, n, W, seed=11, cap=0.0, beta=beta, scale=0.1)
    A = np.sqrt(P.S * P.d_omega)
    s = np.array([math.sqrt(1.0 - P.terms(k)["sigma"]) for k in range(n)])
    var = 2.0 * float(np.sum(P.S * P.d_omega))
    m3 = 0.0
    for k in range(n):
        for j in range(0, k // 2 + 1):
            i = k - j
            if i >= W:
                continue
            c = 1.0 if i == j else 2.0
            bt = TWO_PI * float(P.beta[i, j]) / 2.0 ** 32
            m3 += 6.0 * c * A[k] * A[i] * A[j] * s[i] * s[j] * math.sqrt(P.b2[i, j]) * math.cos(bt)
    X1, X2, X3 = np.zeros(R), np.zeros(R), np.zeros(R)
    for r in range(R):
        u = oracle_mod.process_field(P.coefficients(seed=700 + r), nt)
        X1[r], X2[r], X3[r] = u.mean(), np.mean(u ** 2), np.mean(u ** 3)
    assert abs(X1.mean()) <= NSIG * _se(X1) + 1e-12
    assert abs(X2.mean() - var) <= NSIG * _se(X2)
    assert abs(X3.mean() - m3) <= NSIG * _se(X3)
    if beta == "zero":
        # a real positive bispectrum gives a clearly positive third moment
        assert m3 > 4 * _se(X3)
