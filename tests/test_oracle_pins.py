"""Pins of the FP64 oracle against mathematics and published values (CPU only).

Each test ties one part of the oracle to something other than itself:

* Philox4x32-10 known-answer vectors (Salmon et al., SC'11)        -> RNG
* literal direct double cosine sum (Section 4.1, Eq.
  truncated_cosines_1d_wave) with 4-index pair enumeration            -> coefficients + transform
* Gaussian limit b = 0: the 2nd-order SRM sum (Section 3) and numpy's
  inverse 2-D FFT (Section 3, Eq. 2_order_fft)                        -> transform, sign, scaling
* separable bicoherence with additive biphase: the pair sum is half a
  2-D linear autoconvolution plus the self-pair diagonal (numpy FFT)  -> pair set P(k), cap, support
* closed-form pair counts                                            -> enumeration bounds
* per-realization invariants (zero grid mean, Parseval)              -> transform
"""
import math
import os

import numpy as np
import pytest

import srm3_inputs as inp

HERE = os.path.dirname(os.path.abspath(__file__))
TWO32 = 4294967296.0


def _problem(oracle_mod, nk, nw, W, S, b2, beta, cap, dk=0.37, dw=0.21):
    return oracle_mod.Problem(nk, nw, W, dk, dw, S, b2, beta, cap)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# --------------------------------------------------------------------------
def test_philox_known_answers(oracle_mod):
    path = os.path.join(HERE, "golden", "philox4x32_10_kat.txt")
    n = 0
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(x, 16) for x in line.split()]
        out = oracle_mod.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]
        n += 1
    assert n == 3


def test_phase_and_biphase_streams(oracle_mod):
    """Phases: word kw mod 4 of counter (kk, floor(kw / 4), 0, 0), so one call
    serves four consecutive frequencies; biphases (max, min, 1, 0), symmetric."""
    nw = 11
    U = oracle_mod.phases(3, nw, seed=0x1234_5678_9ABC)
    key = [0x56789ABC, 0x1234]
    for kk in range(3):
        for kw in range(-(nw - 1), nw):
            ctr = [kk, (kw // 4) & 0xFFFFFFFF, 0, 0]
            assert U[kk, kw + nw - 1] == oracle_mod.philox4x32_10(ctr, key)[kw % 4]
    # the four words of one call, e.g. counter (2, -2): k_w = -8 .. -5
    w = oracle_mod.philox4x32_10([2, (-2) & 0xFFFFFFFF, 0, 0], key)
    assert [int(x) for x in U[2, -8 + nw - 1:-4 + nw - 1]] == [int(x) for x in w]
    assert len(set(int(x) for x in U.ravel())) == U.size   # no word serves two lines
    B = oracle_mod.biphase(3, seed=77)
    assert np.array_equal(B, B.T)
    assert B[4, 0] == oracle_mod.philox4x32_10([2, (-2) & 0xFFFFFFFF, 1, 0], [77, 0])[0]
    assert B[0, 4] == B[4, 0]
    assert not np.any(oracle_mod.biphase(3, None))
    # uniformity sanity: fixed-point phases cover the circle evenly
    U = oracle_mod.phases(64, 64, seed=5).astype(np.float64) / TWO32
    hist = np.histogram(U, bins=8, range=(0, 1))[0]
    assert hist.min() > 0.9 * U.size / 8


# --------------------------------------------------------------------------
def _brute_force_field(nk, nw, W, dk, dw, nx, nt, S, b2, beta, U, cap):
    """Literal direct double cosine sum of Section 4.1 (plain Python loops).

    Pairs are found by enumerating every ordered pair of lines (4 indices),
    keeping i + j = k, the support |w| < W and one member of each unordered
    pair (lexicographic on (kappa, omega)).  Angles are formed in floating
    point from x = mx dx, t = mt dt with dk dx = 2 pi / nx, dw dt = 2 pi / nt.
    """
    lines = [(kk, kw) for kk in range(nk) for kw in range(-(nw - 1), nw)]
    phi = {k: 2 * math.pi * float(U[k[0], k[1] + nw - 1]) / TWO32 for k in lines}
    pairs = {k: [] for k in lines}
    for i in lines:
        for j in lines:
            k = (i[0] + j[0], i[1] + j[1])
            if k not in pairs or abs(i[1]) >= W or abs(j[1]) >= W or i < j:
                continue
            pairs[k].append((i, j))
    dx, dt = 2 * math.pi / (nx * dk), 2 * math.pi / (nt * dw)
    X, T = np.meshgrid(np.arange(nx) * dx, np.arange(nt) * dt, indexing="ij")
    u = np.zeros((nx, nt))
    for k in lines:
        kap, om = k[0] * dk, k[1] * dw
        Sk = S[k[0], k[1] + nw - 1]
        braw = [b2[i[1] + W - 1, j[1] + W - 1] for i, j in pairs[k]]
        sraw = sum(braw)
        rho = min(1.0, cap / sraw) if (cap > 0 and sraw > 0) else 1.0
        Sp = Sk * (1.0 - rho * sraw)
        u += 2 * math.sqrt(Sp * dk * dw) * np.cos(kap * X + om * T + phi[k])
        for (i, j), br in zip(pairs[k], braw):
            bt = 2 * math.pi * float(beta[i[1] + W - 1, j[1] + W - 1]) / TWO32
            u += 2 * math.sqrt(Sk * dk * dw) * math.sqrt(rho * br) * \
                np.cos(kap * X + om * T + phi[i] + phi[j] + bt)
    return u


@pytest.mark.parametrize("nk,nw,W,nx,nt,cap", [(4, 4, 4, 8, 8, 0.9), (3, 4, 3, 8, 9, 0.9),
                                               (4, 3, 2, 9, 6, 0.0)])
def test_brute_force_literal_sum(oracle_mod, nk, nw, W, nx, nt, cap):
    S = inp.random_spectrum(nk, nw, seed=11)
    scale = 0.3 if cap > 0 else 0.05
    b2 = inp.random_b2_dense(W, seed=12, scale=scale)
    beta = inp.random_beta_table(W, seed=13)
    U = oracle_mod.phases(nk, nw, seed=99)
    P = _problem(oracle_mod, nk, nw, W, S, b2, beta, cap)
    u = oracle_mod.field(P.coefficients(U=U), nx, nt)
    ref = _brute_force_field(nk, nw, W, P.d_kappa, P.d_omega, nx, nt, S, b2, beta, U, cap)
    assert _rel(u, ref) < 1e-12


# --------------------------------------------------------------------------
def test_gaussian_limit_matches_second_order_srm_and_ifft2(oracle_mod):
    nk, nw, nx, nt = 6, 5, 16, 12
    S = inp.random_spectrum(nk, nw, seed=3)
    W = nw
    b2 = np.zeros((2 * W - 1, 2 * W - 1))
    beta = inp.random_beta_table(W, seed=4)
    P = _problem(oracle_mod, nk, nw, W, S, b2, beta, 0.9)
    U = oracle_mod.phases(nk, nw, seed=2024)
    C = P.coefficients(U=U)
    phi = 2 * math.pi * U.astype(np.float64) / TWO32
    A = 2 * np.sqrt(S * P.d_kappa * P.d_omega)
    assert np.allclose(C, A * np.exp(1j * phi), rtol=0, atol=1e-14 * A.max())
    u = oracle_mod.field(C, nx, nt)
    # numpy inverse FFT (normalised by 1/(nx nt)) of the coefficients placed at
    # bins (kk, kw mod nt)
    buf = np.zeros((nx, nt), dtype=complex)
    for c in range(2 * nw - 1):
        buf[:nk, (c - (nw - 1)) % nt] = C[:, c]
    ref_fft = np.real(np.fft.ifft2(buf)) * nx * nt
    assert _rel(u, ref_fft) < 1e-12
    # 2nd-order SRM: u = 2 sum_k sum_{w>=0} sum_{+-} sqrt(S(k, +-w) dk dw) cos(k x +- w t + phi^{+-})
    dx, dt = 2 * math.pi / (nx * P.d_kappa), 2 * math.pi / (nt * P.d_omega)
    X, T = np.meshgrid(np.arange(nx) * dx, np.arange(nt) * dt, indexing="ij")
    ref2 = np.zeros((nx, nt))
    for kk in range(nk):
        for kw in range(0, nw):
            for sgn in (+1, -1):
                if kw == 0 and sgn < 0:
                    continue          # one line at omega = 0 (S(., 0) = 0 here)
                c = sgn * kw + nw - 1
                ref2 += 2 * math.sqrt(S[kk, c] * P.d_kappa * P.d_omega) * np.cos(
                    kk * P.d_kappa * X + sgn * kw * P.d_omega * T + phi[kk, c])
    assert _rel(u, ref2) < 1e-12


# --------------------------------------------------------------------------
def _conv2_full(a, b):
    """Full 2-D linear convolution by zero-padded numpy FFT."""
    sh = (a.shape[0] + b.shape[0] - 1, a.shape[1] + b.shape[1] - 1)
    return np.fft.ifft2(np.fft.fft2(a, sh) * np.fft.fft2(b, sh))


@pytest.mark.parametrize("nk,nw,W,cap,beta_kind", [(8, 8, 8, 0.9, "zero"), (8, 8, 5, 0.9, "additive"),
                                                   (5, 6, 6, 0.0, "additive"), (7, 5, 3, 0.5, "zero")])
def test_separable_pair_sum_is_half_autoconvolution(oracle_mod, nk, nw, W, cap, beta_kind):
    nc, nwc = 2 * nw - 1, 2 * W - 1
    S = inp.random_spectrum(nk, nw, seed=21)
    rng = np.random.default_rng(22)
    q = rng.uniform(0.0, 0.3 if cap > 0 else 0.02, size=nwc)      # b2_raw = q_i q_j
    b2 = np.outer(q, q)
    if beta_kind == "zero":
        beta = np.zeros((nwc, nwc), dtype=np.uint32)
        gam = np.zeros(nwc)
    else:
        g32 = rng.integers(0, 2 ** 32, size=nwc, dtype=np.uint64)
        beta = ((g32[:, None] + g32[None, :]) % 2 ** 32).astype(np.uint32)
        gam = 2 * math.pi * g32.astype(np.float64) / TWO32
    P = _problem(oracle_mod, nk, nw, W, S, b2, beta, cap)
    U = oracle_mod.phases(nk, nw, seed=31)
    C = P.coefficients(U=U)
    z = np.exp(2j * math.pi * U.astype(np.float64) / TWO32)
    # y = sqrt(q) e^{i gamma} z on the support, zero elsewhere
    off = nw - W
    y = np.zeros((nk, nc), dtype=complex)
    Q = np.zeros((nk, nc))
    y[:, off:off + nwc] = (np.sqrt(q) * np.exp(1j * gam))[None, :] * z[:, off:off + nwc]
    Q[:, off:off + nwc] = q[None, :]
    yy = _conv2_full(y, y)
    QQ = np.real(_conv2_full(Q, Q))
    ref = np.zeros((nk, nc), dtype=complex)
    for kk in range(nk):
        for c in range(nc):
            kw = c - (nw - 1)
            r = kw + 2 * (nw - 1)                   # column of (y*y) for output kw
            T = yy[kk, r]
            sr = QQ[kk, r]
            if kk % 2 == 0 and kw % 2 == 0 and abs(kw // 2) < W:
                hc = kw // 2 + nw - 1
                T += y[kk // 2, hc] ** 2
                sr += Q[kk // 2, hc] ** 2
            T *= 0.5
            sr *= 0.5
            rho = min(1.0, cap / sr) if (cap > 0 and sr > 0) else 1.0
            amp = 2 * math.sqrt(S[kk, c] * P.d_kappa * P.d_omega)
            ref[kk, c] = amp * (math.sqrt(1 - rho * sr) * z[kk, c] + math.sqrt(rho) * T)
    assert _rel(C, ref) < 1e-11


# --------------------------------------------------------------------------
@pytest.mark.parametrize("nk,nw,W", [(6, 5, 5), (5, 7, 3)])
def test_pair_count_closed_form(oracle_mod, nk, nw, W):
    nwc = 2 * W - 1
    P = _problem(oracle_mod, nk, nw, W, inp.random_spectrum(nk, nw, 1),
                 np.zeros((nwc, nwc)), np.zeros((nwc, nwc), np.uint32), 0.9)
    for kk in range(nk):
        for kw in range(-(nw - 1), nw):
            n_w = sum(1 for iw in range(-(W - 1), W) if abs(kw - iw) < W)   # ordered splits
            diag = 1 if (kk % 2 == 0 and kw % 2 == 0 and abs(kw // 2) < W) else 0
            assert P.line_terms(kk, kw)["npairs"] == ((kk + 1) * n_w + diag) // 2


def test_c0_pair_total_and_cap(oracle_mod):
    """Pair total of the 32x64 workload, and the cap bites on every line with pairs."""
    wl = inp.C0
    P = oracle_mod.Problem.from_workload(wl)
    tot = 0
    for kk in range(wl.n_kappa):
        for kw in range(-(wl.n_omega - 1), wl.n_omega):
            t = P.line_terms(kk, kw)
            tot += t["npairs"]
            assert t["sigma"] <= wl.cap + 1e-15
    nw, nk = wl.n_omega, wl.n_kappa
    ordered_w = sum(2 * nw - 1 - abs(kw) for kw in range(-(nw - 1), nw))
    even_kk = len(range(0, nk, 2))
    even_kw = sum(1 for kw in range(-(nw - 1), nw) if kw % 2 == 0)
    assert 2 * tot == nk * (nk + 1) // 2 * ordered_w + even_kk * even_kw
    assert tot == 3194112


# --------------------------------------------------------------------------
def test_transform_invariants_c0(oracle_mod):
    """Zero grid mean (S(0,0) = 0) and Parseval with the kappa = 0 row pairing."""
    wl = inp.C0
    P = oracle_mod.Problem.from_workload(wl)
    C = P.coefficients(seed=0)
    u = oracle_mod.field_nested(C, wl.n_x, wl.n_t)
    nw = wl.n_omega
    assert abs(u.mean()) < 1e-12 * np.abs(u).max()
    row0 = C[0]
    parse = 0.5 * np.sum(np.abs(C[1:]) ** 2) + 0.25 * np.sum(np.abs(row0 + np.conj(row0[::-1])) ** 2)
    assert abs(np.mean(u ** 2) - parse) < 1e-12 * parse


def test_nested_equals_flat_field(oracle_mod):
    wl = inp.small_grid(8, 16)
    P = oracle_mod.Problem.from_workload(wl)
    C = P.coefficients(seed=7)
    a = oracle_mod.field(C, wl.n_x, wl.n_t)
    b = oracle_mod.field_nested(C, wl.n_x, wl.n_t)
    assert _rel(b, a) < 1e-12
    rng = np.random.default_rng(0)
    mx = rng.integers(0, wl.n_x, 50)
    mt = rng.integers(0, wl.n_t, 50)
    assert _rel(oracle_mod.field_points(C, wl.n_x, wl.n_t, mx, mt), a[mx, mt]) < 1e-12


def test_sigma_error_without_cap(oracle_mod):
    wl = inp.small_grid(8, 8)
    P = oracle_mod.Problem.from_workload(wl, cap=0.0)
    assert max(P.line_terms(kk, kw)["status"] for kk in range(8) for kw in range(-7, 8)) == 2
    with pytest.raises(ValueError):
        P.coefficients(seed=1)
