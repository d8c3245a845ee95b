"""Plan-time host logic of the kappa-dependent bicoherence (CPU only): the
library's wind line factors (fixed point through 2-D FFT autoconvolutions)
against the FP64 oracle's partial-bicoherence recursion (explicit pair
enumeration, Jacobi sweeps); argument errors."""
import math

import numpy as np
import pytest

import srm3_inputs as inp


@pytest.fixture(scope="module")
def lib():
    import paper_2310_03979_amd as p
    p.load()
    return p


CASES = [
    # nk, nw, W, alpha, cap
    (4, 5, 5, 0.4, 0.0),
    (6, 9, 4, 0.6, 0.0),       # truncated support
    (5, 6, 6, 2.0, 0.3),       # capped
    (1, 4, 4, 0.5, 0.0),       # one kappa line: no pairs (kappa_k = 0 is singular)
    (9, 3, 2, 0.8, 0.5),
    (6, 8, 8, 0.3, 0.0),       # odd n_omega - 1: self pairs at even k_omega only
    (7, 10, 6, 0.5, 0.2),
]


@pytest.mark.parametrize("case", CASES, ids=[str(c) for c in CASES])
def test_wind_factors_match_oracle_recursion(lib, oracle_mod, case):
    nk, nw, W, alpha, cap = case
    S = inp.random_spectrum(nk, nw, seed=nk + nw)
    grid = dict(n_kappa=nk, n_omega=nw, d_kappa=0.37, d_omega=0.21)
    c, r, sig, sweeps = lib.srm3_wind_factors(grid, S, alpha, cap, W)
    P = oracle_mod.WindProblem(nk, nw, W, 0.37, 0.21, S, alpha, cap)
    P.solve()
    sig_ref = np.where(S > 0, 1.0 - P.Sp / np.where(S > 0, S, 1.0), 0.0)
    assert np.max(np.abs(sig - sig_ref)) <= 1e-13
    r_ref = np.where(S > 0, np.sqrt(S / np.where(P.Sp > 0, P.Sp, 1.0)), 0.0)
    assert np.max(np.abs(r - r_ref)) <= 1e-13
    kk = np.arange(nk)[:, None]
    kw = np.abs(np.arange(-(nw - 1), nw))[None, :]
    with np.errstate(divide="ignore"):
        c_ref = alpha * 2.0 / (3.0 * math.sqrt(3.0)) / np.sqrt(kw * kk)
    c_ref[~np.isfinite(c_ref)] = 0.0
    assert np.allclose(c, c_ref, rtol=1e-15, atol=0)
    assert sweeps >= 1


def test_wind_errors(lib):
    S = inp.random_spectrum(3, 4, seed=1)
    grid = dict(n_kappa=3, n_omega=4, d_kappa=0.5, d_omega=0.4)
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3_wind_factors(grid, S, 50.0, 0.0, 4)       # no admissible pure spectrum
    assert ei.value.status == 2
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3_wind_factors(grid, S, -1.0, 0.0, 4)
    assert ei.value.status == 1
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3_wind_factors(grid, S, 1.0, 1.5, 4)
    assert ei.value.status == 1
    c, r, sig, _ = lib.srm3_wind_factors(grid, S, 50.0, 0.6, 4)   # the cap makes it admissible
    assert sig.max() <= 0.6 + 1e-15


def _product_inputs(nk, nw, W, seed, scale):
    rng = np.random.default_rng(seed)
    S = inp.random_spectrum(nk, nw, seed=seed)
    shape = S.shape
    F = scale * rng.uniform(0.2, 1.0, shape) * np.exp(1j * rng.uniform(0, 2 * np.pi, shape))
    G = np.sqrt(S) * rng.uniform(0.5, 1.0, shape) * np.exp(1j * rng.uniform(0, 2 * np.pi, shape))
    A = rng.uniform(0.3, 1.0, (2 * W - 1, 2 * W - 1)) * np.exp(1j * rng.uniform(0, 2 * np.pi, (2 * W - 1, 2 * W - 1)))
    return S, F, G, 0.5 * (A + A.T)


@pytest.mark.parametrize("with_h", [True, False])
@pytest.mark.parametrize("case", [(4, 5, 5, 0.4, 0.0), (6, 8, 5, 2.0, 0.5), (3, 7, 7, 0.6, 0.0),
                                  (16, 24, 12, 2.0, 0.7)],   # sweeps settle at the rounding floor of the sums
                         ids=str)
def test_product_factors_match_oracle_recursion(lib, oracle_mod, case, with_h):
    nk, nw, W, scale, cap = case
    S, F, G, H = _product_inputs(nk, nw, W, nk * nw, scale)
    if not with_h:
        H = None
    grid = dict(n_kappa=nk, n_omega=nw, d_kappa=0.5, d_omega=0.4)
    c, rho, sig, sweeps = lib.srm3_product_factors(grid, S, F, G, H, W, cap)
    P = oracle_mod.ProductProblem(nk, nw, W, 0.5, 0.4, S, F, G, H, cap)
    P.solve()
    pos = S > 0
    sig_ref = np.where(pos, 1.0 - P.Sp / np.where(pos, S, 1.0), 0.0)
    assert np.max(np.abs(sig - sig_ref)) <= 1e-13
    c_ref = np.where(pos, F * np.sqrt(0.5 * 0.4 / np.where(pos, S, 1.0)), 0.0)
    assert np.max(np.abs(c - c_ref)) <= 1e-13 * np.max(np.abs(c_ref))
    rho_ref = np.where(pos, G / np.sqrt(np.where(pos, P.Sp, 1.0)), 0.0)
    assert np.max(np.abs(rho - rho_ref)) <= 1e-12 * np.max(np.abs(rho_ref))
    assert sweeps >= 1
