"""Seeded synthetic inputs for the 3rd-order SRM wave generator.

This module only *produces inputs*: a power spectrum sampled on the line grid,
a bicoherence description, biphase tables and realization seeds.  It holds none
of the simulation method's arithmetic (no pure spectrum, no pair sums, no
transform), so both the FP64 oracle and the GPU library may consume what it
returns without sharing any of the method's code.

Workloads follow the wind-field example of the paper (Section 5): a Kaimal
frequency spectrum times a Davenport-derived wavenumber shape,

    S(kappa, omega) = S_w(|omega|) * G(kappa | omega)
    S_w(w) = 200 u*^2 (z/U) / (1 + 50 f z/U)^(5/3),   f = w / (2 pi)
    G(k|w) = (a/pi) / (a^2 + k^2),                    a = lam |w| / (2 pi U)

with S(., 0) := 0, and a separable bicoherence
b^2_raw(w1, w2) = c * exp(-(|w1| + |w2|) / (0.5 w_u)), rescaled per line by the
generator to a cap of 0.9.  The normalisation of S_w follows the workload
definition, not the printed Kaimal constant of the paper's Section 5 (it differs
by 4 pi); the wavenumber shape is the exact Fourier transform of the Davenport
coherence.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

BETA_SEED_DEFAULT = 0x5EEDB1FA


@dataclasses.dataclass(frozen=True)
class Workload:
    """A grid + spectra + batch description (one row of the workload table)."""

    name: str
    n_kappa: int
    n_omega: int
    d_kappa: float
    d_omega: float
    n_x: int
    n_t: int
    support_w: int
    batch: int
    omega_u: float
    cap: float = 0.9
    beta_seed: int = BETA_SEED_DEFAULT
    b2_scale: float = 0.3
    U: float = 30.0
    u_star: float = 1.5
    z: float = 50.0
    lam: float = 10.0
    seed_base: int = 0
    spectrum_form: str = "workload"     # "paper": the printed closed form of Section 5
    alpha: float = 0.0                  # > 0: the wind bispectrum of Section 5, scaled

    @property
    def n_cols(self) -> int:
        return 2 * self.n_omega - 1

    @property
    def n_lines(self) -> int:
        return self.n_kappa * self.n_cols

    @property
    def grid_points(self) -> int:
        return self.n_x * self.n_t

    def seeds(self, batch: Optional[int] = None) -> np.ndarray:
        b = self.batch if batch is None else batch
        return np.arange(b, dtype=np.uint64) + np.uint64(self.seed_base)

    def spectrum(self) -> np.ndarray:
        if self.spectrum_form == "paper":
            return kaimal_davenport_paper(self.n_kappa, self.n_omega, self.d_kappa, self.d_omega,
                                          U=self.U, u_star=self.u_star, z=self.z, lam=self.lam)
        return kaimal_davenport_lines(self.n_kappa, self.n_omega, self.d_kappa,
                                      self.d_omega, U=self.U, u_star=self.u_star,
                                      z=self.z, lam=self.lam)

    def g2(self) -> np.ndarray:
        return exp_bicoherence_g2(self.support_w, self.d_omega, self.omega_u,
                                  scale=self.b2_scale)

    def b2_dense(self) -> np.ndarray:
        g = self.g2()
        return np.outer(g, g)

    def grid_dict(self) -> dict:
        return dict(n_kappa=self.n_kappa, n_omega=self.n_omega,
                    d_kappa=self.d_kappa, d_omega=self.d_omega,
                    n_x=self.n_x, n_t=self.n_t)

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def kaimal_davenport_lines(n_kappa: int, n_omega: int, d_kappa: float, d_omega: float,
                           U: float = 30.0, u_star: float = 1.5, z: float = 50.0,
                           lam: float = 10.0) -> np.ndarray:
    """S on the line grid, shape [n_kappa][2 n_omega - 1], column c <-> k_w = c - (n_omega-1).

    S(kappa, 0) is set to 0 (the Davenport shape degenerates at omega = 0).
    """
    kw = np.arange(-(n_omega - 1), n_omega, dtype=np.float64)
    w = np.abs(kw) * d_omega
    kap = np.arange(n_kappa, dtype=np.float64) * d_kappa
    f = w / (2.0 * math.pi)
    s_w = 200.0 * u_star ** 2 * (z / U) / (1.0 + 50.0 * f * z / U) ** (5.0 / 3.0)
    a = lam * w / (2.0 * math.pi * U)
    with np.errstate(divide="ignore", invalid="ignore"):
        gam = (a[None, :] / math.pi) / (a[None, :] ** 2 + kap[:, None] ** 2)
    S = s_w[None, :] * gam
    S[:, kw == 0] = 0.0
    return np.ascontiguousarray(S)


def kaimal_davenport_paper(n_kappa: int, n_omega: int, d_kappa: float, d_omega: float,
                           U: float = 40.0, u_star: float = 0.4 * 40.0 / math.log(50.0 / 0.03),
                           z: float = 50.0, lam: float = 10.0) -> np.ndarray:
    """The closed form printed in Section 5 for the bridge example, on the line
    grid with |omega| (S is even in omega) and S(., 0) := 0:
    S = (1/2)(200/2pi) u*^2 (z/U) / [1 + 50 w z/(2 pi U)]^(5/3) * a / (kappa^2 + a^2),
    a = lam w / (pi U), u* = k U / ln(z / z0) with k = 0.4, z0 = 0.03."""
    kw = np.arange(-(n_omega - 1), n_omega, dtype=np.float64)
    w = np.abs(kw) * d_omega
    kap = np.arange(n_kappa, dtype=np.float64) * d_kappa
    s_w = 0.5 * 200.0 / (2.0 * math.pi) * u_star ** 2 * (z / U) / (1.0 + 50.0 * w * z / (2.0 * math.pi * U)) ** (5.0 / 3.0)
    a = lam * w / (math.pi * U)
    with np.errstate(divide="ignore", invalid="ignore"):
        S = s_w[None, :] * a[None, :] / (kap[:, None] ** 2 + a[None, :] ** 2)
    S[:, kw == 0] = 0.0
    return np.ascontiguousarray(S)


def bridge(alpha: float = 1.0, cap: float = 0.9, batch: int = 16) -> Workload:
    """The long-span bridge example of Section 5: L = 628 m, dk = 2 pi / L,
    w_u = pi with dw = w_u / (N_w - 1), N_w = 128, N_kappa = 256, N_x = 1024,
    N_t = 2048, the printed Kaimal/Davenport closed form (U = 40 m/s, z = 50 m,
    z0 = 0.03, lam = 10), the wind bispectrum scaled by alpha, full support."""
    nk, nw = 256, 128
    L = 628.0
    return Workload(f"bridge_alpha{alpha:g}_cap{cap:g}", nk, nw, 2.0 * math.pi / L, math.pi / (nw - 1),
                    1024, 2048, nw, batch, math.pi, cap=cap, U=40.0,
                    u_star=0.4 * 40.0 / math.log(50.0 / 0.03), z=50.0, lam=10.0, seed_base=7000,
                    spectrum_form="paper", alpha=alpha)


def exp_bicoherence_g2(support_w: int, d_omega: float, omega_u: float,
                       scale: float = 0.3) -> np.ndarray:
    """Separable factor g2 over signed omega index |i_w| < W (length 2W-1).

    b^2_raw(i, j) = g2[i] * g2[j] = scale * exp(-(|w_i| + |w_j|) / (0.5 omega_u)).
    """
    kw = np.arange(-(support_w - 1), support_w, dtype=np.float64)
    return math.sqrt(scale) * np.exp(-np.abs(kw) * d_omega / (0.5 * omega_u))


# --------------------------------------------------------------------------
# Workload table.  Line grid N_kappa x N_omega, field N_x x N_t.
# --------------------------------------------------------------------------

def _c0() -> Workload:
    nk, nw = 32, 64
    return Workload("c0_32x64_fp64_b1", nk, nw, 2 * math.pi / (nk * 10.0),
                    4 * math.pi / nw, 2 * nk, 2 * nw, nw, 1, 4 * math.pi,
                    seed_base=0)


def _c1() -> Workload:
    nk, nw = 256, 1024
    return Workload("c1_256x1024_b64", nk, nw, 2 * math.pi / (nk * 10.0),
                    4 * math.pi / nw, 2 * nk, 2 * nw, nw, 64, 4 * math.pi,
                    seed_base=1000)


def _c2() -> Workload:
    nk, nw = 512, 8192
    nx, nt = 1024, 16384
    dx, dt = 2.0, 0.05
    dk = 2 * math.pi / (nx * dx)
    dw = 2 * math.pi / (nt * dt)
    omega_u = nw * dw
    # partners restricted to |omega| < 0.25 omega_u  ->  |k_w| < nw / 4
    return Workload("c2_512x8192_w2048_b16", nk, nw, dk, dw, nx, nt, nw // 4, 16,
                    omega_u, seed_base=2000)


C0 = _c0()
C1 = _c1()
C2 = _c2()
WORKLOADS = {"c0": C0, "c1": C1, "c2": C2}


def small_grid(n_kappa: int, n_omega: int, support_w: Optional[int] = None,
               batch: int = 1, n_x: Optional[int] = None, n_t: Optional[int] = None,
               seed_base: int = 0, **kw) -> Workload:
    """A c0-like workload on another line grid (same spectra recipe)."""
    w = n_omega if support_w is None else support_w
    return Workload(f"grid_{n_kappa}x{n_omega}_w{w}", n_kappa, n_omega,
                    2 * math.pi / (n_kappa * 10.0), 4 * math.pi / n_omega,
                    next_pow2(2 * n_kappa) if n_x is None else n_x,
                    next_pow2(2 * n_omega) if n_t is None else n_t, w, batch, 4 * math.pi,
                    seed_base=seed_base, **kw)


def uneven_requests(n: int = 256, seed: int = 3, log2_kappa=(6, 9), log2_omega=(7, 12),
                    scale=(0.05, 0.3), seed_base: int = 3000):
    """The uneven-batch workload: n realizations whose line grids are drawn
    log-uniformly (log2 N_kappa and log2 N_omega uniform integers, so every grid
    has power-of-two sides) from 64x128 to 512x4096 lines, each with its own
    bicoherence amplitude scale c ~ U[0.05, 0.3] (b^2_raw = c exp(...)).  Grids
    follow the 32x64 recipe (dk = 2 pi / (N_kappa 10 m), omega_u = 4 pi, field
    2N_kappa x 2N_omega).  Returns [(Workload with unit scale, c, seed)]."""
    rng = np.random.default_rng(seed)
    lk = rng.integers(log2_kappa[0], log2_kappa[1] + 1, n)
    lw = rng.integers(log2_omega[0], log2_omega[1] + 1, n)
    cs = rng.uniform(scale[0], scale[1], n)
    out = []
    for i in range(n):
        wl = small_grid(1 << int(lk[i]), 1 << int(lw[i]), b2_scale=1.0)
        out.append((wl, float(cs[i]), seed_base + i))
    return out


def next_pow2(n: int) -> int:
    p = 1
    while p < n:
        p *= 2
    return p


# --------------------------------------------------------------------------
# Generic seeded random inputs for tests (tiny grids, arbitrary spectra).
# --------------------------------------------------------------------------

def random_spectrum(n_kappa: int, n_omega: int, seed: int, zero_dc: bool = True) -> np.ndarray:
    rng = np.random.default_rng(seed)
    S = rng.uniform(0.1, 2.0, size=(n_kappa, 2 * n_omega - 1))
    S = 0.5 * (S + S[:, ::-1])          # S(k, w) = S(k, -w)
    if zero_dc:
        S[:, n_omega - 1] = 0.0
    return np.ascontiguousarray(S)


def random_b2_dense(support_w: int, seed: int, scale: float = 0.3) -> np.ndarray:
    rng = np.random.default_rng(seed)
    n = 2 * support_w - 1
    A = rng.uniform(0.0, scale, size=(n, n))
    return np.ascontiguousarray(0.5 * (A + A.T))


def random_beta_table(support_w: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    n = 2 * support_w - 1
    A = rng.integers(0, 2 ** 32, size=(n, n), dtype=np.uint64)
    A = np.triu(A) + np.triu(A, 1).T    # symmetric
    return np.ascontiguousarray(A.astype(np.uint32))


def additive_beta_table(support_w: int, seed: int) -> np.ndarray:
    """A symmetric biphase of the form gamma(i) + gamma(j) (mod 2^32)."""
    rng = np.random.default_rng(seed)
    g = rng.integers(0, 2 ** 32, size=2 * support_w - 1, dtype=np.uint64)
    return np.ascontiguousarray(((g[:, None] + g[None, :]) % (2 ** 32)).astype(np.uint32))


def random_coefficients(n_kappa: int, n_omega: int, batch: int, seed: int) -> np.ndarray:
    """Complex line coefficients [batch][n_kappa][2 n_omega - 1] (for transform tests)."""
    rng = np.random.default_rng(seed)
    shape = (batch, n_kappa, 2 * n_omega - 1)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex128)


# --------------------------------------------------------------------------
# The 1-D stochastic process u(t) (time only).  One-sided frequencies
# w_k = k dw, 0 <= k < n; the Kaimal frequency spectrum of the wave recipe
# (S(0) := 0) and the same exponential separable bicoherence over 0 <= i < W.
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class ProcessWorkload:
    name: str
    n: int
    d_omega: float
    n_t: int
    support_w: int
    batch: int
    omega_u: float
    cap: float = 0.9
    beta_seed: int = BETA_SEED_DEFAULT
    b2_scale: float = 0.3
    U: float = 30.0
    u_star: float = 1.5
    z: float = 50.0
    seed_base: int = 0

    @property
    def grid_points(self) -> int:
        return self.n_t

    def seeds(self, batch: Optional[int] = None) -> np.ndarray:
        b = self.batch if batch is None else batch
        return np.arange(b, dtype=np.uint64) + np.uint64(self.seed_base)

    def spectrum(self) -> np.ndarray:
        return kaimal_process(self.n, self.d_omega, U=self.U, u_star=self.u_star, z=self.z)

    def g2(self) -> np.ndarray:
        w = np.arange(self.support_w, dtype=np.float64) * self.d_omega
        return math.sqrt(self.b2_scale) * np.exp(-w / (0.5 * self.omega_u))

    def b2_dense(self) -> np.ndarray:
        g = self.g2()
        return np.outer(g, g)

    def grid_dict(self) -> dict:
        return dict(n_omega=self.n, d_omega=self.d_omega, n_t=self.n_t)

    def with_(self, **kw) -> "ProcessWorkload":
        return dataclasses.replace(self, **kw)


def kaimal_process(n: int, d_omega: float, U: float = 30.0, u_star: float = 1.5,
                   z: float = 50.0) -> np.ndarray:
    """One-sided S_w(w_k), k = 0 .. n-1, with S(0) := 0."""
    w = np.arange(n, dtype=np.float64) * d_omega
    f = w / (2.0 * math.pi)
    S = 200.0 * u_star ** 2 * (z / U) / (1.0 + 50.0 * f * z / U) ** (5.0 / 3.0)
    S[0] = 0.0
    return np.ascontiguousarray(S)


def small_process(n: int, support_w: Optional[int] = None, batch: int = 1,
                  n_t: Optional[int] = None, seed_base: int = 0, **kw) -> ProcessWorkload:
    w = n if support_w is None else support_w
    return ProcessWorkload(f"process_{n}_w{w}", n, 4 * math.pi / n,
                           next_pow2(2 * n) if n_t is None else n_t, w, batch, 4 * math.pi,
                           seed_base=seed_base, **kw)


def _p1() -> ProcessWorkload:
    n = 4096
    return ProcessWorkload("p1_4096_b4096", n, 4 * math.pi / n, 2 * n, n, 4096, 4 * math.pi,
                           seed_base=5000)


P1 = _p1()


def random_process_spectrum(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(0.1, 2.0, size=n))


def random_b2_quadrant(support_w: int, seed: int, scale: float = 0.3) -> np.ndarray:
    """Symmetric raw squared bicoherence over 0 <= i, j < W."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(0.0, scale, size=(support_w, support_w))
    return np.ascontiguousarray(0.5 * (A + A.T))


def random_beta_quadrant(support_w: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    A = rng.integers(0, 2 ** 32, size=(support_w, support_w), dtype=np.uint64)
    A = np.triu(A) + np.triu(A, 1).T
    return np.ascontiguousarray(A.astype(np.uint32))
