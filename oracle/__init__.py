"""FP64 CPU oracle for the 3rd-order SRM stochastic wave (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The GPU library never imports,
links or executes anything here, and this package imports nothing from it.

The arithmetic lives in ``srm3_oracle.c`` (plain C, FP64, libm cos/sin, OpenMP
over independent outputs).  This file only builds and marshals:

* ``phases``          -- fixed-point phase angle of every line (Philox4x32-10)
* ``biphase``         -- fixed-point biphase table (seeded or zero)
* ``line_terms``      -- raw bicoherence sum, rescale factor, Sigma, pair count
* ``coefficients``    -- C_k by explicit enumeration of the pair set P(k)
* ``field`` / ``field_points`` / ``field_nested`` -- direct cosine sums
* ``WindProblem``, ``ProductProblem`` -- kappa-dependent bispectra through the
  partial-bicoherence recursion (Section 4.1, Section 5)
* ``ProcessProblem``, ``process_phases``, ``process_biphase``,
  ``process_field`` -- the 1-D stochastic process u(t) (Section 3)

Every function cites the part of the paper it follows in the C source.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "srm3_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_lp = ctypes.POINTER(ctypes.c_long)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` with gcc (FP64, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Problem(ctypes.Structure):
    _fields_ = [("nk", ctypes.c_int), ("nw", ctypes.c_int), ("W", ctypes.c_int),
                ("dk", ctypes.c_double), ("dw", ctypes.c_double),
                ("S", _dp), ("b2", _dp), ("beta", _u32p), ("cap", ctypes.c_double),
                ("line_c", _dp), ("line_r", _dp), ("mode", ctypes.c_int), ("alpha", ctypes.c_double),
                ("Sp", _dp), ("F", _dp), ("G", _dp), ("H", _dp), ("hash_key", ctypes.c_uint64)]


class _Process(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("W", ctypes.c_int), ("dw", ctypes.c_double),
                ("S", _dp), ("b2", _dp), ("beta", _u32p), ("cap", ctypes.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        L.oracle_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.oracle_phases.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, _u32p]
        L.oracle_biphase.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, _u32p]
        L.oracle_line_terms.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int, ctypes.c_int,
                                        _dp, _dp, _dp, _lp]
        L.oracle_line_terms.restype = ctypes.c_int
        L.oracle_coefficients.argtypes = [ctypes.POINTER(_Problem), _u32p, ctypes.c_long,
                                          _lp, _dp]
        L.oracle_coefficients.restype = ctypes.c_int
        L.oracle_field_flat.argtypes = [ctypes.c_int] * 4 + [_dp, _dp]
        L.oracle_field_nested.argtypes = [ctypes.c_int] * 4 + [_dp, _dp]
        L.oracle_field_points.argtypes = [ctypes.c_int] * 4 + [_dp, ctypes.c_long, _ip, _ip, _dp]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_wind_solve.argtypes = [ctypes.POINTER(_Problem), _dp, ctypes.c_int, ctypes.c_double]
        L.oracle_wind_solve.restype = ctypes.c_int
        L.oracle_process_phases.argtypes = [ctypes.c_int, ctypes.c_uint64, _u32p]
        L.oracle_process_biphase.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, _u32p]
        L.oracle_process_terms.argtypes = [ctypes.POINTER(_Process), ctypes.c_int, _dp, _dp, _dp, _lp]
        L.oracle_process_terms.restype = ctypes.c_int
        L.oracle_process_coefficients.argtypes = [ctypes.POINTER(_Process), _u32p, _dp]
        L.oracle_process_coefficients.restype = ctypes.c_int
        L.oracle_process_field.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp]
        _lib = L
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(t)


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c, _u32p), _ptr(k, _u32p), _ptr(out, _u32p))
    return out


def phases(n_kappa: int, n_omega: int, seed: int) -> np.ndarray:
    U = np.zeros((n_kappa, 2 * n_omega - 1), dtype=np.uint32)
    lib().oracle_phases(n_kappa, n_omega, ctypes.c_uint64(int(seed)), _ptr(U, _u32p))
    return U


def biphase(support_w: int, seed: Optional[int]) -> np.ndarray:
    """Seeded biphase table; ``seed=None`` gives beta == 0."""
    n = 2 * support_w - 1
    B = np.zeros((n, n), dtype=np.uint32)
    mode = 1 if seed is None else 0
    lib().oracle_biphase(support_w, mode, ctypes.c_uint64(0 if seed is None else int(seed)),
                         _ptr(B, _u32p))
    return B


class Problem:
    """Inputs of one simulation (host FP64 arrays), kept alive for ctypes."""

    def __init__(self, n_kappa, n_omega, support_w, d_kappa, d_omega, S, b2, beta, cap,
                 line_c=None, line_r=None):
        self.S = np.ascontiguousarray(S, dtype=np.float64)
        self.b2 = np.ascontiguousarray(b2, dtype=np.float64)
        self.beta = np.ascontiguousarray(beta, dtype=np.uint32)
        nc, nwc = 2 * n_omega - 1, 2 * support_w - 1
        assert self.S.shape == (n_kappa, nc)
        assert self.b2.shape == (nwc, nwc) and self.beta.shape == (nwc, nwc)
        assert 1 <= support_w <= n_omega
        self.n_kappa, self.n_omega, self.W = n_kappa, n_omega, support_w
        self.d_kappa, self.d_omega, self.cap = d_kappa, d_omega, cap
        self.line_c = None if line_c is None else np.ascontiguousarray(line_c, dtype=np.float64)
        self.line_r = None if line_r is None else np.ascontiguousarray(line_r, dtype=np.float64)
        for a in (self.line_c, self.line_r):
            assert a is None or a.shape == (n_kappa, nc)
        self._c = _Problem(n_kappa, n_omega, support_w, d_kappa, d_omega,
                           _ptr(self.S, _dp), _ptr(self.b2, _dp), _ptr(self.beta, _u32p), cap,
                           None if self.line_c is None else _ptr(self.line_c, _dp),
                           None if self.line_r is None else _ptr(self.line_r, _dp), 0, 0.0, None)

    @classmethod
    def from_workload(cls, wl, beta_zero: bool = False, b2=None, beta=None, S=None,
                      cap=None):
        b2 = wl.b2_dense() if b2 is None else b2
        if beta is None:
            beta = biphase(wl.support_w, None if beta_zero else wl.beta_seed)
        return cls(wl.n_kappa, wl.n_omega, wl.support_w, wl.d_kappa, wl.d_omega,
                   wl.spectrum() if S is None else S, b2, beta,
                   wl.cap if cap is None else cap)

    @property
    def n_cols(self):
        return 2 * self.n_omega - 1

    def line_terms(self, kk: int, kw: int):
        sr, rho, sig = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        npairs = ctypes.c_long()
        st = lib().oracle_line_terms(ctypes.byref(self._c), kk, kw, ctypes.byref(sr),
                                     ctypes.byref(rho), ctypes.byref(sig), ctypes.byref(npairs))
        return dict(status=st, sigma_raw=sr.value, rho=rho.value, sigma=sig.value,
                    npairs=npairs.value)

    def coefficients(self, seed: Optional[int] = None, U: Optional[np.ndarray] = None,
                     lines: Optional[np.ndarray] = None) -> np.ndarray:
        """C_k (complex128) for all lines ([n_kappa][2nw-1]) or the given flat line ids."""
        if U is None:
            U = phases(self.n_kappa, self.n_omega, seed)
        U = np.ascontiguousarray(U, dtype=np.uint32)
        full = lines is None
        if full:
            lines = np.arange(self.n_kappa * self.n_cols, dtype=np.int64)
        lines = np.ascontiguousarray(lines, dtype=np.int64)
        out = np.zeros((lines.size, 2), dtype=np.float64)
        st = lib().oracle_coefficients(ctypes.byref(self._c), _ptr(U, _u32p), lines.size,
                                       lines.ctypes.data_as(_lp), _ptr(out, _dp))
        if st != 0:
            raise ValueError(f"oracle: pure spectrum not positive (status {st})")
        C = out[:, 0] + 1j * out[:, 1]
        return C.reshape(self.n_kappa, self.n_cols) if full else C


class WindProblem(Problem):
    """The wind bispectrum of Section 5 (scaled by alpha, beta = 0) through the
    partial-bicoherence recursion of Section 4.1; ``solve()`` finds S_p."""

    def __init__(self, n_kappa, n_omega, support_w, d_kappa, d_omega, S, alpha, cap):
        W = support_w
        super().__init__(n_kappa, n_omega, W, d_kappa, d_omega, S, np.zeros((2 * W - 1, 2 * W - 1)),
                         np.zeros((2 * W - 1, 2 * W - 1), dtype=np.uint32), cap)
        self.alpha = alpha
        self._c.alpha = alpha
        self.Sp = self.S.copy()
        self.sweeps = None

    def solve(self, max_iter: int = 500, tol: float = 1e-15) -> int:
        it = lib().oracle_wind_solve(ctypes.byref(self._c), _ptr(self.Sp, _dp), max_iter, tol)
        if it == -2:
            raise ValueError("oracle: no admissible pure spectrum (Sigma >= 1)")
        if it == -1:
            raise ValueError("oracle: the recursion did not converge")
        self.sweeps = it
        return it

    def _ensure(self):
        if self.sweeps is None:
            self.solve()

    def line_terms(self, kk: int, kw: int):
        self._ensure()
        return super().line_terms(kk, kw)

    def coefficients(self, *a, **kw):
        self._ensure()
        return super().coefficients(*a, **kw)

    def bispectrum(self, ik, iw, jk, jw) -> float:
        """|B| of the pair (Section 5, Eq. bispectrum, scaled), 0 where singular."""
        kk, kw = ik + jk, iw + jw
        if kk == 0 or kw == 0:
            return 0.0
        nw = self.n_omega
        Si, Sj, Sk = self.S[ik, iw + nw - 1], self.S[jk, jw + nw - 1], self.S[kk, kw + nw - 1]
        return self.alpha * 2.0 * math.sqrt(Si * Sj * Sk) / (
            3.0 * math.sqrt(3.0 * abs(kw * self.d_omega) * kk * self.d_kappa))


class ProductProblem(WindProblem):
    """A prescribed product bispectrum B(i, j) = F_k G_i G_j H(i_w, j_w)
    (complex; H may be None = 1) through the partial-bicoherence recursion of
    Section 4.1, with beta = atan2(Im B, Re B); ``solve()`` finds S_p."""

    def __init__(self, n_kappa, n_omega, support_w, d_kappa, d_omega, S, F, G, H, cap):
        super().__init__(n_kappa, n_omega, support_w, d_kappa, d_omega, S, 0.0, cap)
        nc, nwc = 2 * n_omega - 1, 2 * support_w - 1
        self.F = _cbuf(np.asarray(F).reshape(n_kappa, nc))
        self.G = _cbuf(np.asarray(G).reshape(n_kappa, nc))
        self.H = None if H is None else _cbuf(np.asarray(H).reshape(nwc, nwc))
        self._c.mode = 2
        self._c.F = _ptr(self.F, _dp)
        self._c.G = _ptr(self.G, _dp)
        self._c.H = None if self.H is None else _ptr(self.H, _dp)

    def bispectrum_c(self, ik, iw, jk, jw) -> complex:
        nw, W = self.n_omega, self.W
        F = self.F[ik + jk, iw + jw + nw - 1]
        G1, G2 = self.G[ik, iw + nw - 1], self.G[jk, jw + nw - 1]
        B = complex(F[0], F[1]) * complex(G1[0], G1[1]) * complex(G2[0], G2[1])
        if self.H is not None:
            h = self.H[iw + W - 1, jw + W - 1]
            B *= complex(h[0], h[1])
        return B


class HashedProblem(Problem):
    """A bispectrum drawn per 4-index pair: for the canonical member (i, j) of
    an unordered pair (k = i + j), with m = floor(i_w / 8) and t = i_w - 8 m,
    Philox4x32-10 (key ``key``, counter (i_kappa, m, j_kappa, k_w)) gives in
    word floor(t / 2) the 16-bit half h of the pair (high half for even t,
    low half for odd t); u = h >> 8, v = h & 255, b2_raw = scale (u / 2^8)^2
    and beta = 2 pi v / 2^8."""

    def __init__(self, n_kappa, n_omega, support_w, d_kappa, d_omega, S, scale, key, cap):
        W = support_w
        super().__init__(n_kappa, n_omega, W, d_kappa, d_omega, S, np.zeros((2 * W - 1, 2 * W - 1)),
                         np.zeros((2 * W - 1, 2 * W - 1), dtype=np.uint32), cap)
        self._c.mode = 3
        self._c.alpha = scale
        self._c.hash_key = int(key)


def _cbuf(C):
    C = np.ascontiguousarray(C, dtype=np.complex128)
    return np.ascontiguousarray(np.stack([C.real, C.imag], axis=-1))


def field(C: np.ndarray, n_x: int, n_t: int) -> np.ndarray:
    """Direct cosine sum over all lines at every grid point, [n_x][n_t]."""
    nk, nc = C.shape
    nw = (nc + 1) // 2
    buf = _cbuf(C)
    u = np.zeros((n_x, n_t), dtype=np.float64)
    lib().oracle_field_flat(nk, nw, n_x, n_t, _ptr(buf, _dp), _ptr(u, _dp))
    return u


def field_nested(C: np.ndarray, n_x: int, n_t: int) -> np.ndarray:
    nk, nc = C.shape
    nw = (nc + 1) // 2
    buf = _cbuf(C)
    u = np.zeros((n_x, n_t), dtype=np.float64)
    lib().oracle_field_nested(nk, nw, n_x, n_t, _ptr(buf, _dp), _ptr(u, _dp))
    return u


def field_points(C: np.ndarray, n_x: int, n_t: int, mx, mt) -> np.ndarray:
    nk, nc = C.shape
    nw = (nc + 1) // 2
    buf = _cbuf(C)
    mx = np.ascontiguousarray(mx, dtype=np.int32)
    mt = np.ascontiguousarray(mt, dtype=np.int32)
    u = np.zeros(mx.size, dtype=np.float64)
    lib().oracle_field_points(nk, nw, n_x, n_t, _ptr(buf, _dp), mx.size,
                              _ptr(mx, _ip), _ptr(mt, _ip), _ptr(u, _dp))
    return u


def num_threads() -> int:
    return int(lib().oracle_num_threads())


# ---- the 1-D stochastic process u(t) (Section 3) ----

def process_phases(n: int, seed: int) -> np.ndarray:
    U = np.zeros(n, dtype=np.uint32)
    lib().oracle_process_phases(n, ctypes.c_uint64(int(seed)), _ptr(U, _u32p))
    return U


def process_biphase(support_w: int, seed: Optional[int]) -> np.ndarray:
    """Biphase over 0 <= i, j < W; ``seed=None`` gives beta == 0."""
    B = np.zeros((support_w, support_w), dtype=np.uint32)
    lib().oracle_process_biphase(support_w, 1 if seed is None else 0,
                                 ctypes.c_uint64(0 if seed is None else int(seed)), _ptr(B, _u32p))
    return B


class ProcessProblem:
    """Inputs of one process simulation: n one-sided frequencies, support W,
    b2 and beta over 0 <= i, j < W."""

    def __init__(self, n, support_w, d_omega, S, b2, beta, cap):
        self.S = np.ascontiguousarray(S, dtype=np.float64)
        self.b2 = np.ascontiguousarray(b2, dtype=np.float64)
        self.beta = np.ascontiguousarray(beta, dtype=np.uint32)
        assert self.S.shape == (n,) and 1 <= support_w <= n
        assert self.b2.shape == (support_w, support_w) and self.beta.shape == (support_w, support_w)
        self.n, self.W, self.d_omega, self.cap = n, support_w, d_omega, cap
        self._c = _Process(n, support_w, d_omega, _ptr(self.S, _dp), _ptr(self.b2, _dp),
                           _ptr(self.beta, _u32p), cap)

    def terms(self, k: int):
        sr, rho, sig = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        npairs = ctypes.c_long()
        st = lib().oracle_process_terms(ctypes.byref(self._c), k, ctypes.byref(sr), ctypes.byref(rho),
                                        ctypes.byref(sig), ctypes.byref(npairs))
        return dict(status=st, sigma_raw=sr.value, rho=rho.value, sigma=sig.value, npairs=npairs.value)

    def coefficients(self, seed: Optional[int] = None, U: Optional[np.ndarray] = None) -> np.ndarray:
        if U is None:
            U = process_phases(self.n, seed)
        U = np.ascontiguousarray(U, dtype=np.uint32)
        out = np.zeros((self.n, 2), dtype=np.float64)
        st = lib().oracle_process_coefficients(ctypes.byref(self._c), _ptr(U, _u32p), _ptr(out, _dp))
        if st != 0:
            raise ValueError(f"oracle: pure spectrum not positive (status {st})")
        return out[:, 0] + 1j * out[:, 1]


def process_field(C: np.ndarray, n_t: int) -> np.ndarray:
    """u(t_m) = sum_k Re[C_k exp(2 pi i k m / n_t)], direct cosine sum, [n_t]."""
    buf = _cbuf(C)
    u = np.zeros(n_t, dtype=np.float64)
    lib().oracle_process_field(C.size, n_t, _ptr(buf, _dp), _ptr(u, _dp))
    return u
