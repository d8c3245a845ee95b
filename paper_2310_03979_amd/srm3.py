"""Python binding of ``libsrm3.so`` (argument marshalling only).

Every step of the generator runs in the HIP library; PyTorch supplies device
memory (tensors) and the current HIP stream.  Function names mirror the C-ABI
declared in ``include/srm3.h``.  If the library is not built this module
raises on first use -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsrm3.so")

SRM3_FP64, SRM3_FP32 = 0, 1
SRM3_BISPEC_NONE, SRM3_BISPEC_SEPARABLE, SRM3_BISPEC_DENSE = 0, 1, 2
SRM3_BETA_SEEDED, SRM3_BETA_ZERO, SRM3_BETA_TABLE = 0, 1, 2
STATUS = {0: "SRM3_OK", 1: "SRM3_E_INVALID", 2: "SRM3_E_PURE_NEGATIVE", 3: "SRM3_E_NOMEM",
          4: "SRM3_E_DEVICE", 5: "SRM3_E_UNSUPPORTED"}
KERNELS = ("phases", "pairsum", "tfft", "xfft")

_dp = ctypes.POINTER(ctypes.c_double)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


class Srm3Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Grid(ctypes.Structure):
    _fields_ = [("n_kappa", ctypes.c_int32), ("n_omega", ctypes.c_int32),
                ("d_kappa", ctypes.c_double), ("d_omega", ctypes.c_double),
                ("n_x", ctypes.c_int32), ("n_t", ctypes.c_int32)]


class _Spectrum(ctypes.Structure):
    _fields_ = [("S", _dp)]


class _Bispectrum(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("g2", _dp), ("b2", _dp), ("beta", _u32p),
                ("support_w", ctypes.c_int32), ("cap", ctypes.c_double),
                ("beta_mode", ctypes.c_int32), ("beta_seed", ctypes.c_uint64),
                ("line_c", _dp), ("line_r", _dp), ("alpha", ctypes.c_double),
                ("prod_f", _dp), ("prod_g", _dp), ("prod_h", _dp)]


class _ProcessGrid(ctypes.Structure):
    _fields_ = [("n_omega", ctypes.c_int32), ("d_omega", ctypes.c_double), ("n_t", ctypes.c_int32)]


class _Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 4), ("launches", ctypes.c_int64 * 4)]


class _KaimalDavenport(ctypes.Structure):
    _fields_ = [("u_star", ctypes.c_double), ("z", ctypes.c_double), ("U", ctypes.c_double),
                ("lam", ctypes.c_double)]


class _Request(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("seed", ctypes.c_uint64), ("b2_scale", ctypes.c_double),
                ("S_dev", ctypes.c_void_p), ("out_dev", ctypes.c_void_p)]


class _BatchStats(ctypes.Structure):
    _fields_ = [("pair_terms", ctypes.c_double), ("run_ms", ctypes.c_double),
                ("pairsum_ms", ctypes.c_double), ("rows_per_wave", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("work_items", ctypes.c_int32),
                ("groups", ctypes.c_int32), ("mfma_shape", ctypes.c_int32)]


SRM3_BATCH_GRAPH, SRM3_BATCH_AUTOTUNE = 1, 2


_lib = None


def load():
    """Load libsrm3.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libsrm3.so not found at {LIB_PATH}; build it with "
                          "`python -m paper_2310_03979_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.srm3_plan.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Spectrum),
                            ctypes.POINTER(_Bispectrum), ctypes.c_int32, vp, ctypes.POINTER(vp)]
    L.srm3_generate.argtypes = [vp, _u64p, ctypes.c_int32, vp, vp]
    L.srm3_coefficients.argtypes = [vp, _u64p, ctypes.c_int32, vp, vp]
    L.srm3_generate_noalloc.argtypes = [vp, _u64p, ctypes.c_int32, vp, vp]
    L.srm3_transform.argtypes = [vp, vp, ctypes.c_int32, vp, vp]
    L.srm3_workspace_bytes.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
    L.srm3_workspace_fill.argtypes = [vp, ctypes.c_int32, ctypes.c_uint32, vp]
    L.srm3_pair_terms.argtypes = [vp, _dp]
    L.srm3_rows_per_wave.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.srm3_plan_set_algorithm.argtypes = [vp, ctypes.c_int32, vp]
    L.srm3_wind_factors.argtypes = [ctypes.POINTER(_Grid), _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                    _dp, _dp, _dp, ctypes.POINTER(ctypes.c_int32)]
    L.srm3_product_factors.argtypes = [ctypes.POINTER(_Grid), _dp, _dp, _dp, _dp, ctypes.c_int32, ctypes.c_double,
                                       _dp, _dp, _dp, ctypes.POINTER(ctypes.c_int32)]
    L.srm3_process_plan.argtypes = [ctypes.POINTER(_ProcessGrid), _dp, ctypes.POINTER(_Bispectrum),
                                    ctypes.c_int32, vp, ctypes.POINTER(vp)]
    L.srm3_algorithm_terms.argtypes = [vp, _dp]
    L.srm3_plan_set_mfma_shape.argtypes = [vp, ctypes.c_int32]
    L.srm3_mfma_shape.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32)]
    L.srm3_profile_enable.argtypes = [vp, ctypes.c_int32]
    L.srm3_profile_read.argtypes = [vp, ctypes.POINTER(_Profile)]
    L.srm3_destroy.argtypes = [vp]
    L.srm3_destroy.restype = None
    L.srm3_last_error.restype = ctypes.c_char_p
    L.srm3_set_spectrum.argtypes = [vp, ctypes.POINTER(_Spectrum), vp]
    L.srm3_spectrum_kaimal_davenport.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_KaimalDavenport),
                                                 vp, vp]
    L.srm3_batch_create.argtypes = [ctypes.POINTER(_Request), ctypes.c_int32, ctypes.c_int32, vp,
                                    ctypes.POINTER(vp)]
    L.srm3_batch_run.argtypes = [vp, _u64p, vp]
    L.srm3_batch_info.argtypes = [vp, ctypes.POINTER(_BatchStats)]
    L.srm3_batch_destroy.argtypes = [vp]
    L.srm3_batch_destroy.restype = None
    L.srm3_generate_uneven.argtypes = [ctypes.POINTER(_Request), ctypes.c_int32, vp]
    for f in ("srm3_plan", "srm3_process_plan", "srm3_wind_factors", "srm3_product_factors", "srm3_generate", "srm3_generate_noalloc", "srm3_coefficients", "srm3_transform",
              "srm3_workspace_bytes", "srm3_workspace_fill", "srm3_pair_terms", "srm3_rows_per_wave", "srm3_plan_set_algorithm",
              "srm3_algorithm_terms", "srm3_plan_set_mfma_shape", "srm3_mfma_shape", "srm3_profile_enable",
              "srm3_profile_read", "srm3_set_spectrum", "srm3_spectrum_kaimal_davenport",
              "srm3_batch_create", "srm3_batch_run", "srm3_batch_info", "srm3_generate_uneven"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def srm3_last_error() -> str:
    return load().srm3_last_error().decode()


def _check(status: int):
    if status != 0:
        raise Srm3Error(status, srm3_last_error())


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        if not torch.cuda.is_available():
            return None
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Plan:
    """Owner of a ``srm3_plan_t`` handle plus the sizes needed to check tensors."""

    def __init__(self, handle, grid: dict, precision: int, support_w: int):
        self._h = handle
        self.grid = dict(grid)
        self.precision = precision
        self.support_w = support_w
        self.process = False

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("plan destroyed")
        return self._h

    @property
    def field_shape(self):
        return (self.grid["n_x"], self.grid["n_t"])

    @property
    def coeff_shape(self):
        return (self.grid["n_kappa"], 2 * self.grid["n_omega"] - 1)

    @property
    def real_dtype(self):
        import torch
        return torch.float64 if self.precision == SRM3_FP64 else torch.float32

    def __del__(self):
        try:
            if self._h is not None and _lib is not None:
                _lib.srm3_destroy(self._h)
                self._h = None
        except Exception:
            pass


def _precision(p) -> int:
    if isinstance(p, str):
        return {"fp64": SRM3_FP64, "f64": SRM3_FP64, "fp32": SRM3_FP32, "f32": SRM3_FP32}[p.lower()]
    return int(p)


def _bispectrum(bispectrum: Optional[dict], default_w: int):
    """Marshal a bispectrum dict into the C struct; returns (struct or None, arrays to keep alive, W)."""
    if bispectrum is None:
        return None, [], 1
    kinds = {"none": 0, "separable": 1, "dense": 2, "wind": 3, "product": 4, "hashed": 5}
    modes = {"seeded": 0, "zero": 1, "table": 2}
    kind = bispectrum.get("kind", "separable")
    kind = kinds[kind] if isinstance(kind, str) else int(kind)
    mode = bispectrum.get("beta_mode", "seeded")
    mode = modes[mode] if isinstance(mode, str) else int(mode)
    W = int(bispectrum.get("support_w", default_w))
    b = _Bispectrum()
    b.kind = kind
    b.support_w = W
    b.cap = float(bispectrum.get("cap", 0.9))
    b.beta_mode = mode
    b.beta_seed = int(bispectrum.get("beta_seed", 0))
    keep = []
    if bispectrum.get("g2") is not None:
        g2 = np.ascontiguousarray(bispectrum["g2"], dtype=np.float64)
        keep.append(g2)
        b.g2 = g2.ctypes.data_as(_dp)
    if bispectrum.get("b2") is not None:
        b2 = np.ascontiguousarray(bispectrum["b2"], dtype=np.float64)
        keep.append(b2)
        b.b2 = b2.ctypes.data_as(_dp)
    if bispectrum.get("beta") is not None:
        bt = np.ascontiguousarray(bispectrum["beta"], dtype=np.uint32)
        keep.append(bt)
        b.beta = bt.ctypes.data_as(_u32p)
    for name in ("line_c", "line_r"):
        if bispectrum.get(name) is not None:
            f = np.ascontiguousarray(bispectrum[name], dtype=np.float64)
            keep.append(f)
            setattr(b, name, f.ctypes.data_as(_dp))
    b.alpha = float(bispectrum.get("alpha", 0.0))
    for key, field in (("F", "prod_f"), ("G", "prod_g"), ("H", "prod_h")):
        if bispectrum.get(key) is not None:
            f = _complex_buf(bispectrum[key])
            keep.append(f)
            setattr(b, field, f.ctypes.data_as(_dp))
    return b, keep, W


def _complex_buf(a) -> np.ndarray:
    """Complex array -> contiguous interleaved (re, im) float64."""
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return np.ascontiguousarray(np.stack([a.real, a.imag], axis=-1))


def srm3_plan(grid: dict, S: np.ndarray, bispectrum: Optional[dict] = None, precision="fp64",
              stream=None) -> Plan:
    """Build a plan.  ``grid``: n_kappa, n_omega, d_kappa, d_omega, n_x, n_t.

    ``bispectrum`` keys: kind ('none' | 'separable' | 'dense'), g2, b2, beta (uint32
    table), support_w, cap, beta_mode ('seeded' | 'zero' | 'table'), beta_seed.
    """
    L = load()
    g = _Grid(int(grid["n_kappa"]), int(grid["n_omega"]), float(grid["d_kappa"]),
              float(grid["d_omega"]), int(grid["n_x"]), int(grid["n_t"]))
    S = np.ascontiguousarray(S, dtype=np.float64)
    spec = _Spectrum(S.ctypes.data_as(_dp))
    b, keep, W = _bispectrum(bispectrum, int(grid["n_omega"]))
    keep.append(S)
    bp = ctypes.byref(b) if b is not None else None
    h = ctypes.c_void_p()
    _check(L.srm3_plan(ctypes.byref(g), ctypes.byref(spec), bp, _precision(precision),
                       _stream_ptr(stream), ctypes.byref(h)))
    del keep
    return Plan(h, grid, _precision(precision), W)


def _seeds(seeds) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64).reshape(-1))


def _check_tensor(t, dtype, numel, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} dtype {t.dtype} != {dtype}")
    if not t.is_contiguous() or t.numel() < numel:
        raise ValueError(f"{what} must be contiguous with >= {numel} elements")


def srm3_generate(plan: Plan, seeds: Sequence[int], out, stream=None):
    """Write ``len(seeds)`` fields into ``out`` ([B][n_x][n_t], plan precision)."""
    s = _seeds(seeds)
    nx, nt = plan.field_shape
    _check_tensor(out, plan.real_dtype, s.size * nx * nt, "out")
    _check(load().srm3_generate(plan.handle, s.ctypes.data_as(_u64p), s.size,
                                ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def srm3_generate_noalloc(plan: Plan, seeds: Sequence[int], out, stream=None):
    """srm3_generate with the workspace in the library's fixed scratch array
    (no device allocation; calls on one GPU must not overlap)."""
    s = _seeds(seeds)
    nx, nt = plan.field_shape
    _check_tensor(out, plan.real_dtype, s.size * nx * nt, "out")
    _check(load().srm3_generate_noalloc(plan.handle, s.ctypes.data_as(_u64p), s.size,
                                        ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def srm3_coefficients(plan: Plan, seeds: Sequence[int], C_out, stream=None):
    """Coefficients C_k ([B][n_kappa][2 n_omega - 1] complex) into ``C_out``."""
    import torch
    s = _seeds(seeds)
    nk, nc = plan.coeff_shape
    cdt = torch.complex128 if plan.precision == SRM3_FP64 else torch.complex64
    _check_tensor(C_out, cdt, s.size * nk * nc, "C_out")
    _check(load().srm3_coefficients(plan.handle, s.ctypes.data_as(_u64p), s.size,
                                    ctypes.c_void_p(C_out.data_ptr()), _stream_ptr(stream)))
    return C_out


def srm3_transform(plan: Plan, C, out, batch: Optional[int] = None, stream=None):
    import torch
    nk, nc = plan.coeff_shape
    nx, nt = plan.field_shape
    B = C.numel() // (nk * nc) if batch is None else batch
    cdt = torch.complex128 if plan.precision == SRM3_FP64 else torch.complex64
    _check_tensor(C, cdt, B * nk * nc, "C")
    _check_tensor(out, plan.real_dtype, B * nx * nt, "out")
    _check(load().srm3_transform(plan.handle, ctypes.c_void_p(C.data_ptr()), B,
                                 ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def srm3_workspace_bytes(plan: Plan, batch: int) -> int:
    n = ctypes.c_size_t()
    _check(load().srm3_workspace_bytes(plan.handle, batch, ctypes.byref(n)))
    return int(n.value)


def srm3_workspace_fill(plan: Plan, batch: int, word: int, stream=None):
    """Fill the plan's workspace for ``batch`` realizations with a 32-bit pattern
    (e.g. 0x7FC00000, a NaN) by a kernel on the stream."""
    _check(load().srm3_workspace_fill(plan.handle, int(batch), ctypes.c_uint32(int(word) & 0xFFFFFFFF),
                                      _stream_ptr(stream)))


def srm3_pair_terms(plan: Plan) -> float:
    v = ctypes.c_double()
    _check(load().srm3_pair_terms(plan.handle, ctypes.byref(v)))
    return float(v.value)


SRM3_ALGO_DIRECT, SRM3_ALGO_KAPPA_FFT, SRM3_ALGO_FFT2D, SRM3_ALGO_MFMA = 0, 1, 2, 3
_ALGOS = {"direct": SRM3_ALGO_DIRECT, "kappa_fft": SRM3_ALGO_KAPPA_FFT, "fft2d": SRM3_ALGO_FFT2D,
          "mfma": SRM3_ALGO_MFMA}


def srm3_plan_set_algorithm(plan: Plan, algorithm="direct", stream=None):
    """Pair-sum algorithm of the plan: "direct", "kappa_fft", "fft2d" or "mfma" (or the enum)."""
    a = _ALGOS[algorithm] if isinstance(algorithm, str) else int(algorithm)
    _check(load().srm3_plan_set_algorithm(plan.handle, a, _stream_ptr(stream)))


def srm3_plan_set_mfma_shape(plan: Plan, shape: int):
    """Tile shape (0, 1, 2) of the plan's matrix-core pair sum."""
    _check(load().srm3_plan_set_mfma_shape(plan.handle, int(shape)))


def srm3_mfma_shape(precision, shape: int):
    """(rows, cols) of outputs a wave owns under a matrix-core tile shape."""
    r, c = ctypes.c_int32(), ctypes.c_int32()
    _check(load().srm3_mfma_shape(_precision(precision), int(shape), ctypes.byref(r), ctypes.byref(c)))
    return int(r.value), int(c.value)


def srm3_algorithm_terms(plan: Plan) -> float:
    v = ctypes.c_double()
    _check(load().srm3_algorithm_terms(plan.handle, ctypes.byref(v)))
    return float(v.value)


def srm3_rows_per_wave(plan: Plan) -> int:
    v = ctypes.c_int32()
    _check(load().srm3_rows_per_wave(plan.handle, ctypes.byref(v)))
    return int(v.value)


def srm3_profile_enable(plan: Plan, enable: bool = True):
    _check(load().srm3_profile_enable(plan.handle, 1 if enable else 0))


def srm3_profile_read(plan: Plan) -> dict:
    p = _Profile()
    _check(load().srm3_profile_read(plan.handle, ctypes.byref(p)))
    return {k: (p.ms[i], int(p.launches[i])) for i, k in enumerate(KERNELS)}


def srm3_destroy(plan: Plan):
    if plan._h is not None:
        load().srm3_destroy(plan._h)
        plan._h = None


def plan_from_workload(wl, precision="fp64", beta_mode="seeded", stream=None, dense=False,
                       **overrides) -> Plan:
    """Convenience: plan for a ``srm3_inputs.Workload`` (separable bicoherence)."""
    bis = dict(kind="dense" if dense else "separable", support_w=wl.support_w, cap=wl.cap,
               beta_mode=beta_mode, beta_seed=wl.beta_seed)
    if dense:
        bis["b2"] = wl.b2_dense()
    else:
        bis["g2"] = wl.g2()
    bis.update(overrides)
    return srm3_plan(wl.grid_dict(), wl.spectrum(), bis, precision, stream)


def srm3_process_plan(grid: dict, S: np.ndarray, bispectrum: Optional[dict] = None, precision="fp64",
                      stream=None) -> Plan:
    """Plan for the 1-D process u(t): grid = dict(n_omega, d_omega, n_t), S one-sided
    [n_omega], bispectrum tables over 0 <= i, j < support_w.  Fields are [B][1][n_t]."""
    L = load()
    g = _ProcessGrid(int(grid["n_omega"]), float(grid["d_omega"]), int(grid["n_t"]))
    S = np.ascontiguousarray(S, dtype=np.float64)
    b, keep, W = _bispectrum(bispectrum, int(grid["n_omega"]))
    keep.append(S)
    h = ctypes.c_void_p()
    _check(L.srm3_process_plan(ctypes.byref(g), S.ctypes.data_as(_dp),
                               ctypes.byref(b) if b is not None else None, _precision(precision),
                               _stream_ptr(stream), ctypes.byref(h)))
    del keep
    wave_grid = dict(n_kappa=1, n_omega=int(grid["n_omega"]), d_kappa=1.0, d_omega=float(grid["d_omega"]),
                     n_x=1, n_t=int(grid["n_t"]))
    p = Plan(h, wave_grid, _precision(precision), W)
    p.process = True
    return p


def srm3_wind_factors(grid: dict, S: np.ndarray, alpha: float, cap: float = 0.0, support_w: Optional[int] = None):
    """Line factors (c, r), Sigma and sweep count of the wind bispectrum
    (host computation; no GPU needed)."""
    L = load()
    g = _Grid(int(grid["n_kappa"]), int(grid["n_omega"]), float(grid["d_kappa"]),
              float(grid["d_omega"]), int(grid.get("n_x", 1)), int(grid.get("n_t", 1)))
    S = np.ascontiguousarray(S, dtype=np.float64)
    c, r, sig = np.zeros_like(S), np.zeros_like(S), np.zeros_like(S)
    it = ctypes.c_int32()
    W = int(grid["n_omega"]) if support_w is None else int(support_w)
    _check(L.srm3_wind_factors(ctypes.byref(g), S.ctypes.data_as(_dp), float(alpha), float(cap), W,
                               c.ctypes.data_as(_dp), r.ctypes.data_as(_dp), sig.ctypes.data_as(_dp),
                               ctypes.byref(it)))
    return c, r, sig, int(it.value)


def srm3_product_factors(grid: dict, S: np.ndarray, F, G, H=None, support_w: Optional[int] = None,
                         cap: float = 0.0):
    """Complex line factors (c, rho), Sigma and sweep count of a prescribed
    product bispectrum (host computation; no GPU needed)."""
    L = load()
    g = _Grid(int(grid["n_kappa"]), int(grid["n_omega"]), float(grid["d_kappa"]),
              float(grid["d_omega"]), int(grid.get("n_x", 1)), int(grid.get("n_t", 1)))
    S = np.ascontiguousarray(S, dtype=np.float64)
    Fb, Gb = _complex_buf(F), _complex_buf(G)
    Hb = None if H is None else _complex_buf(H)
    c = np.zeros(S.shape + (2,))
    rho = np.zeros(S.shape + (2,))
    sig = np.zeros_like(S)
    it = ctypes.c_int32()
    W = int(grid["n_omega"]) if support_w is None else int(support_w)
    _check(L.srm3_product_factors(ctypes.byref(g), S.ctypes.data_as(_dp), Fb.ctypes.data_as(_dp),
                                  Gb.ctypes.data_as(_dp), None if Hb is None else Hb.ctypes.data_as(_dp), W,
                                  float(cap), c.ctypes.data_as(_dp), rho.ctypes.data_as(_dp),
                                  sig.ctypes.data_as(_dp), ctypes.byref(it)))
    return c[..., 0] + 1j * c[..., 1], rho[..., 0] + 1j * rho[..., 1], sig, int(it.value)


def process_plan_from_workload(wl, precision="fp64", beta_mode="seeded", stream=None, dense=False,
                               **overrides) -> Plan:
    """Convenience: plan for a ``srm3_inputs.ProcessWorkload`` (separable bicoherence)."""
    bis = dict(kind="dense" if dense else "separable", support_w=wl.support_w, cap=wl.cap,
               beta_mode=beta_mode, beta_seed=wl.beta_seed)
    if dense:
        bis["b2"] = wl.b2_dense()
    else:
        bis["g2"] = wl.g2()
    bis.update(overrides)
    return srm3_process_plan(wl.grid_dict(), wl.spectrum(), bis, precision, stream)


def srm3_set_spectrum(plan: Plan, S: np.ndarray, stream=None):
    S = np.ascontiguousarray(S, dtype=np.float64)
    want = (plan.grid["n_omega"],) if plan.process else plan.coeff_shape
    if S.shape != want:
        raise ValueError(f"S shape {S.shape} != {want}")
    spec = _Spectrum(S.ctypes.data_as(_dp))
    _check(load().srm3_set_spectrum(plan.handle, ctypes.byref(spec), _stream_ptr(stream)))


def srm3_spectrum_kaimal_davenport(grid: dict, S_out, u_star=1.5, z=50.0, U=30.0, lam=10.0,
                                   stream=None):
    """Evaluate the wind-field spectrum on the line grid into the device tensor S_out (float64)."""
    import torch
    nk, nc = int(grid["n_kappa"]), 2 * int(grid["n_omega"]) - 1
    _check_tensor(S_out, torch.float64, nk * nc, "S_out")
    g = _Grid(nk, int(grid["n_omega"]), float(grid["d_kappa"]), float(grid["d_omega"]),
              int(grid.get("n_x", 1)), int(grid.get("n_t", 1)))
    p = _KaimalDavenport(u_star, z, U, lam)
    _check(load().srm3_spectrum_kaimal_davenport(ctypes.byref(g), ctypes.byref(p),
                                                 ctypes.c_void_p(S_out.data_ptr()), _stream_ptr(stream)))
    return S_out


def _requests(reqs):
    """reqs: sequence of dicts with plan, seed, out, optional b2_scale, S (device tensor)."""
    arr = (_Request * len(reqs))()
    for i, r in enumerate(reqs):
        plan, out = r["plan"], r["out"]
        nx, nt = plan.field_shape
        _check_tensor(out, plan.real_dtype, nx * nt, f"request {i} out")
        S = r.get("S")
        if S is not None:
            import torch
            _check_tensor(S, torch.float64, plan.coeff_shape[0] * plan.coeff_shape[1], f"request {i} S")
        arr[i] = _Request(plan.handle, int(r["seed"]), float(r.get("b2_scale", 1.0)),
                          None if S is None else S.data_ptr(), out.data_ptr())
    return arr


class Batch:
    """An uneven batch (srm3_batch_t); keeps the request tensors alive."""

    def __init__(self, reqs, flags=0, stream=None):
        self._reqs = list(reqs)
        arr = _requests(self._reqs)
        h = ctypes.c_void_p()
        _check(load().srm3_batch_create(arr, len(arr), int(flags), _stream_ptr(stream), ctypes.byref(h)))
        self._h = h

    def run(self, seeds=None, stream=None):
        if seeds is None:
            _check(load().srm3_batch_run(self._h, None, _stream_ptr(stream)))
        else:
            s = _seeds(seeds)
            if s.size != len(self._reqs):
                raise ValueError("one seed per request")
            _check(load().srm3_batch_run(self._h, s.ctypes.data_as(_u64p), _stream_ptr(stream)))

    def info(self) -> dict:
        st = _BatchStats()
        _check(load().srm3_batch_info(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _BatchStats._fields_}

    def destroy(self):
        if self._h is not None and _lib is not None:
            _lib.srm3_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def srm3_batch_create(reqs, flags=0, stream=None) -> Batch:
    return Batch(reqs, flags, stream)


def srm3_batch_run(batch: Batch, seeds=None, stream=None):
    batch.run(seeds, stream)


def srm3_batch_info(batch: Batch) -> dict:
    return batch.info()


def srm3_batch_destroy(batch: Batch):
    batch.destroy()


def srm3_generate_uneven(reqs, stream=None):
    arr = _requests(reqs)
    _check(load().srm3_generate_uneven(arr, len(arr), _stream_ptr(stream)))


# ---------------------------------------------------------------------------
# request server
# ---------------------------------------------------------------------------
class _ServerConfig(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_active", ctypes.c_int32),
                ("hbm_budget", ctypes.c_size_t), ("step_pair_terms", ctypes.c_double),
                ("policy", ctypes.c_int32), ("pair_kernel", ctypes.c_int32), ("mfma_shape", ctypes.c_int32)]


SRM3_SERVE_SHORTEST_FIRST, SRM3_SERVE_ROUND_ROBIN = 0, 1


class _ServerState(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int32), ("active", ctypes.c_int32), ("finishing", ctypes.c_int32),
                ("completed", ctypes.c_int32), ("launched", ctypes.c_int32), ("steps", ctypes.c_int64)]


def _server_lib():
    L = load()
    if not getattr(L, "_srv_ready", False):
        vp = ctypes.c_void_p
        L.srm3_server_create.argtypes = [ctypes.POINTER(_ServerConfig), vp, ctypes.POINTER(vp)]
        L.srm3_server_submit.argtypes = [vp, ctypes.POINTER(_Request), ctypes.POINTER(_KaimalDavenport),
                                         ctypes.POINTER(ctypes.c_int64)]
        L.srm3_server_step.argtypes = [vp, ctypes.POINTER(_ServerState)]
        L.srm3_server_poll.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32)]
        L.srm3_server_destroy.argtypes = [vp]
        L.srm3_server_destroy.restype = None
        for f in ("srm3_server_create", "srm3_server_submit", "srm3_server_step", "srm3_server_poll"):
            getattr(L, f).restype = ctypes.c_int
        L._srv_ready = True
    return L


class Server:
    """srm3_server_t: continuous batching of generation requests."""

    def __init__(self, precision="fp32", max_active=64, hbm_budget=32 << 30, step_pair_terms=0.0,
                 policy="shortest", stream=None, pair_kernel="direct", mfma_shape=0):
        L = _server_lib()
        pol = {"shortest": SRM3_SERVE_SHORTEST_FIRST, "round_robin": SRM3_SERVE_ROUND_ROBIN}[policy]
        pk = _ALGOS[pair_kernel] if isinstance(pair_kernel, str) else int(pair_kernel)
        cfg = _ServerConfig(_precision(precision), int(max_active), int(hbm_budget), float(step_pair_terms), pol, pk,
                            int(mfma_shape))
        h = ctypes.c_void_p()
        _check(L.srm3_server_create(ctypes.byref(cfg), _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        self._keep = {}
        self._buf = (ctypes.c_int64 * 1024)()

    def submit(self, plan: Plan, seed: int, out, b2_scale: float = 1.0, S=None, spectrum=None) -> int:
        arr = _requests([dict(plan=plan, seed=seed, out=out, b2_scale=b2_scale, S=S)])
        sp = None
        if spectrum is not None:
            sp = ctypes.byref(_KaimalDavenport(float(spectrum.get("u_star", 1.5)), float(spectrum.get("z", 50.0)),
                                               float(spectrum["U"]), float(spectrum.get("lam", 10.0))))
        t = ctypes.c_int64()
        _check(_server_lib().srm3_server_submit(self._h, arr, sp, ctypes.byref(t)))
        self._keep[t.value] = (out, S)
        return t.value

    def step(self) -> dict:
        st = _ServerState()
        _check(_server_lib().srm3_server_step(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _ServerState._fields_}

    def poll(self):
        n = ctypes.c_int32()
        _check(_server_lib().srm3_server_poll(self._h, self._buf, len(self._buf), ctypes.byref(n)))
        done = [int(self._buf[i]) for i in range(n.value)]
        for t in done:
            self._keep.pop(t, None)
        return done

    def destroy(self):
        if self._h is not None and _lib is not None:
            _lib.srm3_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
