"""GPU path vs the FP64 oracle, element by element, through the C-ABI.

Tolerances (relative L2 per realization, max over the batch):
FP64 path <= 1e-10, FP32 fixed-point-phase path <= 2e-5.
"""
import math

import numpy as np
import pytest

import srm3_inputs as inp

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 2e-5}


@pytest.fixture(scope="module")
def lib():
    import torch
    import paper_2310_03979_amd as p
    p.load()
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    return p


def _torch():
    import torch
    return torch


def _rel_l2(a, b):
    a = np.asarray(a).reshape(a.shape[0], -1) if np.ndim(a) > 1 else np.asarray(a)[None]
    b = np.asarray(b).reshape(b.shape[0], -1) if np.ndim(b) > 1 else np.asarray(b)[None]
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))


def _bispec(wl, kind, beta_mode, seed=5):
    b = dict(kind=kind, support_w=wl.support_w, cap=wl.cap, beta_mode=beta_mode,
             beta_seed=wl.beta_seed)
    if kind == "separable":
        b["g2"] = wl.g2()
        b2 = wl.b2_dense()
    else:
        b2 = inp.random_b2_dense(wl.support_w, seed, scale=0.3)
        b["b2"] = b2
    if beta_mode == "table":
        b["beta"] = inp.random_beta_table(wl.support_w, seed + 1)
    return b, b2


def _oracle_problem(oracle_mod, wl, bis, b2):
    if bis.get("beta_mode") == "table":
        beta = bis["beta"]
    elif bis.get("beta_mode") == "zero":
        beta = oracle_mod.biphase(wl.support_w, None)
    else:
        beta = oracle_mod.biphase(wl.support_w, wl.beta_seed)
    return oracle_mod.Problem(wl.n_kappa, wl.n_omega, wl.support_w, wl.d_kappa, wl.d_omega,
                              wl.spectrum(), b2, beta, bis["cap"])


def _gpu_field(lib, wl, bis, precision, seeds):
    torch = _torch()
    print(f"[gpu] {wl.name} {precision} B={len(seeds)}", flush=True)
    plan = lib.srm3_plan(wl.grid_dict(), wl.spectrum(), bis, precision)
    out = torch.empty((len(seeds), wl.n_x, wl.n_t), dtype=plan.real_dtype, device="cuda")
    lib.srm3_generate(plan, seeds, out)
    torch.cuda.synchronize()
    return plan, out.double().cpu().numpy()


def _gpu_coeffs(lib, plan, seeds):
    torch = _torch()
    cdt = torch.complex128 if plan.precision == lib.SRM3_FP64 else torch.complex64
    C = torch.empty((len(seeds),) + plan.coeff_shape, dtype=cdt, device="cuda")
    lib.srm3_coefficients(plan, seeds, C)
    torch.cuda.synchronize()
    return C


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c0_field_matches_oracle(lib, oracle_mod, precision):
    wl = inp.C0
    bis, b2 = _bispec(wl, "separable", "seeded")
    plan, u = _gpu_field(lib, wl, bis, precision, wl.seeds())
    P = _oracle_problem(oracle_mod, wl, bis, b2)
    ref = oracle_mod.field(P.coefficients(seed=int(wl.seeds()[0])), wl.n_x, wl.n_t)
    assert _rel_l2(u[0], ref) <= TOL[precision]
    C = _gpu_coeffs(lib, plan, wl.seeds()).cpu().numpy()[0]
    Cref = P.coefficients(seed=int(wl.seeds()[0]))
    assert np.linalg.norm(C - Cref) / np.linalg.norm(Cref) <= TOL[precision]


SMALL = [
    # nk, nw, W, nx, nt, kind, beta_mode
    (5, 40, 40, 8, 128, "dense", "table"),      # two column tiles, ragged rows
    (24, 70, 33, 32, 256, "dense", "seeded"),   # truncated support, ragged columns
    (17, 9, 9, 32, 32, "separable", "zero"),    # non power-of-two rows, beta == 0
    (1, 8, 8, 1, 16, "separable", "seeded"),    # a single kappa row
    (3, 5, 1, 4, 16, "dense", "seeded"),        # support of one frequency (omega = 0)
    (2, 1, 1, 2, 1, "separable", "seeded"),     # only the omega = 0 lines
    (32, 32, 32, 64, 64, "dense", "table"),     # square, several row blocks
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", SMALL, ids=[f"{c[0]}x{c[1]}w{c[2]}_{c[5]}_{c[6]}" for c in SMALL])
def test_small_grids_match_oracle(lib, oracle_mod, case, precision):
    nk, nw, W, nx, nt, kind, beta_mode = case
    wl = inp.small_grid(nk, nw, support_w=W, n_x=nx, n_t=nt, batch=3, seed_base=77)
    bis, b2 = _bispec(wl, kind, beta_mode)
    plan, u = _gpu_field(lib, wl, bis, precision, wl.seeds())
    P = _oracle_problem(oracle_mod, wl, bis, b2)
    C = _gpu_coeffs(lib, plan, wl.seeds()).cpu().numpy()
    for r, s in enumerate(wl.seeds()):
        Cref = P.coefficients(seed=int(s))
        ref = oracle_mod.field(Cref, nx, nt)
        if np.linalg.norm(ref) == 0:          # omega = 0 lines only: S(., 0) = 0
            assert np.all(u[r] == 0) and np.all(C[r] == 0)
            continue
        assert _rel_l2(u[r], ref) <= TOL[precision], (r, _rel_l2(u[r], ref))
        assert np.linalg.norm(C[r] - Cref) / np.linalg.norm(Cref) <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_invariance_and_determinism(lib, precision):
    torch = _torch()
    wl = inp.small_grid(24, 70, support_w=33, n_x=32, n_t=256)
    bis, _ = _bispec(wl, "separable", "seeded")
    plan = lib.srm3_plan(wl.grid_dict(), wl.spectrum(), bis, precision)
    seeds = [11, 12, 13, 14, 15]
    out = torch.empty((5, wl.n_x, wl.n_t), dtype=plan.real_dtype, device="cuda")
    lib.srm3_generate(plan, seeds, out)
    again = torch.empty_like(out)
    lib.srm3_generate(plan, seeds, again)
    one = torch.empty((1, wl.n_x, wl.n_t), dtype=plan.real_dtype, device="cuda")
    lib.srm3_generate(plan, [13], one)
    torch.cuda.synchronize()
    assert torch.equal(out, again)
    assert torch.equal(out[2], one[0])


def test_batch_orders_agree(lib):
    """Batches of 5 (interleaved block order) and 12 (XCD-blocked order) give
    bitwise the same realizations."""
    torch = _torch()
    wl = inp.small_grid(32, 96, support_w=80, n_x=32, n_t=256)
    bis, _ = _bispec(wl, "separable", "seeded")
    plan = lib.srm3_plan(wl.grid_dict(), wl.spectrum(), bis, "fp32")
    seeds = list(range(100, 112))
    big = torch.empty((12, wl.n_x, wl.n_t), dtype=torch.float32, device="cuda")
    lib.srm3_generate(plan, seeds, big)
    small = torch.empty((5, wl.n_x, wl.n_t), dtype=torch.float32, device="cuda")
    lib.srm3_generate(plan, seeds[3:8], small)
    torch.cuda.synchronize()
    assert torch.equal(big[3:8], small)


def test_zero_batch_and_bad_tensors(lib):
    torch = _torch()
    wl = inp.small_grid(4, 4)
    bis, _ = _bispec(wl, "separable", "seeded")
    plan = lib.srm3_plan(wl.grid_dict(), wl.spectrum(), bis, "fp32")
    out = torch.empty((1, wl.n_x, wl.n_t), dtype=torch.float32, device="cuda")
    lib.srm3_generate(plan, [], out)
    with pytest.raises(TypeError):
        lib.srm3_generate(plan, [1], out.double())
    with pytest.raises(ValueError):
        lib.srm3_generate(plan, [1, 2], out)


# ---------------------------------------------------------------------------
# Full-size workloads: sampled lines against the oracle, transform against
# the oracle's direct sum at sampled points, and properties of the whole field.
# ---------------------------------------------------------------------------
def _sample_lines(wl, n, seed):
    rng = np.random.default_rng(seed)
    nc = wl.n_cols
    kk = np.concatenate([[0, wl.n_kappa - 1, wl.n_kappa - 2, wl.n_kappa // 2],
                         rng.integers(0, wl.n_kappa, n - 4)])
    c = np.concatenate([[wl.n_omega - 1, 0, nc - 1, wl.n_omega], rng.integers(0, nc, n - 4)])
    return (kk * nc + c).astype(np.int64)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c1_full_size_sampled_lines(lib, oracle_mod, precision):
    torch = _torch()
    wl = inp.C1
    bis, b2 = _bispec(wl, "separable", "seeded")
    print(f"[gpu] c1 coefficients {precision}", flush=True)
    plan = lib.srm3_plan(wl.grid_dict(), wl.spectrum(), bis, precision)
    seeds = wl.seeds()
    C = _gpu_coeffs(lib, plan, seeds)
    P = _oracle_problem(oracle_mod, wl, bis, b2)
    for r in (0, 31, 63):
        lines = _sample_lines(wl, 4096 if r == 0 else 48, r)   # split parity on 4096 random lines
        ref = P.coefficients(seed=int(seeds[r]), lines=lines)
        got = C[r].reshape(-1)[torch.as_tensor(lines, device="cuda")].cpu().numpy()
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= TOL[precision], r
    # the fused generate path equals transform(coefficients)
    u = torch.empty((len(seeds), wl.n_x, wl.n_t), dtype=plan.real_dtype, device="cuda")
    lib.srm3_generate(plan, seeds, u)
    u2 = torch.empty_like(u)
    lib.srm3_transform(plan, C, u2)
    torch.cuda.synchronize()
    assert torch.equal(u, u2)
    # S(0, 0) = 0: every realization has zero grid mean
    mean = u.double().mean(dim=(1, 2)).abs().max().item()
    rms = u.double().pow(2).mean().sqrt().item()
    assert mean <= (1e-12 if precision == "fp64" else 1e-6) * rms


@pytest.mark.parametrize("wl_name,precision", [("c1", "fp64"), ("c1", "fp32"), ("c2", "fp32")])
def test_transform_full_size_sampled_points(lib, oracle_mod, wl_name, precision):
    torch = _torch()
    wl = inp.WORKLOADS[wl_name]
    print(f"[gpu] transform {wl_name} {precision}", flush=True)
    plan = lib.srm3_plan(wl.grid_dict(), wl.spectrum(), None, precision)
    Cnp = inp.random_coefficients(wl.n_kappa, wl.n_omega, 2, seed=123)
    cdt = torch.complex128 if precision == "fp64" else torch.complex64
    C = torch.as_tensor(Cnp).to(cdt).cuda()
    u = torch.empty((2, wl.n_x, wl.n_t), dtype=plan.real_dtype, device="cuda")
    lib.srm3_transform(plan, C, u)
    torch.cuda.synchronize()
    un = u.double().cpu().numpy()
    rng = np.random.default_rng(7)
    npts = 64 if wl_name == "c2" else 256
    for r in range(2):
        Cr = Cnp[r] if precision == "fp64" else Cnp[r].astype(np.complex64).astype(np.complex128)
        mx = rng.integers(0, wl.n_x, npts)
        mt = rng.integers(0, wl.n_t, npts)
        ref = oracle_mod.field_points(Cr, wl.n_x, wl.n_t, mx, mt)
        assert np.linalg.norm(un[r][mx, mt] - ref) / np.linalg.norm(ref) <= TOL[precision]
        # Parseval over the whole field (kappa = 0 row pairs k_w with -k_w)
        row0 = Cr[0]
        parse = 0.5 * np.sum(np.abs(Cr[1:]) ** 2) + 0.25 * np.sum(np.abs(row0 + np.conj(row0[::-1])) ** 2)
        assert abs(np.mean(un[r] ** 2) - parse) <= 10 * TOL[precision] * parse


def test_c2_full_size_sampled_lines(lib, oracle_mod):
    torch = _torch()
    wl = inp.C2
    bis, b2 = _bispec(wl, "separable", "seeded")
    print("[gpu] c2 coefficients fp32", flush=True)
    plan = lib.srm3_plan(wl.grid_dict(), wl.spectrum(), bis, "fp32")
    seeds = wl.seeds()
    C = _gpu_coeffs(lib, plan, seeds)
    P = _oracle_problem(oracle_mod, wl, bis, b2)
    for r in (0, 15):
        lines = _sample_lines(wl, 4096 if r == 0 else 24, 100 + r)
        ref = P.coefficients(seed=int(seeds[r]), lines=lines)
        got = C[r].reshape(-1)[torch.as_tensor(lines, device="cuda")].cpu().numpy()
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= TOL["fp32"], r


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_zero_bicoherence_is_the_gaussian_srm(lib, oracle_mod, precision):
    """With no bicoherence the plan skips the pair sum (2nd-order SRM); the field
    equals the oracle's with b = 0 and no pair terms are reported."""
    torch = _torch()
    for wl in (inp.C0, inp.small_grid(17, 40, batch=2, seed_base=55)):
        print(f"[gpu] gaussian {wl.name} {precision}", flush=True)
        plan = lib.srm3_plan(wl.grid_dict(), wl.spectrum(), None, precision)
        assert lib.srm3_pair_terms(plan) == 0
        seeds = wl.seeds()
        out = torch.empty((len(seeds), wl.n_x, wl.n_t), dtype=plan.real_dtype, device="cuda")
        lib.srm3_generate(plan, seeds, out)
        torch.cuda.synchronize()
        u = out.double().cpu().numpy()
        P = oracle_mod.Problem(wl.n_kappa, wl.n_omega, 1, wl.d_kappa, wl.d_omega, wl.spectrum(),
                               np.zeros((1, 1)), oracle_mod.biphase(1, None), 0.0)
        for r, s in enumerate(seeds):
            ref = oracle_mod.field(P.coefficients(seed=int(s)), wl.n_x, wl.n_t)
            assert _rel_l2(u[r], ref) <= TOL[precision]
