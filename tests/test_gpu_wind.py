"""Kappa-dependent bicoherence on the GPU against the FP64 oracle, through the
C-ABI: per-line factors (b2_raw = c_k^2 r_i^2 r_j^2 b2(i_w, j_w)) and the wind
bispectrum of Section 5 through the partial-bicoherence recursion, both pair-sum
algorithms, FP64 <= 1e-10 and FP32 <= 2e-5 relative L2; the bridge example
at full size on sampled lines; batches and the server."""
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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _run(lib, plan, nx, nt, seeds):
    torch = _torch()
    cdt = torch.complex128 if plan.precision == lib.SRM3_FP64 else torch.complex64
    C = torch.empty((len(seeds),) + plan.coeff_shape, dtype=cdt, device="cuda")
    lib.srm3_coefficients(plan, seeds, C)
    u = torch.empty((len(seeds), nx, nt), dtype=plan.real_dtype, device="cuda")
    lib.srm3_generate(plan, seeds, u)
    torch.cuda.synchronize()
    return C.to(torch.complex128).cpu().numpy(), u.double().cpu().numpy()


LINE_CASES = [
    # nk, nw, W, nx, nt, kind, beta_mode, cap
    (8, 12, 12, 16, 32, "separable", "seeded", 0.9),
    (13, 20, 9, 32, 64, "dense", "table", 0.5),
    (1, 8, 8, 1, 16, "separable", "zero", 0.0),
    (24, 40, 40, 64, 128, "dense", "seeded", 0.7),
]


@pytest.mark.parametrize("algorithm", ["direct", "mfma", "kappa_fft"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", LINE_CASES, ids=[f"{c[0]}x{c[1]}w{c[2]}_{c[5]}_{c[6]}_cap{c[7]}" for c in LINE_CASES])
def test_line_factors_match_oracle(lib, oracle_mod, case, precision, algorithm):
    nk, nw, W, nx, nt, kind, beta_mode, cap = case
    print(f"[gpu] line factors {case} {precision} {algorithm}", flush=True)
    S = inp.random_spectrum(nk, nw, seed=nk * nw)
    rng = np.random.default_rng(nk + nw)
    lc = rng.uniform(0.1, 0.6, size=S.shape)
    lr = rng.uniform(0.6, 1.3, size=S.shape)
    if kind == "separable":
        g2 = inp.exp_bicoherence_g2(W, 4 * np.pi / nw, 4 * np.pi, scale=0.1)
        b2 = np.outer(g2, g2)
    else:
        b2 = inp.random_b2_dense(W, 7, scale=0.05)
    bis = dict(kind=kind, support_w=W, cap=cap, beta_mode=beta_mode, beta_seed=99, line_c=lc, line_r=lr)
    if kind == "separable":
        bis["g2"] = g2
    else:
        bis["b2"] = b2
    if beta_mode == "table":
        beta = inp.random_beta_table(W, 8)
        bis["beta"] = beta
    else:
        beta = oracle_mod.biphase(W, None if beta_mode == "zero" else 99)
    grid = dict(n_kappa=nk, n_omega=nw, d_kappa=0.3, d_omega=0.2, n_x=nx, n_t=nt)
    plan = lib.srm3_plan(grid, S, bis, precision)
    lib.srm3_plan_set_algorithm(plan, algorithm)
    P = oracle_mod.Problem(nk, nw, W, 0.3, 0.2, S, b2, beta, cap, line_c=lc, line_r=lr)
    seeds = [5, 6, 7]
    C, u = _run(lib, plan, nx, nt, seeds)
    for i, s in enumerate(seeds):
        Cref = P.coefficients(seed=s)
        assert _rel(C[i], Cref) <= TOL[precision], i
        assert _rel(u[i], oracle_mod.field(Cref, nx, nt)) <= TOL[precision], i


WIND_CASES = [
    # nk, nw, W, nx, nt, alpha, cap, spectrum
    (6, 10, 10, 8, 32, 0.3, 0.0, "random"),
    (16, 24, 12, 32, 64, 1.0, 0.8, "paper"),
    (5, 7, 7, 8, 16, 0.5, 0.0, "paper"),
    (33, 17, 17, 64, 64, 2.0, 0.6, "random"),
]


@pytest.mark.parametrize("algorithm", ["direct", "mfma", "kappa_fft"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", WIND_CASES, ids=[f"{c[0]}x{c[1]}w{c[2]}_a{c[5]}_cap{c[6]}_{c[7]}" for c in WIND_CASES])
def test_wind_plans_match_oracle(lib, oracle_mod, case, precision, algorithm):
    nk, nw, W, nx, nt, alpha, cap, form = case
    print(f"[gpu] wind {case} {precision} {algorithm}", flush=True)
    dk, dw = 0.05, 0.1
    S = inp.random_spectrum(nk, nw, seed=3) if form == "random" else inp.kaimal_davenport_paper(nk, nw, dk, dw)
    grid = dict(n_kappa=nk, n_omega=nw, d_kappa=dk, d_omega=dw, n_x=nx, n_t=nt)
    plan = lib.srm3_plan(grid, S, dict(kind="wind", alpha=alpha, cap=cap, support_w=W), precision)
    lib.srm3_plan_set_algorithm(plan, algorithm)
    P = oracle_mod.WindProblem(nk, nw, W, dk, dw, S, alpha, cap)
    P.solve()
    seeds = [11, 12]
    C, u = _run(lib, plan, nx, nt, seeds)
    for i, s in enumerate(seeds):
        Cref = P.coefficients(seed=s)
        assert _rel(C[i], Cref) <= TOL[precision], i
        assert _rel(u[i], oracle_mod.field(Cref, nx, nt)) <= TOL[precision], i


def test_wind_plan_errors(lib):
    wl = inp.small_grid(6, 8)
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3_plan(wl.grid_dict(), wl.spectrum(), dict(kind="wind", alpha=100.0, cap=0.0, support_w=8), "fp32")
    assert ei.value.status == 2
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3_plan(wl.grid_dict(), wl.spectrum(), dict(kind="wind", alpha=0.0, cap=0.5, support_w=8), "fp32")
    assert ei.value.status == 1
    bad = np.ones(wl.spectrum().shape)
    bad[2, 3] = 0.0
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3_plan(wl.grid_dict(), wl.spectrum(), dict(kind="separable", g2=wl.g2(), support_w=8, line_r=bad),
                      "fp32")
    assert ei.value.status == 1
    pw = inp.small_process(16)
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3_process_plan(pw.grid_dict(), pw.spectrum(), dict(kind="wind", alpha=0.1, support_w=16), "fp32")
    assert ei.value.status == 5


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_bridge_full_size_sampled_lines(lib, oracle_mod, precision):
    """The bridge example of Section 5 (256 x 128 lines, 1024 x 2048 field,
    the wind bispectrum with cap 0.9) at full size: coefficients of sampled
    lines against the oracle's pair enumeration with the same line factors
    (the factorisation and the recursion are pinned on small grids)."""
    torch = _torch()
    wl = inp.bridge(alpha=1.0, cap=0.9, batch=4)
    print(f"[gpu] bridge {precision}", flush=True)
    S = wl.spectrum()
    plan = lib.srm3_plan(wl.grid_dict(), S, dict(kind="wind", alpha=wl.alpha, cap=wl.cap, support_w=wl.support_w),
                         precision)
    c, r, sig, _ = lib.srm3_wind_factors(wl.grid_dict(), S, wl.alpha, wl.cap, wl.support_w)
    W = wl.support_w
    P = oracle_mod.Problem(wl.n_kappa, wl.n_omega, W, wl.d_kappa, wl.d_omega, S, np.ones((2 * W - 1, 2 * W - 1)),
                           oracle_mod.biphase(W, None), wl.cap, line_c=c, line_r=r)
    seeds = wl.seeds()
    cdt = torch.complex128 if precision == "fp64" else torch.complex64
    C = torch.empty((len(seeds),) + plan.coeff_shape, dtype=cdt, device="cuda")
    lib.srm3_coefficients(plan, seeds, C)
    u = torch.empty((len(seeds), wl.n_x, wl.n_t), dtype=plan.real_dtype, device="cuda")
    lib.srm3_generate(plan, seeds, u)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    for b in (0, len(seeds) - 1):
        kk = np.concatenate([[wl.n_kappa - 1, 1, 0], rng.integers(0, wl.n_kappa, 29)])
        cc = np.concatenate([[0, wl.n_cols - 1, wl.n_omega], rng.integers(0, wl.n_cols, 29)])
        lines = (kk * wl.n_cols + cc).astype(np.int64)
        ref = P.coefficients(seed=int(seeds[b]), lines=lines)
        got = C[b].reshape(-1)[torch.as_tensor(lines, device="cuda")].to(torch.complex128).cpu().numpy()
        assert _rel(got, ref) <= TOL[precision], b
    # the field is the transform of the coefficients (checked elsewhere) and skewed
    x = u.double()
    x = x - x.mean(dim=(1, 2), keepdim=True)
    skew = (x.pow(3).mean() / x.pow(2).mean().pow(1.5)).item()
    assert skew > 0.02


def test_wind_plans_in_batches_and_the_server(lib):
    torch = _torch()
    wl = inp.small_grid(16, 32)
    S = inp.kaimal_davenport_paper(16, 32, 0.05, 0.1)
    grid = dict(wl.grid_dict(), d_kappa=0.05, d_omega=0.1)
    plan = lib.srm3_plan(grid, S, dict(kind="wind", alpha=1.0, cap=0.8, support_w=32), "fp32")
    kplan = lib.srm3_plan(grid, S, dict(kind="wind", alpha=1.0, cap=0.8, support_w=32), "fp32")
    lib.srm3_plan_set_algorithm(kplan, "kappa_fft")
    reqs, singles = [], []
    for i in range(6):
        p = plan if i % 2 == 0 else kplan
        out = torch.empty(p.field_shape, dtype=torch.float32, device="cuda")
        one = torch.empty((1,) + p.field_shape, dtype=torch.float32, device="cuda")
        lib.srm3_generate(p, [40 + i], one)
        reqs.append(dict(plan=p, seed=40 + i, out=out))
        singles.append(one[0])
    print("[gpu] wind batch", flush=True)
    b = lib.Batch(reqs, flags=lib.SRM3_BATCH_GRAPH)
    for _ in range(2):
        for r in reqs:
            r["out"].zero_()
        b.run()
        torch.cuda.synchronize()
        for r, s in zip(reqs, singles):
            assert torch.equal(r["out"], s)
    print("[gpu] wind server", flush=True)
    srv = lib.srm3.Server("fp32", max_active=3, hbm_budget=1 << 30)
    for r in reqs:
        r["out"].zero_()
    tickets = [srv.submit(r["plan"], r["seed"], r["out"]) for r in reqs]
    done = []
    for _ in range(10000):
        srv.step()
        done += srv.poll()
        if len(done) == len(tickets):
            break
    torch.cuda.synchronize()
    assert sorted(done) == sorted(tickets)
    for r, s in zip(reqs, singles):
        assert torch.equal(r["out"], s)


PRODUCT_CASES = [
    # nk, nw, W, nx, nt, scale, cap, with_h
    (6, 10, 10, 8, 32, 0.4, 0.0, True),
    (16, 24, 12, 32, 64, 2.0, 0.7, True),
    (9, 12, 12, 16, 32, 0.25, 0.0, False),
]


@pytest.mark.parametrize("algorithm", ["direct", "mfma", "kappa_fft", "fft2d"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", PRODUCT_CASES, ids=[f"{c[0]}x{c[1]}w{c[2]}_s{c[5]}_cap{c[6]}_H{c[7]}" for c in PRODUCT_CASES])
def test_product_bispectrum_matches_oracle(lib, oracle_mod, case, precision, algorithm):
    """A prescribed complex bispectrum B = F_k G_i G_j H(i_w, j_w) through the
    partial-bicoherence recursion, beta = atan2(Im B, Re B)."""
    nk, nw, W, nx, nt, scale, cap, with_h = case
    if algorithm == "fft2d" and with_h:
        pytest.skip("the 2-D FFT pair sum needs rank-one weights (H = 1)")
    print(f"[gpu] product {case} {precision} {algorithm}", flush=True)
    rng = np.random.default_rng(nk * nw)
    S = inp.random_spectrum(nk, nw, seed=nk * nw)
    F = scale * rng.uniform(0.2, 1.0, S.shape) * np.exp(1j * rng.uniform(0, 2 * np.pi, S.shape))
    G = np.sqrt(S) * rng.uniform(0.5, 1.0, S.shape) * np.exp(1j * rng.uniform(0, 2 * np.pi, S.shape))
    H = None
    if with_h:
        A = rng.uniform(0.3, 1.0, (2 * W - 1, 2 * W - 1)) * np.exp(1j * rng.uniform(0, 2 * np.pi, (2 * W - 1, 2 * W - 1)))
        H = 0.5 * (A + A.T)
    dk, dw = 0.5, 0.4
    grid = dict(n_kappa=nk, n_omega=nw, d_kappa=dk, d_omega=dw, n_x=nx, n_t=nt)
    bis = dict(kind="product", F=F, G=G, H=H, cap=cap, support_w=W)
    plan = lib.srm3_plan(grid, S, bis, precision)
    lib.srm3_plan_set_algorithm(plan, algorithm)
    P = oracle_mod.ProductProblem(nk, nw, W, dk, dw, S, F, G, H, cap)
    P.solve()
    seeds = [21, 22]
    C, u = _run(lib, plan, nx, nt, seeds)
    for i, s in enumerate(seeds):
        Cref = P.coefficients(seed=s)
        assert _rel(C[i], Cref) <= TOL[precision], i
        assert _rel(u[i], oracle_mod.field(Cref, nx, nt)) <= TOL[precision], i


HASH_CASES = [
    # nk, nw, W, nx, nt, scale, cap
    (6, 10, 10, 8, 32, 0.02, 0.5),
    (13, 20, 9, 32, 64, 0.01, 0.0),
    (1, 8, 8, 1, 16, 0.05, 0.0),
    (24, 40, 40, 64, 128, 0.004, 0.9),
    # several 256-column groups, a ragged last wave, partner range below the line range
    (20, 300, 120, 32, 1024, 0.002, 0.5),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", HASH_CASES, ids=[f"{c[0]}x{c[1]}w{c[2]}_cap{c[6]}" for c in HASH_CASES])
def test_hashed_bispectrum_matches_oracle(lib, oracle_mod, case, precision):
    """b and beta generated per 4-index pair inside the kernel."""
    nk, nw, W, nx, nt, scale, cap = case
    print(f"[gpu] hashed {case} {precision}", flush=True)
    S = inp.random_spectrum(nk, nw, seed=nk + nw)
    grid = dict(n_kappa=nk, n_omega=nw, d_kappa=0.3, d_omega=0.2, n_x=nx, n_t=nt)
    key = 0x1234ABCD5678
    plan = lib.srm3_plan(grid, S, dict(kind="hashed", alpha=scale, beta_seed=key, cap=cap, support_w=W), precision)
    P = oracle_mod.HashedProblem(nk, nw, W, 0.3, 0.2, S, scale, key, cap)
    seeds = [31, 32]
    C, u = _run(lib, plan, nx, nt, seeds)
    for i, s in enumerate(seeds):
        Cref = P.coefficients(seed=s)
        assert _rel(C[i], Cref) <= TOL[precision], i
        assert _rel(u[i], oracle_mod.field(Cref, nx, nt)) <= TOL[precision], i
    one = _run(lib, plan, nx, nt, [seeds[1]])[0]
    assert np.array_equal(one[0], C[1])


def test_hashed_full_size_sampled_lines_and_errors(lib, oracle_mod):
    torch = _torch()
    wl = inp.C1.with_(batch=1)
    print("[gpu] hashed c1", flush=True)
    S = wl.spectrum()
    key = 77
    bis = dict(kind="hashed", alpha=1e-4, beta_seed=key, cap=0.9, support_w=wl.support_w)
    plan = lib.srm3_plan(wl.grid_dict(), S, bis, "fp32")
    C = torch.empty((1,) + plan.coeff_shape, dtype=torch.complex64, device="cuda")
    lib.srm3_coefficients(plan, wl.seeds(), C)
    torch.cuda.synchronize()
    P = oracle_mod.HashedProblem(wl.n_kappa, wl.n_omega, wl.support_w, wl.d_kappa, wl.d_omega, S, 1e-4, key, 0.9)
    rng = np.random.default_rng(12)
    kk = np.concatenate([[wl.n_kappa - 1, 0], rng.integers(0, wl.n_kappa, 30)])
    cc = np.concatenate([[wl.n_omega - 1, 0], rng.integers(0, wl.n_cols, 30)])
    lines = (kk * wl.n_cols + cc).astype(np.int64)
    ref = P.coefficients(seed=int(wl.seeds()[0]), lines=lines)
    got = C[0].reshape(-1)[torch.as_tensor(lines, device="cuda")].to(torch.complex128).cpu().numpy()
    assert _rel(got, ref) <= TOL["fp32"]
    for algo in ("kappa_fft", "fft2d"):
        with pytest.raises(lib.Srm3Error) as ei:
            lib.srm3_plan_set_algorithm(plan, algo)
        assert ei.value.status == 5
    out = torch.empty(plan.field_shape, dtype=torch.float32, device="cuda")
    with pytest.raises(lib.Srm3Error) as ei:
        lib.Batch([dict(plan=plan, seed=1, out=out)])
    assert ei.value.status == 5
    srv = lib.srm3.Server("fp32", max_active=2, hbm_budget=1 << 30)
    with pytest.raises(lib.Srm3Error) as ei:
        srv.submit(plan, 1, out)
    assert ei.value.status == 5


def test_product_plan_keeps_its_spectrum(lib):
    torch = _torch()
    nk, nw, W = 6, 10, 10
    rng = np.random.default_rng(2)
    S = inp.random_spectrum(nk, nw, seed=2)
    F = 0.3 * rng.uniform(0.2, 1.0, S.shape) + 0j
    G = np.sqrt(S) + 0j
    grid = dict(n_kappa=nk, n_omega=nw, d_kappa=0.5, d_omega=0.4, n_x=8, n_t=32)
    plan = lib.srm3_plan(grid, S, dict(kind="product", F=F, G=G, cap=0.5, support_w=W), "fp32")
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3_set_spectrum(plan, S)
    assert ei.value.status == 5
    out = torch.empty(plan.field_shape, dtype=torch.float32, device="cuda")
    Sd = torch.as_tensor(S, device="cuda")
    with pytest.raises(lib.Srm3Error) as ei:
        lib.Batch([dict(plan=plan, seed=1, out=out, S=Sd)])
    assert ei.value.status == 5
    srv = lib.srm3.Server("fp32", max_active=2, hbm_budget=1 << 28)
    with pytest.raises(lib.Srm3Error) as ei:
        srv.submit(plan, 1, out, spectrum=dict(U=30.0))
    assert ei.value.status == 5
    b = lib.Batch([dict(plan=plan, seed=1, out=out)])        # its own spectrum is fine
    b.run()
    torch.cuda.synchronize()
