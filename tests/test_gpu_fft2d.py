"""The pair sum as a 2-D FFT autoconvolution (SRM3_ALGO_FFT2D: rank-one
weights, separable b^2 with beta = 0) against the FP64 oracle through the
C-ABI, FP64 <= 1e-10 and FP32 <= 2e-5 relative L2: small and degenerate
grids, wind plans, a process plan, the 256x1024 and 512x8192 grids and the
bridge example at full size on sampled lines, batches, errors."""
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


SMALL = [
    # nk, nw, W, nx, nt
    (32, 64, 64, 64, 128),
    (5, 40, 40, 8, 128),
    (24, 70, 33, 32, 256),      # truncated support
    (1, 8, 8, 1, 16),           # one kappa row
    (3, 5, 1, 4, 16),           # support of one frequency (L = 1)
    (40, 300, 300, 128, 1024),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", SMALL, ids=[f"{c[0]}x{c[1]}w{c[2]}" for c in SMALL])
def test_small_grids_match_oracle(lib, oracle_mod, case, precision):
    nk, nw, W, nx, nt = case
    print(f"[gpu] fft2d {case} {precision}", flush=True)
    wl = inp.small_grid(nk, nw, support_w=W, n_x=nx, n_t=nt, batch=3, seed_base=17)
    plan = lib.plan_from_workload(wl, precision, beta_mode="zero")
    lib.srm3_plan_set_algorithm(plan, "fft2d")
    P = oracle_mod.Problem.from_workload(wl, beta_zero=True)
    C, u = _run(lib, plan, nx, nt, wl.seeds())
    for r, s in enumerate(wl.seeds()):
        Cref = P.coefficients(seed=int(s))
        assert _rel(C[r], Cref) <= TOL[precision], r
        assert _rel(u[r], oracle_mod.field(Cref, nx, nt)) <= TOL[precision], r


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_wind_plans_and_agreement(lib, oracle_mod, precision):
    torch = _torch()
    nk, nw, W, nx, nt = 16, 24, 12, 32, 64
    dk, dw = 0.05, 0.1
    S = inp.kaimal_davenport_paper(nk, nw, dk, dw)
    grid = dict(n_kappa=nk, n_omega=nw, d_kappa=dk, d_omega=dw, n_x=nx, n_t=nt)
    bis = dict(kind="wind", alpha=1.0, cap=0.8, support_w=W)
    plans = {}
    for algo in ("direct", "kappa_fft", "fft2d"):
        plans[algo] = lib.srm3_plan(grid, S, bis, precision)
        lib.srm3_plan_set_algorithm(plans[algo], algo)
    P = oracle_mod.WindProblem(nk, nw, W, dk, dw, S, 1.0, 0.8)
    P.solve()
    seeds = [3, 4]
    res = {a: _run(lib, p, nx, nt, seeds) for a, p in plans.items()}
    for i, s in enumerate(seeds):
        Cref = P.coefficients(seed=s)
        assert _rel(res["fft2d"][0][i], Cref) <= TOL[precision]
        assert _rel(res["fft2d"][1][i], oracle_mod.field(Cref, nx, nt)) <= TOL[precision]
    assert _rel(res["fft2d"][0], res["direct"][0]) <= (1e-12 if precision == "fp64" else 2e-5)
    # batch invariance
    one = _run(lib, plans["fft2d"], nx, nt, [seeds[1]])[1]
    assert np.array_equal(one[0], res["fft2d"][1][1])
    del torch


def test_process_plan(lib, oracle_mod):
    wl = inp.small_process(300, support_w=200, batch=9, seed_base=4)
    plan = lib.process_plan_from_workload(wl, "fp32", beta_mode="zero")
    lib.srm3_plan_set_algorithm(plan, "fft2d")
    P = oracle_mod.ProcessProblem(wl.n, wl.support_w, wl.d_omega, wl.spectrum(), wl.b2_dense(),
                                  oracle_mod.process_biphase(wl.support_w, None), wl.cap)
    C, u = _run(lib, plan, 1, wl.n_t, wl.seeds())
    for r, s in enumerate(wl.seeds()):
        Cref = P.coefficients(seed=int(s))
        assert _rel(C[r, 0, wl.n - 1:], Cref) <= TOL["fp32"], r
        assert _rel(u[r, 0], oracle_mod.process_field(Cref, wl.n_t)) <= TOL["fp32"], r


def test_errors_and_terms(lib):
    wl = inp.small_grid(8, 16)
    seeded = lib.plan_from_workload(wl, "fp32")                  # random biphase: not rank one
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3_plan_set_algorithm(seeded, "fft2d")
    assert ei.value.status == 5
    dense = lib.plan_from_workload(wl, "fp32", beta_mode="zero", dense=True)
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3_plan_set_algorithm(dense, "fft2d")
    assert ei.value.status == 5
    big = inp.small_grid(2, 2049, support_w=2049, n_x=2, n_t=8192)
    pb = lib.plan_from_workload(big, "fp64", beta_mode="zero")
    with pytest.raises(lib.Srm3Error) as ei:                       # FP64: L = 16384 > 8192
        lib.srm3_plan_set_algorithm(pb, "fft2d")
    assert ei.value.status == 5
    ok = lib.plan_from_workload(wl, "fp32", beta_mode="zero")
    lib.srm3_plan_set_algorithm(ok, "fft2d")
    # M = 16 kappa frequencies x (L log2 L + L) with L = 64
    assert lib.srm3_algorithm_terms(ok) == 16 * (64 * 6 + 64)


@pytest.mark.parametrize("name,precision", [("c1", "fp32"), ("c1", "fp64"), ("c2", "fp32")])
def test_full_size_grids_sampled_lines(lib, oracle_mod, name, precision):
    torch = _torch()
    wl = inp.WORKLOADS[name].with_(batch=2)
    print(f"[gpu] fft2d {name} {precision}", flush=True)
    plan = lib.plan_from_workload(wl, precision, beta_mode="zero")
    lib.srm3_plan_set_algorithm(plan, "fft2d")
    seeds = wl.seeds()
    cdt = torch.complex128 if precision == "fp64" else torch.complex64
    C = torch.empty((len(seeds),) + plan.coeff_shape, dtype=cdt, device="cuda")
    lib.srm3_coefficients(plan, seeds, C)
    torch.cuda.synchronize()
    P = oracle_mod.Problem.from_workload(wl, beta_zero=True)
    rng = np.random.default_rng(8)
    kk = np.concatenate([[0, wl.n_kappa - 1], rng.integers(0, wl.n_kappa, 22)])
    c = (wl.n_omega - 1) + rng.integers(-(2 * wl.support_w - 2), 2 * wl.support_w - 1, 24)
    c = np.clip(c, 0, wl.n_cols - 1)
    lines = (kk * wl.n_cols + c).astype(np.int64)
    ref = P.coefficients(seed=int(seeds[1]), lines=lines)
    got = C[1].reshape(-1)[torch.as_tensor(lines, device="cuda")].to(torch.complex128).cpu().numpy()
    assert _rel(got, ref) <= TOL[precision]


def test_bridge_and_batches(lib, oracle_mod):
    torch = _torch()
    wl = inp.bridge(alpha=1.0, cap=0.9, batch=2)
    S = wl.spectrum()
    bis = dict(kind="wind", alpha=wl.alpha, cap=wl.cap, support_w=wl.support_w)
    plan = lib.srm3_plan(wl.grid_dict(), S, bis, "fp32")
    lib.srm3_plan_set_algorithm(plan, "fft2d")
    c, r, _, _ = lib.srm3_wind_factors(wl.grid_dict(), S, wl.alpha, wl.cap, wl.support_w)
    W = wl.support_w
    P = oracle_mod.Problem(wl.n_kappa, wl.n_omega, W, wl.d_kappa, wl.d_omega, S, np.ones((2 * W - 1, 2 * W - 1)),
                           oracle_mod.biphase(W, None), wl.cap, line_c=c, line_r=r)
    seeds = wl.seeds()
    C = torch.empty((2,) + plan.coeff_shape, dtype=torch.complex64, device="cuda")
    lib.srm3_coefficients(plan, seeds, C)
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    lines = (rng.integers(0, wl.n_kappa, 40) * wl.n_cols + rng.integers(0, wl.n_cols, 40)).astype(np.int64)
    ref = P.coefficients(seed=int(seeds[0]), lines=lines)
    got = C[0].reshape(-1)[torch.as_tensor(lines, device="cuda")].to(torch.complex128).cpu().numpy()
    assert _rel(got, ref) <= TOL["fp32"]
    # fft2d plans in a batch and the server, bitwise equal to single generation
    small = inp.small_grid(16, 32)
    sp = lib.plan_from_workload(small, "fp32", beta_mode="zero")
    lib.srm3_plan_set_algorithm(sp, "fft2d")
    reqs, singles = [], []
    for i in range(4):
        out = torch.empty(sp.field_shape, dtype=torch.float32, device="cuda")
        one = torch.empty((1,) + sp.field_shape, dtype=torch.float32, device="cuda")
        lib.srm3_generate(sp, [60 + i], one)
        reqs.append(dict(plan=sp, seed=60 + i, out=out))
        singles.append(one[0])
    b = lib.Batch(reqs, flags=lib.SRM3_BATCH_GRAPH)
    for _ in range(2):
        b.run()
        torch.cuda.synchronize()
        for q, s in zip(reqs, singles):
            assert torch.equal(q["out"], s)
    srv = lib.srm3.Server("fp32", max_active=2, hbm_budget=1 << 30)
    for q in reqs:
        q["out"].zero_()
    tickets = [srv.submit(q["plan"], q["seed"], q["out"]) for q in reqs]
    done = []
    for _ in range(10000):
        srv.step()
        done += srv.poll()
        if len(done) == len(tickets):
            break
    torch.cuda.synchronize()
    assert sorted(done) == sorted(tickets)
    for q, s in zip(reqs, singles):
        assert torch.equal(q["out"], s)
