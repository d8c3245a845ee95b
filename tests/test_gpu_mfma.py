"""The direct-form pair sum on the matrix cores (SRM3_ALGO_MFMA) against the
FP64 oracle through the C-ABI, FP64 <= 1e-10 and FP32 <= 2e-5 relative L2: small, ragged and
degenerate grids with every bispectrum form (the 256x1024 and 512x8192 grids at
full batch: 4096 sampled lines each, in test_gpu_large.py), agreement with the vector kernel, batch
invariance, uneven batches (matrix-core items in the persistent launch) equal
to single generation, a process plan, a wind plan with line factors, and
errors."""
import numpy as np
import pytest

import srm3_inputs as inp

pytestmark = pytest.mark.gpu

TOL = 2e-5
TOLS = {"fp64": 1e-10, "fp32": 2e-5}


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


def _bispec(wl, kind, beta_mode, seed=5):
    b = dict(kind=kind, support_w=wl.support_w, cap=wl.cap, beta_mode=beta_mode, beta_seed=wl.beta_seed)
    if kind == "separable":
        b["g2"] = wl.g2()
        b2 = wl.b2_dense()
    else:
        b2 = inp.random_b2_dense(wl.support_w, seed, scale=0.3)
        b["b2"] = b2
    if beta_mode == "table":
        b["beta"] = inp.random_beta_table(wl.support_w, seed + 1)
    return b, b2


def _problem(oracle_mod, wl, bis, b2):
    if bis.get("beta_mode") == "table":
        beta = bis["beta"]
    elif bis.get("beta_mode") == "zero":
        beta = oracle_mod.biphase(wl.support_w, None)
    else:
        beta = oracle_mod.biphase(wl.support_w, wl.beta_seed)
    return oracle_mod.Problem(wl.n_kappa, wl.n_omega, wl.support_w, wl.d_kappa, wl.d_omega,
                              wl.spectrum(), b2, beta, bis["cap"])


def _plan(lib, wl, bis, precision="fp32"):
    plan = lib.srm3_plan(wl.grid_dict(), wl.spectrum(), bis, precision)
    lib.srm3_plan_set_algorithm(plan, "mfma")
    return plan


def _coeffs(lib, plan, seeds):
    torch = _torch()
    cdt = torch.complex128 if plan.precision == lib.SRM3_FP64 else torch.complex64
    C = torch.empty((len(seeds),) + plan.coeff_shape, dtype=cdt, device="cuda")
    lib.srm3_coefficients(plan, seeds, C)
    torch.cuda.synchronize()
    return C


def _field(lib, plan, nx, nt, seeds):
    torch = _torch()
    out = torch.empty((len(seeds), nx, nt), dtype=plan.real_dtype, device="cuda")
    lib.srm3_generate(plan, seeds, out)
    torch.cuda.synchronize()
    return out


SMALL = [
    # nk, nw, W, nx, nt, kind, beta_mode
    (32, 64, 64, 64, 128, "separable", "seeded"),   # one row group, several column tiles
    (5, 40, 40, 16, 128, "dense", "table"),         # rows below one 16-row tile
    (24, 70, 33, 64, 256, "dense", "seeded"),       # truncated support, ragged column tile
    (17, 9, 9, 64, 32, "separable", "zero"),        # odd rows, beta == 0
    (1, 8, 8, 2, 16, "separable", "seeded"),        # a single kappa row (every split is the half one)
    (3, 5, 1, 8, 16, "dense", "seeded"),            # support of one frequency
    (2, 1, 1, 4, 1, "separable", "seeded"),         # only the omega = 0 lines
    (70, 33, 17, 256, 128, "dense", "table"),       # three row groups, the last ragged
    (40, 300, 300, 128, 1024, "separable", "seeded"),   # many partner steps, two row groups
]


@pytest.mark.parametrize("shape", [0, 1, 2])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", SMALL, ids=[f"{c[0]}x{c[1]}w{c[2]}_{c[5]}_{c[6]}" for c in SMALL])
def test_small_grids_match_oracle(lib, oracle_mod, case, precision, shape):
    nk, nw, W, nx, nt, kind, beta_mode = case
    wl = inp.small_grid(nk, nw, support_w=W, n_x=nx, n_t=nt, batch=3, seed_base=71)
    print(f"[gpu] mfma {case} {precision} shape {shape}", flush=True)
    bis, b2 = _bispec(wl, kind, beta_mode)
    plan = _plan(lib, wl, bis, precision)
    lib.srm3_plan_set_mfma_shape(plan, shape)
    C = _coeffs(lib, plan, wl.seeds()).to(_torch().complex128).cpu().numpy()
    u = _field(lib, plan, nx, nt, wl.seeds()).double().cpu().numpy()
    P = _problem(oracle_mod, wl, bis, b2)
    for r, s in enumerate(wl.seeds()):
        Cref = P.coefficients(seed=int(s))
        ref = oracle_mod.field(Cref, nx, nt)
        if np.linalg.norm(ref) == 0:
            assert np.all(C[r] == 0) and np.all(u[r] == 0)
            continue
        assert _rel(C[r], Cref) <= TOLS[precision], r
        assert _rel(u[r], ref) <= TOLS[precision], r


def test_tile_shapes(lib):
    assert lib.srm3_mfma_shape("fp32", 0) == (32, 32)
    assert lib.srm3_mfma_shape("fp32", 1) == (32, 16)
    assert lib.srm3_mfma_shape("fp64", 2) == (16, 32)
    wl = inp.small_grid(8, 16)
    bis, _ = _bispec(wl, "separable", "seeded")
    plan = _plan(lib, wl, bis)
    for bad in (-1, 3):
        with pytest.raises(lib.Srm3Error) as ei:
            lib.srm3_plan_set_mfma_shape(plan, bad)
        assert ei.value.status == 1


@pytest.mark.parametrize("shape", [1, 2])
def test_shapes_agree(lib, shape):
    """Every tile shape sums the same pair terms: coefficients agree with the
    default shape's to rounding, on a grid with ragged row groups."""
    torch = _torch()
    wl = inp.small_grid(100, 300, support_w=260, batch=5, seed_base=400)
    bis, _ = _bispec(wl, "separable", "seeded")
    ref = _plan(lib, wl, bis)
    other = _plan(lib, wl, bis)
    lib.srm3_plan_set_mfma_shape(other, shape)
    a = _coeffs(lib, ref, wl.seeds()).to(torch.complex128)
    b = _coeffs(lib, other, wl.seeds()).to(torch.complex128)
    rel = ((a - b).abs().pow(2).sum() / a.abs().pow(2).sum()).sqrt().item()
    assert rel <= 2e-6


def test_agrees_with_vector_kernel_and_is_batch_invariant(lib):
    torch = _torch()
    wl = inp.small_grid(64, 200, support_w=150, batch=6, seed_base=300)
    bis, _ = _bispec(wl, "separable", "seeded")
    vec = lib.srm3_plan(wl.grid_dict(), wl.spectrum(), bis, "fp32")
    mat = _plan(lib, wl, bis)
    seeds = wl.seeds()
    a = _coeffs(lib, vec, seeds).to(torch.complex128)
    b = _coeffs(lib, mat, seeds).to(torch.complex128)
    rel = ((a - b).abs().pow(2).sum() / a.abs().pow(2).sum()).sqrt().item()
    assert rel <= 2e-6
    one = _coeffs(lib, mat, [int(seeds[4])])
    assert torch.equal(one[0].to(torch.complex128), b[4])
    again = _coeffs(lib, mat, seeds).to(torch.complex128)
    assert torch.equal(again, b)
    assert lib.srm3_algorithm_terms(mat) == lib.srm3_pair_terms(mat)
    # switching back gives the vector result again, bitwise
    lib.srm3_plan_set_algorithm(mat, "direct")
    assert torch.equal(_coeffs(lib, mat, seeds).to(torch.complex128), a)


def test_process_and_wind_plans(lib, oracle_mod):
    # the 1-D process: one kappa row, one-sided spectrum
    wl = inp.small_process(300, support_w=200, batch=4, seed_base=6)
    bis = dict(kind="separable", g2=wl.g2(), support_w=wl.support_w, cap=wl.cap, beta_mode="seeded",
               beta_seed=wl.beta_seed)
    plan = lib.srm3_process_plan(wl.grid_dict(), wl.spectrum(), bis, "fp32")
    lib.srm3_plan_set_algorithm(plan, "mfma")
    P = oracle_mod.ProcessProblem(wl.n, wl.support_w, wl.d_omega, wl.spectrum(), wl.b2_dense(),
                                  oracle_mod.process_biphase(wl.support_w, wl.beta_seed), wl.cap)
    C = _coeffs(lib, plan, wl.seeds()).to(_torch().complex128).cpu().numpy()[:, 0, :]
    u = _field(lib, plan, 1, wl.n_t, wl.seeds()).double().cpu().numpy()[:, 0, :]
    for r, s in enumerate(wl.seeds()):
        Cref = P.coefficients(seed=int(s))
        assert _rel(C[r, wl.n - 1:], Cref) <= TOL, r
        assert _rel(u[r], oracle_mod.process_field(Cref, wl.n_t)) <= TOL, r
    # the wind bispectrum (kappa-dependent line factors applied at assembly)
    nk, nw, W, nx, nt = 16, 24, 12, 32, 64
    dk, dw = 0.05, 0.1
    S = inp.kaimal_davenport_paper(nk, nw, dk, dw)
    grid = dict(n_kappa=nk, n_omega=nw, d_kappa=dk, d_omega=dw, n_x=nx, n_t=nt)
    wp = lib.srm3_plan(grid, S, dict(kind="wind", alpha=1.0, cap=0.8, support_w=W), "fp32")
    lib.srm3_plan_set_algorithm(wp, "mfma")
    Pw = oracle_mod.WindProblem(nk, nw, W, dk, dw, S, 1.0, 0.8)
    Pw.solve()
    Cw = _coeffs(lib, wp, [3, 4]).to(_torch().complex128).cpu().numpy()
    for i, s in enumerate([3, 4]):
        assert _rel(Cw[i], Pw.coefficients(seed=s)) <= TOL


def test_errors(lib):
    torch = _torch()
    wl = inp.small_grid(8, 16)
    bis, _ = _bispec(wl, "separable", "seeded")
    hashed = lib.srm3_plan(wl.grid_dict(), wl.spectrum(),
                           dict(kind="hashed", alpha=0.5, support_w=wl.support_w, cap=0.9, beta_seed=3), "fp32")
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3_plan_set_algorithm(hashed, "mfma")
    assert ei.value.status == 5
    plan = _plan(lib, wl, bis)
    out = torch.empty(plan.field_shape, dtype=torch.float32, device="cuda")
    vec = lib.srm3_plan(wl.grid_dict(), wl.spectrum(), bis, "fp32")
    out2 = torch.empty(plan.field_shape, dtype=torch.float32, device="cuda")
    with pytest.raises(lib.Srm3Error) as ei:      # one pair-sum kernel per batch
        lib.Batch([dict(plan=plan, seed=1, out=out), dict(plan=vec, seed=2, out=out2)])
    assert ei.value.status == 5
    srv = lib.srm3.Server("fp32", max_active=2, hbm_budget=1 << 28)
    with pytest.raises(lib.Srm3Error) as ei:
        srv.submit(plan, 1, out)
    assert ei.value.status == 5


@pytest.mark.parametrize("flags,precision", [("plain", "fp32"), ("graph_autotune", "fp32"), ("plain", "fp64")])
def test_uneven_batch_equals_single_generation(lib, flags, precision, monkeypatch, tmp_path):
    """Mixed grids (ragged rows and columns, truncated support, a Gaussian
    plan and a kappa-DFT plan beside them) in one batch: each realization
    equals its single generation bitwise, over two runs."""
    torch = _torch()
    monkeypatch.setenv("SRM3_TUNE_CACHE", str(tmp_path / "tune.txt"))
    grids = [(40, 300, 300), (5, 40, 40), (70, 33, 17), (24, 70, 33), (1, 8, 8)]
    plans = []
    for nk, nw, W in grids:
        wl = inp.small_grid(nk, nw, support_w=W)
        bis, _ = _bispec(wl, "separable", "seeded")
        plans.append(_plan(lib, wl, bis, precision))
    wg = inp.small_grid(16, 32)
    plans.append(lib.srm3_plan(wg.grid_dict(), wg.spectrum(), None, precision))        # zero bicoherence
    wk = inp.small_grid(16, 40)
    pk = lib.plan_from_workload(wk, precision)
    lib.srm3_plan_set_algorithm(pk, "kappa_fft")
    plans.append(pk)
    reqs = []
    for i in range(11):
        plan = plans[i % len(plans)]
        reqs.append(dict(plan=plan, seed=700 + 3 * i, out=torch.empty(plan.field_shape, dtype=plan.real_dtype,
                                                                       device="cuda")))
    print(f"[gpu] mfma uneven batch {flags} {precision}", flush=True)
    fl = 0 if flags == "plain" else lib.SRM3_BATCH_GRAPH | lib.SRM3_BATCH_AUTOTUNE
    b = lib.Batch(reqs, flags=fl)
    b.run()
    torch.cuda.synchronize()
    shape = b.info()["mfma_shape"]
    assert shape in (0, 1, 2) and (flags != "plain" or shape == 0)
    # single generation with the tile shape the batch runs (the tuner may pick any)
    singles = []
    for r in reqs:
        lib.srm3_plan_set_mfma_shape(r["plan"], shape)
        one = torch.empty((1,) + r["plan"].field_shape, dtype=r["plan"].real_dtype, device="cuda")
        lib.srm3_generate(r["plan"], [r["seed"]], one)
        singles.append(one[0])
    for _ in range(2):
        for r in reqs:
            r["out"].zero_()
        b.run()
        torch.cuda.synchronize()
        for r, s in zip(reqs, singles):
            assert torch.equal(r["out"], s)


@pytest.mark.parametrize("shape", [0, 2])
def test_server_with_matrix_core_items(lib, shape):
    """A server whose persistent pair-sum launch takes matrix-core items (of a
    given tile shape): mixed grids (and a kappa-DFT and a Gaussian plan beside
    them) give each request's single generation with that shape bitwise; plans
    of the other kernel and unknown kernels or shapes are refused."""
    torch = _torch()
    grids = [(40, 300, 300), (5, 40, 40), (70, 33, 17)]
    plans = []
    for nk, nw, W in grids:
        wl = inp.small_grid(nk, nw, support_w=W)
        bis, _ = _bispec(wl, "separable", "seeded")
        plans.append(_plan(lib, wl, bis))
        lib.srm3_plan_set_mfma_shape(plans[-1], shape)
    wg = inp.small_grid(16, 32)
    plans.append(lib.srm3_plan(wg.grid_dict(), wg.spectrum(), None, "fp32"))
    wk = inp.small_grid(16, 40)
    pk = lib.plan_from_workload(wk, "fp32")
    lib.srm3_plan_set_algorithm(pk, "kappa_fft")
    plans.append(pk)
    reqs, singles = [], []
    for i in range(10):
        plan = plans[i % len(plans)]
        seed = 900 + i
        one = torch.empty((1,) + plan.field_shape, dtype=torch.float32, device="cuda")
        lib.srm3_generate(plan, [seed], one)
        singles.append(one[0])
        reqs.append(dict(plan=plan, seed=seed, out=torch.zeros(plan.field_shape, dtype=torch.float32, device="cuda")))
    print("[gpu] mfma server", flush=True)
    srv = lib.srm3.Server("fp32", max_active=4, hbm_budget=1 << 30, pair_kernel="mfma", mfma_shape=shape)
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
    wl = inp.small_grid(8, 16)
    bis, _ = _bispec(wl, "separable", "seeded")
    vec = lib.srm3_plan(wl.grid_dict(), wl.spectrum(), bis, "fp32")
    out = torch.empty(vec.field_shape, dtype=torch.float32, device="cuda")
    with pytest.raises(lib.Srm3Error) as ei:
        srv.submit(vec, 1, out)
    assert ei.value.status == 5
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3.Server("fp32", max_active=2, hbm_budget=1 << 28, pair_kernel=7)
    assert ei.value.status == 1
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3.Server("fp32", max_active=2, hbm_budget=1 << 28, pair_kernel="mfma", mfma_shape=3)
    assert ei.value.status == 1
