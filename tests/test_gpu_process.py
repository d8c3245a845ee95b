"""The 1-D stochastic process u(t) (Section 3) on the GPU against the FP64
process oracle, through the C-ABI (srm3_process_plan): coefficients and fields
within FP64 1e-10 / FP32 2e-5 relative L2, the negative-frequency columns
exactly zero, both pair-sum algorithms, batch invariance, the full-size
4096-frequency workload, batches and the server."""
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


def _inputs(oracle_mod, wl, kind, beta_mode, seed=3):
    """(bispectrum dict for the library, oracle ProcessProblem)."""
    W = wl.support_w
    bis = dict(kind=kind, support_w=W, cap=wl.cap, beta_mode=beta_mode, beta_seed=wl.beta_seed)
    if kind == "separable":
        bis["g2"] = wl.g2()
        b2 = wl.b2_dense()
    else:
        b2 = inp.random_b2_quadrant(W, seed, scale=0.3)
        bis["b2"] = b2
    if beta_mode == "table":
        beta = inp.random_beta_quadrant(W, seed + 1)
        bis["beta"] = beta
    elif beta_mode == "zero":
        beta = oracle_mod.process_biphase(W, None)
    else:
        beta = oracle_mod.process_biphase(W, wl.beta_seed)
    P = oracle_mod.ProcessProblem(wl.n, W, wl.d_omega, wl.spectrum(), b2, beta, wl.cap)
    return bis, P


def _run(lib, plan, wl, seeds):
    torch = _torch()
    cdt = torch.complex128 if plan.precision == lib.SRM3_FP64 else torch.complex64
    C = torch.empty((len(seeds),) + plan.coeff_shape, dtype=cdt, device="cuda")
    lib.srm3_coefficients(plan, seeds, C)
    u = torch.empty((len(seeds), 1, wl.n_t), dtype=plan.real_dtype, device="cuda")
    lib.srm3_generate(plan, seeds, u)
    torch.cuda.synchronize()
    return C.to(torch.complex128).cpu().numpy()[:, 0, :], u.double().cpu().numpy()[:, 0, :]


CASES = [
    # n, W, n_t, kind, beta_mode, batch
    (64, 64, 128, "separable", "seeded", 3),
    (100, 37, 256, "dense", "table", 3),         # truncated support
    (300, 300, 1024, "separable", "seeded", 20),  # several column tiles, several row tiles of realizations
    (33, 33, 128, "dense", "zero", 9),            # odd n, beta == 0, a ragged row tile
    (2, 1, 4, "separable", "seeded", 2),          # one support frequency
    (1, 1, 1, "dense", "seeded", 1),              # a single frequency
]


@pytest.mark.parametrize("algorithm", ["kappa_fft", "direct", "mfma"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}w{c[1]}_{c[3]}_{c[4]}_b{c[5]}" for c in CASES])
def test_small_processes_match_oracle(lib, oracle_mod, case, precision, algorithm):
    n, W, nt, kind, beta_mode, batch = case
    wl = inp.small_process(n, support_w=W, n_t=nt, batch=batch, seed_base=40)
    print(f"[gpu] process {case} {precision} {algorithm}", flush=True)
    bis, P = _inputs(oracle_mod, wl, kind, beta_mode)
    plan = lib.srm3_process_plan(wl.grid_dict(), wl.spectrum(), bis, precision)
    lib.srm3_plan_set_algorithm(plan, algorithm)
    seeds = wl.seeds()
    C, u = _run(lib, plan, wl, seeds)
    assert np.all(C[:, :n - 1] == 0)
    for r, s in enumerate(seeds):
        Cref = P.coefficients(seed=int(s))
        ref = oracle_mod.process_field(Cref, nt)
        if np.linalg.norm(Cref) == 0:
            assert np.all(C[r] == 0) and np.all(u[r] == 0)
            continue
        assert _rel(C[r, n - 1:], Cref) <= TOL[precision], r
        assert _rel(u[r], ref) <= TOL[precision], r


def test_terms_and_batch_invariance(lib):
    torch = _torch()
    wl = inp.small_process(200, support_w=150, batch=17, seed_base=7)
    plan = lib.process_plan_from_workload(wl, "fp32")
    expect = sum(max(0, k // 2 - max(0, k - 150 + 1) + 1) for k in range(200))
    assert lib.srm3_pair_terms(plan) == expect
    assert lib.srm3_algorithm_terms(plan) == expect
    seeds = wl.seeds()
    _, u = _run(lib, plan, wl, seeds)
    _, one = _run(lib, plan, wl, [int(seeds[13])])
    assert np.array_equal(one[0], u[13])
    # the direct form gives the same numbers to rounding
    lib.srm3_plan_set_algorithm(plan, "direct")
    _, ud = _run(lib, plan, wl, seeds)
    assert _rel(ud, u) <= 2e-5
    del torch


def test_gaussian_process_and_new_spectrum(lib, oracle_mod):
    wl = inp.small_process(128, batch=2, seed_base=3)
    plan = lib.srm3_process_plan(wl.grid_dict(), wl.spectrum(), None, "fp64")
    assert lib.srm3_pair_terms(plan) == 0
    P = oracle_mod.ProcessProblem(wl.n, 1, wl.d_omega, wl.spectrum(), np.zeros((1, 1)),
                                  oracle_mod.process_biphase(1, None), 0.0)
    C, u = _run(lib, plan, wl, wl.seeds())
    for r, s in enumerate(wl.seeds()):
        Cref = P.coefficients(seed=int(s))
        assert _rel(C[r, wl.n - 1:], Cref) <= 1e-12
        assert _rel(u[r], oracle_mod.process_field(Cref, wl.n_t)) <= 1e-12
    # replace the spectrum (one-sided) on a 3rd-order plan
    S2 = inp.random_process_spectrum(wl.n, 9)
    bis, _ = _inputs(oracle_mod, wl, "separable", "seeded")
    p3 = lib.srm3_process_plan(wl.grid_dict(), wl.spectrum(), bis, "fp64")
    lib.srm3_set_spectrum(p3, S2)
    P2 = oracle_mod.ProcessProblem(wl.n, wl.support_w, wl.d_omega, S2, wl.b2_dense(),
                                   oracle_mod.process_biphase(wl.support_w, wl.beta_seed), wl.cap)
    C2, _ = _run(lib, p3, wl, wl.seeds())
    assert _rel(C2[1, wl.n - 1:], P2.coefficients(seed=int(wl.seeds()[1]))) <= 1e-10


def test_process_argument_errors(lib):
    wl = inp.small_process(16)
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3_process_plan(dict(n_omega=16, d_omega=0.1, n_t=16), wl.spectrum(), None, "fp32")
    assert ei.value.status == 1            # n_t < 2 n_omega - 1
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3_process_plan(wl.grid_dict(), wl.spectrum(), dict(kind="separable", g2=np.ones(17),
                                                                  support_w=17), "fp32")
    assert ei.value.status == 1            # support above n_omega
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3_process_plan(wl.grid_dict(), wl.spectrum(),
                              dict(kind="separable", g2=np.full(16, 0.9), support_w=16, cap=0.0), "fp32")
    assert ei.value.status == 2            # pure spectrum not positive
    bad = wl.spectrum().copy()
    bad[3] = -1.0
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3_process_plan(wl.grid_dict(), bad, None, "fp32")
    assert ei.value.status == 1


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_full_size_4096_frequencies(lib, oracle_mod, precision):
    """The 4096-frequency, 8192-point workload at its full batch: whole
    coefficient vectors and fields of sampled realizations against the oracle."""
    torch = _torch()
    wl = inp.P1 if precision == "fp32" else inp.P1.with_(batch=512)
    print(f"[gpu] process p1 {precision} batch {wl.batch}", flush=True)
    bis, P = _inputs(oracle_mod, wl, "separable", "seeded")
    plan = lib.srm3_process_plan(wl.grid_dict(), wl.spectrum(), bis, precision)
    seeds = wl.seeds()
    u = torch.empty((wl.batch, 1, wl.n_t), dtype=plan.real_dtype, device="cuda")
    lib.srm3_generate(plan, seeds, u)
    cdt = torch.complex128 if precision == "fp64" else torch.complex64
    C = torch.empty((wl.batch,) + plan.coeff_shape, dtype=cdt, device="cuda")
    lib.srm3_coefficients(plan, seeds, C)
    torch.cuda.synchronize()
    for r in (0, wl.batch - 1):
        Cref = P.coefficients(seed=int(seeds[r]))
        got = C[r, 0, wl.n - 1:].to(torch.complex128).cpu().numpy()
        assert _rel(got, Cref) <= TOL[precision], r
        ref = oracle_mod.process_field(Cref, wl.n_t)
        assert _rel(u[r, 0].double().cpu().numpy(), ref) <= TOL[precision], r


def test_process_plans_in_batches_and_the_server(lib):
    torch = _torch()
    wls = [inp.small_process(256, batch=1), inp.small_process(1000, support_w=400, batch=1)]
    plans = [lib.process_plan_from_workload(w, "fp32") for w in wls]
    reqs, singles = [], []
    for i in range(8):
        w, p = wls[i % 2], plans[i % 2]
        out = torch.empty((1, w.n_t), dtype=torch.float32, device="cuda")
        one = torch.empty((1, 1, w.n_t), dtype=torch.float32, device="cuda")
        lib.srm3_generate(p, [90 + i], one)
        reqs.append(dict(plan=p, seed=90 + i, out=out))
        singles.append(one[0])
    print("[gpu] process batch", flush=True)
    b = lib.Batch(reqs, flags=lib.SRM3_BATCH_GRAPH)
    for _ in range(2):
        for r in reqs:
            r["out"].zero_()
        b.run()
        torch.cuda.synchronize()
        for r, s in zip(reqs, singles):
            assert torch.equal(r["out"], s)
    print("[gpu] process server", flush=True)
    srv = lib.srm3.Server("fp32", max_active=4, hbm_budget=1 << 30)
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
