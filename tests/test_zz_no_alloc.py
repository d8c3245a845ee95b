"""The allocation-free generation entry point (srm3_generate_noalloc) through
the C-ABI: its fields equal those of srm3_generate bitwise, and the FP64
oracle's within the tolerances (FP64 <= 1e-10, FP32 <= 2e-5 relative L2), on
calls in a row whose inputs shrink (the scratch array keeps the previous
call's contents); a workspace beyond the array is refused."""
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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# (n_kappa, n_omega, support, precision, algorithm, batch), largest first
CALLS = [
    (70, 300, 200, "fp32", "mfma", 3),
    (17, 9, 9, "fp64", "direct", 2),
    (40, 64, 33, "fp32", "kappa_fft", 2),
    (5, 40, 40, "fp64", "mfma", 1),
]


def test_noalloc_equals_generate_on_shrinking_calls(lib, oracle_mod):
    import torch
    for nk, nw, W, precision, algorithm, batch in CALLS:
        print(f"[gpu] noalloc {nk}x{nw} w{W} {precision} {algorithm} batch {batch}", flush=True)
        wl = inp.small_grid(nk, nw, support_w=W, batch=batch, seed_base=930 + nk)
        plan = lib.plan_from_workload(wl, precision)
        lib.srm3_plan_set_algorithm(plan, algorithm)
        seeds = wl.seeds()
        ref = torch.empty((batch,) + plan.field_shape, dtype=plan.real_dtype, device="cuda")
        lib.srm3_generate(plan, seeds, ref)
        got = torch.full_like(ref, float("nan"))
        lib.srm3_generate_noalloc(plan, seeds, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        P = oracle_mod.Problem.from_workload(wl)
        u = got.double().cpu().numpy()
        for r, s in enumerate(seeds):
            assert _rel(u[r], oracle_mod.field(P.coefficients(seed=int(s)), wl.n_x, wl.n_t)) <= TOL[precision]


def test_noalloc_refuses_workspace_beyond_scratch(lib):
    import torch
    wl = inp.C1
    plan = lib.plan_from_workload(wl, "fp32")
    out = torch.empty((wl.batch,) + plan.field_shape, dtype=torch.float32, device="cuda")
    with pytest.raises(lib.Srm3Error) as ei:
        lib.srm3_generate_noalloc(plan, wl.seeds(), out)
    assert ei.value.status == 5
    assert "scratch" in lib.srm3_last_error()
    # one realization of the same grid fits
    one = torch.empty((1,) + plan.field_shape, dtype=torch.float32, device="cuda")
    ref = torch.empty_like(one)
    lib.srm3_generate(plan, wl.seeds()[:1], ref)
    lib.srm3_generate_noalloc(plan, wl.seeds()[:1], one)
    torch.cuda.synchronize()
    assert torch.equal(one, ref)
