"""srm3_generate issues only kernel launches on the caller's stream once its
workspace exists (no allocation, no memset, no host synchronisation), so a
caller may capture it in a graph: every replay equals the eager result, with
the program's own eager work and synchronisations between replays."""
import pytest

import srm3_inputs as inp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    import paper_2310_03979_amd as p
    p.load()
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    return p


def _plans(lib):
    wl = inp.small_grid(32, 64, batch=3, seed_base=5)
    direct = lib.plan_from_workload(wl, "fp32")
    kfft = lib.plan_from_workload(wl, "fp32")
    lib.srm3_plan_set_algorithm(kfft, "kappa_fft")
    fft2d = lib.plan_from_workload(wl, "fp32", beta_mode="zero")
    lib.srm3_plan_set_algorithm(fft2d, "fft2d")
    pw = inp.small_process(256, batch=3)
    proc = lib.process_plan_from_workload(pw, "fp32")
    mfma = lib.plan_from_workload(wl, "fp32")
    lib.srm3_plan_set_algorithm(mfma, "mfma")
    return [("direct", wl, direct), ("kappa_fft", wl, kfft), ("fft2d", wl, fft2d), ("process", pw, proc),
            ("mfma", wl, mfma)]


@pytest.mark.parametrize("which", ["direct", "kappa_fft", "fft2d", "process", "mfma"])
def test_generate_replays_from_a_graph(lib, which):
    import torch
    name, wl, plan = [p for p in _plans(lib) if p[0] == which][0]
    print(f"[gpu] graph capture {name}", flush=True)
    seeds = wl.seeds()
    shape = (len(seeds),) + plan.field_shape
    ref = torch.empty(shape, dtype=torch.float32, device="cuda")
    lib.srm3_generate(plan, seeds, ref)          # eager; also sizes the workspace
    torch.cuda.synchronize()
    out = torch.zeros(shape, dtype=torch.float32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        lib.srm3_generate(plan, seeds, out)      # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        lib.srm3_generate(plan, seeds, out)
    junk = torch.randn(1 << 20, device="cuda")
    for _ in range(3):
        out.zero_()
        junk.mul_(1.0001).add_(0.5)              # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
