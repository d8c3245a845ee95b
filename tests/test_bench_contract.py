"""bench.py's command-line contract on a host without a GPU, and the
workload recipes it measures (CPU only)."""
import math
import os
import subprocess
import sys

import numpy as np

import srm3_inputs as inp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=300)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_no_gpu_fails_loudly():
    r = _bench("--steps", "1", "--warmup", "0")
    assert r.returncode != 0
    assert r.stdout.strip() == ""          # no JSON line without a measurement


def test_bridge_grid_of_section_5():
    wl = inp.bridge()
    assert (wl.n_kappa, wl.n_omega, wl.n_x, wl.n_t) == (256, 128, 1024, 2048)
    assert math.isclose(wl.d_kappa, 2 * math.pi / 628.0)
    assert math.isclose(wl.d_omega, math.pi / 127)
    S = wl.spectrum()
    # the printed closed form at one line, written out
    kk, kw = 3, 5
    w, kap = kw * wl.d_omega, kk * wl.d_kappa
    us = 0.4 * 40.0 / math.log(50.0 / 0.03)
    a = 10.0 * w / (math.pi * 40.0)
    ref = 0.5 * 200.0 / (2 * math.pi) * us ** 2 * (50.0 / 40.0) / (1 + 50 * w * 50.0 / (2 * math.pi * 40.0)) ** (5 / 3) \
        * a / (kap ** 2 + a ** 2)
    assert math.isclose(S[kk, kw + wl.n_omega - 1], ref, rel_tol=1e-13)
    assert np.all(S[:, wl.n_omega - 1] == 0) and np.array_equal(S, S[:, ::-1])


def test_process_workload():
    wl = inp.P1
    assert (wl.n, wl.support_w, wl.n_t, wl.batch) == (4096, 4096, 8192, 4096)
    S = wl.spectrum()
    assert S[0] == 0 and np.all(S[1:] > 0) and np.all(np.diff(S[1:]) < 0)
