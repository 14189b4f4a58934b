"""Host-side logic that needs no GPU: knot interpolation of the trap amplitude,
the benchmark's one-GPU guard, and the separation of the product path from the
oracle."""
import os
import re
import subprocess
import sys

import numpy as np

from paper_1610_05329_amd import knot_matrix

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_knot_matrix_interpolates_piecewise_linearly():
    nk, nsteps, dt = 40, 400, 0.002
    W = knot_matrix(nk, nsteps, dt)
    assert W.shape == (nsteps + 1, nk)
    assert np.allclose(W.sum(axis=1), 1.0, atol=1e-15)
    knots = np.random.default_rng(4).uniform(0.8, 1.2, nk)
    a = W @ knots
    T = nsteps * dt
    tk = np.arange(nk) * T / (nk - 1)
    t = np.arange(nsteps + 1) * dt
    assert np.max(np.abs(a - np.interp(t, tk, knots))) < 1e-14
    assert abs(a[0] - knots[0]) < 1e-15 and abs(a[-1] - knots[-1]) < 1e-14


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_product_path_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_1610_05329_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\boracle\b", text), f
                assert "dgpe_oracle" not in text, f
