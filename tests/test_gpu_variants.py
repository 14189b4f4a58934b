"""Variants of the method on the GPU against the FP64 oracle: the symmetric
(Strang) step, the imaginary-time ground-state driver and the binary density
file.

Tolerances as for the plain step: relative L2 over the whole grid, FP64 <= 1e-12
and FP32 <= 1e-5.
"""
import os

import numpy as np
import pytest

from oracle import dgpe_oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1610_05329_amd as dg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dg.load()
    return torch, dg


def _dtype(torch, prec):
    return torch.complex128 if prec == "f64" else torch.complex64


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _say(*a):
    print(*a, flush=True)


# generic passes (16 x 24 x 32: no compiled split for Nz/2 = 16 with 24-line
# blocks) and the compiled fast path (8 x 32 x 64, 32 x 32 x 128)
STRANG_SHAPES = [
    ((16, 24, 32), (0.4, 0.35, 0.3)),
    ((8, 32, 64), (0.4, 0.35, 0.2)),
    ((32, 32, 128), (0.3, 0.3, 0.12)),
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("real_time", [False, True], ids=["imag", "real"])
@pytest.mark.parametrize("shape", STRANG_SHAPES, ids=lambda s: "x".join(map(str, s[0])))
def test_strang_steps_match_oracle(env, shape, real_time, prec):
    """Six symmetric steps with a varying trap amplitude (real time: the
    merged half steps carry the mean amplitude of neighbouring steps)."""
    torch, dg = env
    n, d = shape
    cfg = W.Config("t", n, d, 0.004, (1.0, 1.2, 1.6), 25.0, 9.0, not real_time, 6, noise=1e-3, seed=31)
    psi0 = W.noisy_gaussian(cfg)
    amp = np.random.default_rng(32).uniform(0.9, 1.1, size=cfg.steps)
    _say(f"strang {n} {'real' if real_time else 'imag'} {prec}")
    plan = dg.Plan(n, d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=real_time, dtype=_dtype(torch, prec))
    plan.set("scheme", "strang")
    # imaginary time on grids with the compiled fused z pass: the fused y schedule
    assert plan.fused_y == (not real_time and n != (16, 24, 32))
    psi = plan.new_state(psi0)
    plan.step(psi, cfg.steps, amp)
    got = psi.cpu().numpy().astype(np.complex128)
    p = O.Params.from_config(cfg)
    ref = O.evolve(p, psi0, cfg.steps, amp, scheme="strang")
    err = _rel(got, ref)
    lie = O.evolve(p, psi0, cfg.steps, amp)
    _say(f"  rel L2 {err:.3e} (first-order step differs by {_rel(lie, ref):.1e})")
    assert err < TOL[prec]
    assert _rel(lie, ref) > 1e-4  # the two steps differ far beyond the FP32 bound
    plan.close()


@pytest.mark.parametrize("real_time", [False, True], ids=["imag", "real"])
def test_strang_single_step_calls_match_one_call(env, real_time):
    """One call of four steps and four calls of one step give the same state to
    rounding (a call of several real-time steps joins the half steps of
    neighbouring steps into one phase)."""
    torch, dg = env
    n, d = (8, 32, 64), (0.4, 0.35, 0.2)
    cfg = W.Config("t", n, d, 0.004, (1.0, 1.2, 1.6), 25.0, 9.0, not real_time, 4, noise=1e-3, seed=33)
    plan = dg.Plan(n, d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=real_time, dtype=torch.complex128)
    plan.set("scheme", 1)
    a = plan.new_state(W.noisy_gaussian(cfg))
    b = a.clone()
    plan.step(a, 4)
    for _ in range(4):
        plan.step(b, 1)
    err = _rel(a.cpu().numpy(), b.cpu().numpy())
    _say(f"strang one call vs single steps ({'real' if real_time else 'imag'}): {err:.3e}")
    assert err < 1e-13
    plan.close()


def test_strang_refuses_the_adjoint(env):
    torch, dg = env
    n, d = (16, 24, 32), (0.4, 0.35, 0.3)
    plan = dg.Plan(n, d, 0.004, (1.0, 1.0, 1.0), 10.0, 3.0, real_time=True)
    plan.set("scheme", "strang")
    psi = plan.new_state(W.gaussian_state(n, d, (1.0, 1.0, 1.0)))
    with pytest.raises(dg.DgpeError) as e:
        plan.adjoint(psi, np.ones(3), ckpt_every=1)
    assert e.value.status == 6
    plan.close()


@pytest.mark.parametrize("scheme", ["lie", "strang"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ground_state_driver_matches_oracle(env, prec, scheme):
    """The driver stops at the same check as the oracle's (FP64) and its state
    matches the oracle's after the same number of steps."""
    torch, dg = env
    n, d = (16, 18, 24), (0.5, 0.5, 0.4)
    cfg = W.Config("t", n, d, 0.01, (1.0, 1.3, 1.7), 15.0, 6.0, True, 0, noise=1e-3, seed=34)
    psi0 = W.noisy_gaussian(cfg)
    tol = 1e-9 if prec == "f64" else 1e-6
    every = 10
    plan = dg.Plan(n, d, cfg.dt, cfg.trap, cfg.g, cfg.gd, dtype=_dtype(torch, prec))
    plan.set("scheme", scheme)
    psi = plan.new_state(psi0)
    out = plan.ground_state(psi, tol=tol, max_steps=3000, check_every=every)
    got = psi.cpu().numpy().astype(np.complex128)
    p = O.Params.from_config(cfg)
    ref, steps, rate, mu = O.ground_state(p, psi0, tol, 3000, every, scheme=scheme)
    _say(f"ground state {scheme} {prec}: steps {out['steps']} (oracle {steps}), "
         f"dmu/step {out['dmu_per_step']:.2e} (oracle {rate:.2e}), mu {out['observables']['mu']:.12f} "
         f"(oracle {mu:.12f})")
    assert out["converged"] and out["dmu_per_step"] < tol
    if prec == "f64":
        assert out["steps"] == steps
        assert abs(out["dmu_per_step"] - rate) < 1e-12
        assert abs(out["observables"]["mu"] - mu) < 1e-12 * abs(mu)
        assert _rel(got, ref) < TOL[prec]
    else:
        # FP32 may stop one check away from the FP64 oracle; compare with the
        # oracle after the FP32 run's own step count
        assert abs(out["steps"] - steps) <= every
        ref32 = O.evolve(p, psi0, out["steps"], scheme=scheme)
        assert _rel(got, ref32) < TOL[prec]
        assert abs(out["observables"]["mu"] - mu) < 1e-5 * abs(mu)
    plan.close()


@pytest.mark.parametrize("scheme", ["lie", "strang"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ground_state_driver_graph_replays_match_plain_steps(env, prec, scheme):
    """The driver captures its check_every steps as a HIP graph on the first
    chunk and replays it for the next ones, with the observables (eager work
    that synchronises) between replays: after 1 to 4 chunks the state equals
    the same number of plain step calls, bit for bit."""
    torch, dg = env
    n, d = (16, 32, 64), (0.5, 0.4, 0.3)
    cfg = W.Config("t", n, d, 0.01, (1.0, 1.3, 1.7), 15.0, 6.0, True, 0, noise=1e-3, seed=35)
    psi0 = W.noisy_gaussian(cfg)
    every = 5
    plan = dg.Plan(n, d, cfg.dt, cfg.trap, cfg.g, cfg.gd, dtype=_dtype(torch, prec))
    plan.set("scheme", scheme)
    for chunks in (1, 2, 3, 4):
        psi = plan.new_state(psi0)
        out = plan.ground_state(psi, tol=1e-300, max_steps=chunks * every, check_every=every)
        assert out["steps"] == chunks * every and not out["converged"]
        ref = plan.new_state(psi0)
        for _ in range(chunks):
            plan.step(ref, every)
        assert torch.equal(psi, ref), f"{chunks} chunks"
    plan.close()


def test_ground_state_driver_arguments(env):
    torch, dg = env
    n, d = (16, 24, 32), (0.4, 0.35, 0.3)
    plan = dg.Plan(n, d, 0.004, (1.0, 1.0, 1.0), 10.0, 3.0)
    psi = plan.new_state(W.gaussian_state(n, d, (1.0, 1.0, 1.0)))
    for kw in ({"tol": 0.0}, {"tol": float("nan")}, {"max_steps": -1}, {"check_every": 0}):
        with pytest.raises(dg.DgpeError) as e:
            plan.ground_state(psi, **kw)
        assert e.value.status == 1
    # no step allowed: no step taken, the rate is undefined (infinite)
    out = plan.ground_state(psi, tol=1e-8, max_steps=0)
    assert out["steps"] == 0 and not out["converged"] and out["dmu_per_step"] == float("inf")
    # a step cap below convergence: stops there, not converged
    out = plan.ground_state(psi, tol=1e-14, max_steps=25, check_every=10)
    assert out["steps"] == 25 and not out["converged"]
    plan.set("real_time", 1)
    with pytest.raises(dg.DgpeError) as e:
        plan.ground_state(psi)
    assert e.value.status == 6
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [((12, 18, 24), (0.5, 0.45, 0.4)), ((64, 48, 32), (0.2, 0.25, 0.3))],
                         ids=lambda s: "x".join(map(str, s[0])))
def test_binary_density_file_matches_oracle(env, tmp_path, shape, prec):
    """The density file of a stepped state read back as float64 [x][y][z]: it is
    |psi|^2 of the returned state and matches the oracle's density after the
    same steps."""
    torch, dg = env
    n, d = shape
    cfg = W.Config("t", n, d, 0.004, (1.0, 1.2, 1.6), 20.0, 8.0, False, 3, noise=1e-3, seed=35)
    psi0 = W.noisy_gaussian(cfg)
    plan = dg.Plan(n, d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=True, dtype=_dtype(torch, prec))
    psi = plan.new_state(psi0)
    plan.step(psi, cfg.steps)
    path = tmp_path / "density.bin"
    plan.write_density(psi, path)
    assert os.path.getsize(path) == 8 * n[0] * n[1] * n[2]
    dens = np.fromfile(path, dtype="<f8").reshape(n)
    host = psi.cpu().numpy().astype(np.complex128)
    own = host.real ** 2 + host.imag ** 2
    tol_own = 1e-15 if prec == "f64" else 2e-7
    assert np.max(np.abs(dens - own)) <= tol_own * np.max(own)
    dev = plan.density(psi).cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(dev, dens)
    ref = np.abs(O.evolve(O.Params.from_config(cfg), psi0, cfg.steps)) ** 2
    err = _rel(dens, ref)
    _say(f"density file {n} {prec}: rel L2 vs oracle {err:.3e}")
    assert err < TOL[prec]
    # the x-plane at index i starts at byte 8 i Ny Nz
    i = n[0] // 3
    with open(path, "rb") as f:
        f.seek(8 * i * n[1] * n[2])
        plane = np.frombuffer(f.read(8 * n[1] * n[2]), dtype="<f8").reshape(n[1], n[2])
    np.testing.assert_array_equal(plane, dens[i])
    with pytest.raises(dg.DgpeError):
        plan.write_density(psi, tmp_path / "missing_dir" / "x.bin")
    plan.close()
