"""Edge cases on the GPU against the oracle: the longest axes the library
accepts (1024 and 2048 points, along each axis in turn: generic FFT passes,
strided sweeps over 64 and 128 segments, blocks of more than 64 KB of LDS for
the z pass; a quasi-2D plane with a 2048-point axis), the smallest grids (4
points per axis: one partial segment per line) and a call with zero steps (the
state is left as it was)."""
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


def _run(env, n, d, real_time, prec, steps, seed):
    torch, dg = env
    cfg = W.Config("t", n, d, 0.002, (1.0, 1.1, 1.3), 20.0, 8.0, not real_time, steps, noise=1e-3,
                   seed=seed)
    psi0 = W.noisy_gaussian(cfg)
    plan = dg.Plan(n, d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=real_time, dtype=_dtype(torch, prec))
    psi = plan.new_state(psi0)
    plan.step(psi, steps)
    got = psi.cpu().numpy().astype(np.complex128)
    plan.close()
    ref = O.evolve(O.Params.from_config(cfg), psi0, steps)
    return _rel(got, ref)


LONGEST = [
    ((1024, 6, 8), (0.03, 0.5, 0.4)),
    ((6, 1024, 8), (0.5, 0.03, 0.4)),
    ((6, 8, 1024), (0.5, 0.4, 0.03)),
    ((2048, 6, 8), (0.015, 0.5, 0.4)),
    ((6, 2048, 8), (0.5, 0.015, 0.4)),
    ((6, 8, 2048), (0.5, 0.4, 0.015)),
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("real_time", [False, True], ids=["imag", "real"])
@pytest.mark.parametrize("shape", LONGEST, ids=lambda s: "x".join(map(str, s[0])))
def test_longest_axis_matches_oracle(env, shape, real_time, prec):
    n, d = shape
    err = _run(env, n, d, real_time, prec, 3, 21)
    print(f"longest axis {n} {'real' if real_time else 'imag'} {prec}: rel L2 {err:.3e}", flush=True)
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("real_time", [False, True], ids=["imag", "real"])
def test_quasi2d_longest_axis_matches_oracle(env, real_time, prec):
    torch, dg = env
    n2, d2, trap3 = (2048, 12), (0.015, 0.5), (1.0, 6.0, 1.4)
    n, d = (n2[0], 1, n2[1]), (d2[0], 1.0, d2[1])
    p = O.Params2D(n2, d2, 0.004, (trap3[0], trap3[2]), trap3[1], 30.0, 12.0, not real_time, "perp")
    xa = (np.arange(n2[0]) - n2[0] // 2) * d2[0]
    xb = (np.arange(n2[1]) - n2[1] // 2) * d2[1]
    psi0 = np.exp(-0.5 * trap3[0] * xa[:, None] ** 2 - 0.5 * trap3[2] * xb[None, :] ** 2)
    psi0 = psi0 + 1e-3 * np.random.default_rng(24).uniform(-1, 1, size=psi0.shape)
    psi0 = (psi0 / np.sqrt(np.sum(np.abs(psi0) ** 2) * d2[0] * d2[1])).astype(np.complex128)
    plan = dg.Plan(n, d, p.dt, trap3, p.g, p.gd, real_time=real_time, dtype=_dtype(torch, prec), q2d="perp")
    psi = plan.new_state(psi0.reshape(n))
    plan.step(psi, 4)
    got = psi.cpu().numpy().astype(np.complex128).reshape(n2)
    plan.close()
    err = _rel(got, O.q2d_evolve(p, psi0, 4))
    print(f"quasi-2D {n2} {'real' if real_time else 'imag'} {prec}: rel L2 {err:.3e}", flush=True)
    assert err < TOL[prec]


SMALLEST = [((4, 4, 4), (0.6, 0.6, 0.6)), ((4, 6, 12), (0.6, 0.5, 0.3))]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("real_time", [False, True], ids=["imag", "real"])
@pytest.mark.parametrize("shape", SMALLEST, ids=lambda s: "x".join(map(str, s[0])))
def test_smallest_grids_match_oracle(env, shape, real_time, prec):
    n, d = shape
    err = _run(env, n, d, real_time, prec, 4, 22)
    print(f"smallest grid {n} {'real' if real_time else 'imag'} {prec}: rel L2 {err:.3e}", flush=True)
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("real_time", [False, True], ids=["imag", "real"])
def test_zero_steps_leave_the_state(env, real_time, prec):
    torch, dg = env
    n, d = (16, 32, 64), (0.4, 0.3, 0.2)
    cfg = W.Config("t", n, d, 0.002, (1.0, 1.1, 1.3), 20.0, 8.0, not real_time, 0, noise=1e-3, seed=23)
    plan = dg.Plan(n, d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=real_time, dtype=_dtype(torch, prec))
    psi = plan.new_state(W.noisy_gaussian(cfg))
    before = psi.clone()
    plan.step(psi, 0)
    torch.cuda.synchronize()
    assert torch.equal(psi, before)
    plan.close()
