"""Quasi-two-dimensional plans (grid (N1, 1, N2), tight trap along the middle
axis) on the GPU against the oracle's quasi-2D equation: both dipole
orientations, imaginary and real time, FP64 and FP32 (relative L2 over the
plane, 1e-12 and 1e-5), observables, a change of the tight trap, the ground
state driver and the calls a quasi-2D plan refuses."""
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


def _case(n2, d2, trap3, g, gd, dt, imag, dipoles):
    """(library grid, spacings, trap) and the oracle's Params2D of one case."""
    n = (n2[0], 1, n2[1])
    d = (d2[0], 1.0, d2[1])
    p = O.Params2D(n2, d2, dt, (trap3[0], trap3[2]), trap3[1], g, gd, imag, dipoles)
    return n, d, p


def _psi0(n2, d2, trap3, seed):
    """A seeded noisy Gaussian on the plane, unit norm over the plane."""
    xa = (np.arange(n2[0]) - n2[0] // 2) * d2[0]
    xb = (np.arange(n2[1]) - n2[1] // 2) * d2[1]
    psi = np.exp(-0.5 * trap3[0] * xa[:, None] ** 2 - 0.5 * trap3[2] * xb[None, :] ** 2)
    rng = np.random.default_rng(seed)
    psi = psi + 1e-3 * rng.uniform(-1, 1, size=psi.shape)
    psi = psi.astype(np.complex128)
    return psi / np.sqrt(np.sum(np.abs(psi) ** 2) * d2[0] * d2[1])


SHAPES = [((64, 48), (0.3, 0.35)), ((96, 128), (0.25, 0.2))]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dipoles", ["perp", "inplane"])
@pytest.mark.parametrize("real_time", [False, True], ids=["imag", "real"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s[0])))
def test_q2d_steps_match_oracle(env, shape, real_time, dipoles, prec):
    torch, dg = env
    n2, d2 = shape
    trap3 = (1.0, 6.0, 1.4)
    n, d, p = _case(n2, d2, trap3, 30.0, 12.0, 0.004, not real_time, dipoles)
    psi0 = _psi0(n2, d2, trap3, 51)
    _say(f"q2d {n2} {dipoles} {'real' if real_time else 'imag'} {prec}")
    plan = dg.Plan(n, d, p.dt, trap3, p.g, p.gd, real_time=real_time, dtype=_dtype(torch, prec), q2d=dipoles)
    assert not plan.fused_y
    psi = plan.new_state(psi0.reshape(n))
    plan.step(psi, 8)
    got = psi.cpu().numpy().astype(np.complex128).reshape(n2)
    ref = O.q2d_evolve(p, psi0, 8)
    err = _rel(got, ref)
    _say(f"  rel L2 {err:.3e}")
    assert err < TOL[prec]
    o = plan.observables(psi)
    r = O.q2d_observables(p, got)  # the oracle's observables of the GPU state
    for k in ("norm", "mu", "energy", "e_kin", "e_trap", "e_contact", "e_dd"):
        assert abs(o[k] - r[k]) <= (1e-12 if prec == "f64" else 2e-6) * max(1.0, abs(r[k])), (k, o[k], r[k])
    assert o["rms"][1] == 0.0
    assert abs(o["rms"][0] - r["rms"][0]) < 1e-10 and abs(o["rms"][2] - r["rms"][1]) < 1e-10
    plan.close()


def test_q2d_potential_matches_oracle(env):
    torch, dg = env
    n2, d2 = (48, 64), (0.3, 0.25)
    for dipoles in ("perp", "inplane"):
        n, d, p = _case(n2, d2, (1.0, 4.0, 1.0), 0.0, 1.0, 0.01, True, dipoles)
        plan = dg.Plan(n, d, p.dt, (1.0, 4.0, 1.0), 0.0, 1.0, dtype=torch.complex128, q2d=dipoles)
        psi0 = _psi0(n2, d2, (1.0, 4.0, 1.0), 52)
        phi = plan.potential(plan.new_state(psi0.reshape(n))).cpu().numpy().reshape(n2)
        ref = O.q2d_potential(p, np.abs(psi0) ** 2)
        err = float(np.max(np.abs(phi - ref)) / np.max(np.abs(ref)))
        _say(f"q2d potential {dipoles}: {err:.3e}")
        assert err < 1e-13
        plan.close()


def test_q2d_tight_trap_change_rebuilds_kernel_and_coupling(env):
    torch, dg = env
    n2, d2 = (64, 48), (0.3, 0.35)
    n, d, p = _case(n2, d2, (1.0, 9.0, 1.4), 30.0, 12.0, 0.004, True, "inplane")
    plan = dg.Plan(n, d, p.dt, (1.0, 3.0, 1.4), p.g, p.gd, dtype=torch.complex128, q2d="inplane")
    plan.set("lambda", 9.0)
    psi0 = _psi0(n2, d2, (1.0, 9.0, 1.4), 53)
    psi = plan.new_state(psi0.reshape(n))
    plan.step(psi, 6)
    err = _rel(psi.cpu().numpy().reshape(n2), O.q2d_evolve(p, psi0, 6))
    _say(f"q2d after the tight trap change: {err:.3e}")
    assert err < 1e-12
    with pytest.raises(dg.DgpeError):
        plan.set("lambda", 0.0)
    plan.close()


def test_q2d_ground_state_driver(env):
    """The driver on a quasi-2D plan runs exactly the plain steps it reports."""
    torch, dg = env
    n2, d2 = (48, 64), (0.35, 0.3)
    trap3 = (1.0, 8.0, 1.5)
    n, d, p = _case(n2, d2, trap3, 20.0, 8.0, 0.01, True, "perp")
    psi0 = _psi0(n2, d2, trap3, 54)
    plan = dg.Plan(n, d, p.dt, trap3, p.g, p.gd, dtype=torch.complex128, q2d="perp")
    psi = plan.new_state(psi0.reshape(n))
    out = plan.ground_state(psi, tol=1e-8, max_steps=4000, check_every=20)
    assert out["converged"] and out["steps"] < 4000
    ref = O.q2d_evolve(p, psi0, out["steps"])
    err = _rel(psi.cpu().numpy().reshape(n2), ref)
    mu = O.q2d_observables(p, ref)["mu"]
    _say(f"q2d ground state: {out['steps']} steps, mu {out['observables']['mu']:.12f} (oracle {mu:.12f}), "
         f"rel L2 {err:.3e}")
    assert err < 1e-11
    assert abs(out["observables"]["mu"] - mu) < 1e-11 * abs(mu)
    plan.close()


def test_q2d_refusals(env):
    torch, dg = env
    with pytest.raises(dg.DgpeError) as e:
        dg.Plan((32, 2, 32), (0.3, 0.3, 0.3), 0.01, (1, 4, 1), 1.0, 1.0, q2d="perp")
    assert e.value.status == 2
    with pytest.raises(dg.DgpeError) as e:
        dg.Plan((32, 1, 32), (0.3, 1.0, 0.3), 0.01, (1, 0.0, 1), 1.0, 1.0, q2d="perp")
    assert e.value.status == 1
    plan = dg.Plan((32, 1, 32), (0.3, 1.0, 0.3), 0.01, (1, 4, 1), 1.0, 1.0, real_time=True, q2d="inplane")
    with pytest.raises(dg.DgpeError) as e:
        plan.set("scheme", "strang")
    assert e.value.status == 6
    psi = plan.new_state(_psi0((32, 32), (0.3, 0.3), (1, 4, 1), 55).reshape(32, 1, 32))
    with pytest.raises(dg.DgpeError) as e:
        plan.adjoint(psi, np.ones(3), ckpt_every=1)
    assert e.value.status == 6
    plan.close()
