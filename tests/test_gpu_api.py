"""C ABI behaviour on the GPU: parameter changes, error reporting, the overlap
objective of the adjoint, and checkpoint-interval independence."""
import ctypes

import numpy as np
import pytest

from oracle import dgpe_oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1610_05329_amd as dg
    assert torch.cuda.is_available()
    dg.load()
    return torch, dg


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_parameter_changes_match_a_fresh_plan(env):
    """dgpe_plan_set (g, gd, trap, dt, time mode) gives the same steps as a plan
    created with the new values."""
    torch, dg = env
    n, d = (24, 32, 36), (0.4, 0.3, 0.3)
    psi0 = W.random_state(n, d, seed=41)
    a = dg.Plan(n, d, 0.004, (1.0, 1.0, 1.0), 10.0, 4.0, dtype=torch.complex128)
    for k, v in (("g", 22.0), ("gd", -7.0), ("nu", 1.3), ("lambda", 0.8), ("gamma", 2.0),
                 ("dt", 0.003), ("real_time", 1)):
        a.set(k, v)
    b = dg.Plan(n, d, 0.003, (1.3, 0.8, 2.0), 22.0, -7.0, real_time=True, dtype=torch.complex128)
    pa, pb = a.new_state(psi0), b.new_state(psi0)
    a.step(pa, 6)
    b.step(pb, 6)
    assert torch.equal(pa, pb)


def test_nonfinite_state_is_reported(env):
    torch, dg = env
    n, d = (16, 16, 16), (0.4,) * 3
    plan = dg.Plan(n, d, 0.01, (1, 1, 1), 1.0, 1.0, dtype=torch.complex128)
    psi = plan.new_state(W.random_state(n, d, seed=3))
    psi[3, 4, 5] = complex(float("nan"), 0.0)
    with pytest.raises(dg.DgpeError) as e:
        plan.observables(psi)
    assert e.value.status == 5  # DGPE_ENONFINITE


def test_invalid_calls_are_rejected(env):
    torch, dg = env
    n, d = (16, 16, 16), (0.4,) * 3
    imag = dg.Plan(n, d, 0.01, (1, 1, 1), 1.0, 1.0, dtype=torch.complex128)
    psi = imag.new_state(W.random_state(n, d, seed=5))
    with pytest.raises(dg.DgpeError) as e:
        imag.adjoint(psi, np.ones(4))
    assert e.value.status == 6  # DGPE_ESTATE: the adjoint needs real time
    with pytest.raises(dg.DgpeError):
        imag.set("dt", -1.0)
    with pytest.raises(dg.DgpeError):
        imag.set("real_time", 0.5)
    lib = imag.lib
    assert lib.dgpe_step(imag.handle, ctypes.c_void_p(psi.data_ptr()), -1, None) == 1
    bad = (ctypes.c_double * 2)(1.0, float("inf"))
    assert lib.dgpe_step(imag.handle, ctypes.c_void_p(psi.data_ptr()), 2, bad) == 1
    ms = (ctypes.c_double * 8)()
    assert lib.dgpe_step_profiled(imag.handle, ctypes.c_void_p(psi.data_ptr()), 2, bad, ms, None) == 1
    assert b"finite" in lib.dgpe_last_error()
    with pytest.raises(ValueError):
        imag.step_profiled(psi, 3, amp=np.ones(2))
    with pytest.raises(dg.DgpeError) as e:
        dg.Plan((20, 16, 16), d, 0.01, (1, 1, 1), 1.0, 1.0)
    assert e.value.status == 2


def _adjoint_errors(out, J, dJ_da, dJ_dt, lam0):
    """Relative errors of J, dJ/da (max norm), dJ/dtrap (max norm) and lam_0
    (relative L2) against the oracle's adjoint."""
    return (abs(out["J"] - J) / abs(J),
            np.max(np.abs(out["dJ_damp"] - dJ_da)) / np.max(np.abs(dJ_da)),
            np.max(np.abs(out["dJ_dtrap"] - dJ_dt)) / np.max(np.abs(dJ_dt)),
            _rel(out["dJ_dpsi0"].cpu().numpy().astype(np.complex128), lam0))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_overlap_adjoint_matches_oracle(env, prec):
    torch, dg = env
    n, d = (16, 18, 24), (0.45, 0.4, 0.35)
    p = O.Params(n, d, 0.01, (1.0, 1.2, 1.7), 15.0, 9.0, False)
    psi0 = W.random_state(n, d, seed=51)
    tgt = W.random_state(n, d, seed=52)
    amp = np.random.default_rng(53).uniform(0.8, 1.2, size=8)
    J, psiN, dJ_da, dJ_dt, lam0 = O.adjoint_evolve(p, psi0, amp, "overlap", tgt)
    dt = torch.complex128 if prec == "f64" else torch.complex64
    plan = dg.Plan(n, d, p.dt, p.trap, p.g, p.gd, real_time=True, dtype=dt)
    out = plan.adjoint(plan.new_state(psi0), amp, ckpt_every=2, objective="overlap",
                       target=plan.new_state(tgt))
    errs = _adjoint_errors(out, J, dJ_da, dJ_dt, lam0)
    print(f"  adjoint {prec}: J {errs[0]:.2e} dJ/da {errs[1]:.2e} dJ/dtrap {errs[2]:.2e} lam0 {errs[3]:.2e}",
          flush=True)
    assert max(errs) < (1e-10 if prec == "f64" else 5e-5)


@pytest.mark.parametrize("ckpt", [3, 1], ids=["ckpt3", "keep_all"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [((8, 32, 64), (0.45, 0.3, 0.2)), ((6, 32, 128), (0.5, 0.3, 0.1)),
                                   ((8, 32, 256), (0.45, 0.3, 0.1))],
                         ids=lambda s: "x".join(map(str, s[0])))
def test_adjoint_with_compiled_z_passes_matches_oracle(env, shape, prec, ckpt):
    """z lines of 64, 128 and 256 points and 32 y lines take the compiled z
    passes of the adjoint (the recompute steps' fused z pass that keeps Phi, the
    adjoint-source R2C, the C2R fused with the nonlinear adjoint update, and the
    conjugate z sweep with coalesced loads and shuffle carries; Nz = 256 is the
    256^3 instantiation); energy objective against the oracle."""
    torch, dg = env
    n, d = shape
    p = O.Params(n, d, 0.004, (1.0, 1.3, 1.1), 12.0, 7.0, False)
    psi0 = W.random_state(n, d, seed=81)
    amp = np.random.default_rng(82).uniform(0.8, 1.2, size=7)
    J, psiN, dJ_da, dJ_dt, lam0 = O.adjoint_evolve(p, psi0, amp, "energy", None)
    dt = torch.complex128 if prec == "f64" else torch.complex64
    plan = dg.Plan(n, d, p.dt, p.trap, p.g, p.gd, real_time=True, dtype=dt)
    out = plan.adjoint(plan.new_state(psi0), amp, ckpt_every=ckpt)
    errs = _adjoint_errors(out, J, dJ_da, dJ_dt, lam0)
    print(f"  adjoint {prec}: J {errs[0]:.2e} dJ/da {errs[1]:.2e} dJ/dtrap {errs[2]:.2e} lam0 {errs[3]:.2e}",
          flush=True)
    assert max(errs) < (1e-10 if prec == "f64" else 5e-5)


def test_adjoint_independent_of_checkpoint_interval(env):
    torch, dg = env
    n, d = (16, 16, 24), (0.45, 0.45, 0.35)
    psi0 = W.random_state(n, d, seed=61)
    amp = np.random.default_rng(62).uniform(0.8, 1.2, size=14)
    plan = dg.Plan(n, d, 0.01, (1.0, 1.1, 1.6), 12.0, 6.0, real_time=True, dtype=torch.complex128)
    ref = plan.adjoint(plan.new_state(psi0), amp, ckpt_every=13)
    for k in (1, 2, 4, 100):  # 1: every state kept, nothing recomputed
        out = plan.adjoint(plan.new_state(psi0), amp, ckpt_every=k)
        assert out["J"] == ref["J"]
        assert np.array_equal(out["dJ_damp"], ref["dJ_damp"])
        assert torch.equal(out["dJ_dpsi0"], ref["dJ_dpsi0"])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjoint_long_x_lines_matches_oracle(env, prec):
    """x lines of 2048 points: the forward and the conjugate x sweeps read their
    Thomas tables from global memory (tables of 128 segments would crowd the
    LDS); energy objective against the oracle."""
    torch, dg = env
    n, d = (2048, 4, 16), (0.02, 0.6, 0.4)
    p = O.Params(n, d, 0.004, (1.0, 1.3, 1.1), 12.0, 7.0, False)
    psi0 = W.random_state(n, d, seed=91)
    amp = np.random.default_rng(92).uniform(0.8, 1.2, size=5)
    J, psiN, dJ_da, dJ_dt, lam0 = O.adjoint_evolve(p, psi0, amp, "energy", None)
    dt = torch.complex128 if prec == "f64" else torch.complex64
    plan = dg.Plan(n, d, p.dt, p.trap, p.g, p.gd, real_time=True, dtype=dt)
    out = plan.adjoint(plan.new_state(psi0), amp, ckpt_every=2)
    errs = _adjoint_errors(out, J, dJ_da, dJ_dt, lam0)
    print(f"  adjoint 2048-point x lines {prec}: J {errs[0]:.2e} dJ/da {errs[1]:.2e} "
          f"dJ/dtrap {errs[2]:.2e} lam0 {errs[3]:.2e}", flush=True)
    assert max(errs) < (1e-10 if prec == "f64" else 5e-5)
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjoint_with_compiled_passes_independent_of_checkpoint_interval(env, prec):
    """With the compiled z passes (z lines of 128 points: the recompute steps'
    fused z pass that keeps Phi, the adjoint-source R2C, and the nonlinear
    adjoint update that also applies the next reverse step's conjugate z
    sweep) the gradients do not depend on the checkpoint interval, bit for
    bit."""
    torch, dg = env
    n, d = (6, 32, 128), (0.5, 0.3, 0.1)
    psi0 = W.random_state(n, d, seed=71)
    amp = np.random.default_rng(72).uniform(0.8, 1.2, size=9)
    dt = torch.complex128 if prec == "f64" else torch.complex64
    plan = dg.Plan(n, d, 0.004, (1.0, 1.3, 1.1), 12.0, 7.0, real_time=True, dtype=dt)
    ref = plan.adjoint(plan.new_state(psi0), amp, ckpt_every=4)
    for k in (1, 3, 100):
        out = plan.adjoint(plan.new_state(psi0), amp, ckpt_every=k)
        assert out["J"] == ref["J"]
        assert np.array_equal(out["dJ_damp"], ref["dJ_damp"])
        assert torch.equal(out["dJ_dpsi0"], ref["dJ_dpsi0"])
    plan.close()


def test_potential_is_linear_and_symmetric(env):
    """Phi is linear in the density and the discrete convolution is symmetric:
    sum n1 Phi[n2] = sum n2 Phi[n1] (real even kernel)."""
    torch, dg = env
    n, d = (32, 24, 48), (0.3, 0.35, 0.25)
    plan = dg.Plan(n, d, 0.01, (1, 1, 1), 0.0, 1.0, dtype=torch.complex128)
    p1 = plan.new_state(W.random_state(n, d, seed=71))
    p2 = plan.new_state(W.random_state(n, d, seed=72))
    f1 = plan.potential(p1).cpu().numpy()
    f2 = plan.potential(p2).cpu().numpy()
    n1 = np.abs(p1.cpu().numpy()) ** 2
    n2 = np.abs(p2.cpu().numpy()) ** 2
    assert abs(np.sum(n1 * f2) - np.sum(n2 * f1)) < 1e-13 * np.sum(np.abs(n1 * f2))
    p3 = plan.new_state(np.sqrt(n1 + 2 * n2))
    f3 = plan.potential(p3).cpu().numpy()
    assert np.max(np.abs(f3 - (f1 + 2 * f2))) < 1e-13 * np.max(np.abs(f3))


def test_fused_y_schedule_follows_the_plan(env):
    """dgpe_plan_fused_y reports the schedule dgpe_step runs: the fused y
    schedule for imaginary-time plans whose grid has it (both precisions), the
    separate y sweep in real time, with DGPE_PARAM_FUSED_Y = 0, without the
    compiled passes, or for a grid with no compiled fused z pass; and
    switching back to imaginary time restores it."""
    torch, dg = env
    d = (0.4, 0.3, 0.2)
    for dtype in (torch.complex64, torch.complex128):
        p = dg.Plan((16, 64, 256), d, 0.002, (1, 1, 1), 10.0, 4.0, dtype=dtype)
        assert p.fused_y
        p.set("real_time", 1)
        assert not p.fused_y
        p.set("real_time", 0)
        assert p.fused_y
        p.set("fused_y", 0)
        assert not p.fused_y
        p.set("fused_y", 1)
        p.set("fast_fft", 0)
        assert not p.fused_y
        p.close()
    q = dg.Plan((16, 24, 32), (0.4, 0.35, 0.3), 0.002, (1, 1, 1), 10.0, 4.0, dtype=torch.complex64)
    assert not q.fused_y  # no compiled fused z pass for this grid
    q.close()
