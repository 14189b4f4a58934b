"""Full-size workloads on the GPU against the FP64 oracle's stored records
(tests/golden/make_fullsize_golden.py), in the launch configuration the
benchmark uses, plus finite-difference checks of the adjoint.

The stored records hold 512 sampled state values per workload; the GPU state is
compared at those points (max |error| / max |psi|) and on the observables.  The
256^3 record is also recomputed on the host for a whole-grid relative L2, and
FP32 states are compared with FP64 ones over the whole grid.  Each side
prepares its own initial state from the same seeded input.
"""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _golden(name):
    return json.load(open(os.path.join(ROOT, "tests", "golden", f"{name}_oracle.json")))


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_1610_05329_amd as dg
    assert torch.cuda.is_available()
    dg.load()
    return torch, dg


def _sample_err(psi, smp):
    flat = psi.reshape(-1).cpu().numpy().astype(np.complex128)
    idx = np.asarray(smp["index"])
    ref = np.asarray(smp["re"]) + 1j * np.asarray(smp["im"])
    return float(np.max(np.abs(flat[idx] - ref)) / smp["max_abs"])


def _dtype(torch, prec):
    return torch.complex128 if prec == "f64" else torch.complex64


@pytest.fixture(scope="module")
def imag256_oracle():
    """The oracle's state after the record's 20 steps of the 256^3 workload,
    computed here on the host (about 40 s of numpy) for the whole-grid
    comparison."""
    from oracle import dgpe_oracle as O
    cfg = W.CONFIGS["imag_256cubed"]
    steps = _golden("imag_256cubed")["steps"]
    _say(f"imag_256cubed: oracle, {steps} steps on the host")
    return O.evolve(O.Params.from_config(cfg), W.noisy_gaussian(cfg), steps)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.timeout(900)
def test_imag_256cubed_whole_grid_matches_oracle(env, imag256_oracle):
    """256^3 imaginary time, 20 steps, in the benchmark's plan shape (FP32: the
    fused y schedule with 16 x segments and 16 y segments; FP64 likewise):
    whole-grid relative L2 of each state against the oracle and of FP32 against
    FP64, plus the stored record's samples and observables."""
    torch, dg = env
    cfg = W.CONFIGS["imag_256cubed"]
    gold = _golden("imag_256cubed")
    ref = imag256_oracle
    states = {}
    for prec in ("f64", "f32"):
        _say(f"imag_256cubed {prec}: stepping")
        plan = dg.Plan(cfg.n, cfg.d, cfg.dt, cfg.trap, cfg.g, cfg.gd, dtype=_dtype(torch, prec))
        assert plan.fused_y
        psi = plan.new_state(W.noisy_gaussian(cfg))
        plan.step(psi, gold["steps"])
        o = plan.observables(psi)
        g = gold["observables"]
        emu = abs(o["mu"] - g["mu"]) / abs(g["mu"])
        een = abs(o["energy"] - g["energy"]) / abs(g["energy"])
        err = _sample_err(psi, gold["samples"])
        host = psi.cpu().numpy().astype(np.complex128)
        l2 = _rel(host, ref)
        _say(f"imag_256cubed {prec}: whole-grid rel L2 {l2:.3e}, sampled {err:.3e}, "
             f"mu rel err {emu:.3e}, energy rel err {een:.3e}")
        tol = 1e-12 if prec == "f64" else 1e-5
        assert l2 < tol and err < tol
        assert emu < tol and een < tol
        assert abs(o["norm"] - 1.0) < (1e-13 if prec == "f64" else 1e-6)
        states[prec] = host
        plan.close()
        del psi, plan
    l2 = _rel(states["f32"], states["f64"])
    _say(f"imag_256cubed: FP32 vs FP64 whole-grid rel L2 {l2:.3e}")
    assert l2 < 1e-5


@pytest.fixture(scope="module")
def quench128_ground_state(env):
    """The 128^3 ground state at gd = 15 from the trap Gaussian by the driver
    (mu checked every 10 steps, stop below 1e-10 per step), FP64, as the record
    prepared its own: it must stop at the same step."""
    torch, dg = env
    cfg = W.CONFIGS["quench_128cubed"]
    gold = _golden("quench_128cubed")
    plan = dg.Plan(cfg.n, cfg.d, cfg.dt, cfg.trap, cfg.g, gold["prep_gd"], dtype=torch.complex128)
    psi = plan.new_state(W.gaussian_state(cfg.n, cfg.d, cfg.trap))
    out = plan.ground_state(psi, tol=gold["prep_tol"], max_steps=gold["prep_max_steps"],
                            check_every=gold["prep_check_every"])
    _say(f"quench_128cubed ground state: {out['steps']} steps (oracle {gold['prep_imag_steps']}), "
         f"dmu/step {out['dmu_per_step']:.3e} (oracle {gold['prep_dmu_per_step']:.3e}), "
         f"mu {out['observables']['mu']:.13f} (oracle {gold['prep_mu']:.13f})")
    assert out["converged"] and out["steps"] == gold["prep_imag_steps"]
    assert abs(out["observables"]["mu"] - gold["prep_mu"]) < 1e-12 * abs(gold["prep_mu"])
    host = psi.cpu().numpy()
    plan.close()
    return host


def test_quench_128cubed_real_time_matches_oracle_record(env, quench128_ground_state):
    """128^3: the driver's ground state at gd = 15 (FP64), quench to gd = 20,
    1000 real-time steps in FP64 and FP32 (the FP32 run starts from the same
    state rounded to FP32): norm conservation and energy drift per dtype, the
    record's samples, and whole-grid relative L2 of the FP32 state against the
    FP64 one (itself within 1e-12 of the oracle at the samples)."""
    torch, dg = env
    cfg = W.CONFIGS["quench_128cubed"]
    gold = _golden("quench_128cubed")
    final = {}
    for prec in ("f64", "f32"):
        plan = dg.Plan(cfg.n, cfg.d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=True, dtype=_dtype(torch, prec))
        psi = plan.new_state(quench128_ground_state)
        o0 = plan.observables(psi)
        plan.step(psi, gold["steps"])
        o1 = plan.observables(psi)
        err = _sample_err(psi, gold["samples"])
        g0, g1 = gold["observables_start"], gold["observables"]
        drift = o1["energy"] - o0["energy"]
        gdrift = g1["energy"] - g0["energy"]
        _say(f"quench_128cubed {prec}: sampled state err {err:.3e}; norm drift {o1['norm'] - o0['norm']:.3e}; "
             f"energy {o0['energy']:.12f} -> {o1['energy']:.12f} (drift {drift:.3e}, oracle {gdrift:.3e})")
        assert abs(o0["energy"] - g0["energy"]) < (1e-11 if prec == "f64" else 1e-6) * abs(g0["energy"])
        if prec == "f64":
            assert err < 1e-12
            assert abs(o1["norm"] - o0["norm"]) < 1e-12
            assert abs(drift - gdrift) < 1e-10 * abs(g0["energy"])
        else:
            assert err < 1e-5
            assert abs(o1["norm"] - o0["norm"]) < 1e-6
            assert abs(drift - gdrift) < 1e-6 * abs(g0["energy"])
        final[prec] = psi.cpu().numpy().astype(np.complex128)
        plan.close()
    l2 = _rel(final["f32"], final["f64"])
    _say(f"quench_128cubed: FP32 vs FP64 whole-grid rel L2 {l2:.3e}")
    assert l2 < 1e-5


def _adjoint_setup(torch, dg, prec, gold):
    cfg = W.CONFIGS["adjoint_96cubed"]
    prep = dg.Plan(cfg.n, cfg.d, cfg.dt, cfg.trap, cfg.g, cfg.gd, dtype=_dtype(torch, prec))
    psi0 = prep.new_state(W.gaussian_state(cfg.n, cfg.d, cfg.trap))
    prep.step(psi0, gold["prep_imag_steps"])
    plan = dg.Plan(cfg.n, cfg.d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=True, dtype=_dtype(torch, prec))
    return cfg, plan, psi0


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjoint_96cubed_matches_oracle_record(env, prec):
    torch, dg = env
    gold = _golden("adjoint_96cubed")
    cfg, plan, psi0 = _adjoint_setup(torch, dg, prec, gold)
    W_ = dg.knot_matrix(len(gold["knots"]), gold["steps"], cfg.dt)
    amp = W_ @ np.asarray(gold["knots"])
    assert np.max(np.abs(amp - np.asarray(gold["amp"]))) < 1e-14
    out = plan.adjoint(psi0, amp, ckpt_every=20)
    dJ = np.asarray(gold["dJ_damp"])
    e_J = abs(out["J"] - gold["J"]) / abs(gold["J"])
    e_a = np.max(np.abs(out["dJ_damp"] - dJ)) / np.max(np.abs(dJ))
    e_t = np.max(np.abs(out["dJ_dtrap"] - np.asarray(gold["dJ_dtrap"]))) / np.max(np.abs(gold["dJ_dtrap"]))
    e_psi = _sample_err(out["psi_final"], gold["samples_psiN"])
    e_lam = _sample_err(out["dJ_dpsi0"], gold["samples_lam0"])
    _say(f"adjoint_96cubed {prec}: J {e_J:.2e}, dJ/da {e_a:.2e}, dJ/dtrap {e_t:.2e}, psi_N {e_psi:.2e}, lam0 {e_lam:.2e}")
    tol = 1e-9 if prec == "f64" else 5e-5
    assert e_J < tol and e_a < tol and e_t < tol and e_lam < tol
    assert e_psi < (1e-11 if prec == "f64" else 1e-5)


@pytest.fixture(scope="module")
def adjoint96_fd(env):
    """Central differences (h = 1e-4) of the final energy with respect to the
    40 knots and (lambda, gamma), from the FP64 GPU forward run."""
    torch, dg = env
    gold = _golden("adjoint_96cubed")
    cfg, plan, psi0 = _adjoint_setup(torch, dg, "f64", gold)
    nsteps = gold["steps"]
    W_ = dg.knot_matrix(len(gold["knots"]), nsteps, cfg.dt)

    def forward(kn, lam, gam):
        plan.set("lambda", lam)
        plan.set("gamma", gam)
        amp = W_ @ kn
        psi = psi0.clone()
        plan.step(psi, nsteps, amp[:-1])
        o = plan.observables(psi, amp[-1])
        return o["e_kin"] + o["e_trap"] + o["e_contact"] + o["e_dd"]

    k0 = np.asarray(gold["knots"])
    h = 1e-4
    fd = np.zeros(len(k0))
    for i in range(len(k0)):
        kp, km = k0.copy(), k0.copy()
        kp[i] += h
        km[i] -= h
        fd[i] = (forward(kp, cfg.trap[1], cfg.trap[2]) - forward(km, cfg.trap[1], cfg.trap[2])) / (2 * h)
    fdl = (forward(k0, cfg.trap[1] + h, cfg.trap[2]) - forward(k0, cfg.trap[1] - h, cfg.trap[2])) / (2 * h)
    fdg = (forward(k0, cfg.trap[1], cfg.trap[2] + h) - forward(k0, cfg.trap[1], cfg.trap[2] - h)) / (2 * h)
    plan.close()
    return fd, np.array([fdl, fdg])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjoint_96cubed_against_finite_differences(env, adjoint96_fd, prec):
    """Knot and (lambda, gamma) gradients through DgpeEvolve in each precision
    against central differences h = 1e-4 of the FP64 GPU forward run:
    max |g - fd| / max |fd| <= 1e-4.  The plan's own trap is unchanged after
    the call."""
    torch, dg = env
    gold = _golden("adjoint_96cubed")
    cfg, plan, psi0 = _adjoint_setup(torch, dg, prec, gold)
    fd, fdt = adjoint96_fd
    nsteps = gold["steps"]
    knots = torch.tensor(gold["knots"], dtype=torch.float64, requires_grad=True)
    # the gradient is taken at the workload's trap: lam_gam carries it
    lg = torch.tensor([cfg.trap[1], cfg.trap[2]], dtype=torch.float64, requires_grad=True)
    plan.set("lambda", 0.75)
    plan.set("gamma", 3.5)
    J = dg.DgpeEvolve.apply(knots, lg, psi0, plan, nsteps, 20, "energy", None)
    J.backward()
    assert plan.trap[1:] == [0.75, 3.5]
    gk, gt = knots.grad.numpy(), lg.grad.numpy()
    ek = np.max(np.abs(gk - fd)) / np.max(np.abs(fd))
    et = float(np.max(np.abs(gt - fdt) / np.abs(fdt)))
    _say(f"adjoint_96cubed FD check {prec}: knots {ek:.2e}, (lambda, gamma) {et:.2e}; "
         f"|dJ/dknots| max {np.max(np.abs(fd)):.3e}")
    assert abs(float(J.detach()) - gold["J"]) < (1e-9 if prec == "f64" else 5e-5) * abs(gold["J"])
    assert ek < 1e-4 and et < 1e-4
