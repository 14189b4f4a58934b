"""The allocation-free plan (dgpe_plan_create_noalloc): the library's static
device scratch as workspace.  Two plans in a row on one device, the second on
a smaller grid, each stepped and measured against a plan on a caller-owned
workspace (dgpe_plan_create) from the same input; the superseded first plan is
then refused."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

# (grid, spacings, real time, precision, steps): the first takes the FP32
# imaginary-time fused y schedule, the second (smaller) FP64 real time
CALLS = [
    ((24, 32, 64), (0.4, 0.35, 0.2), False, "f32", 5),
    ((16, 24, 32), (0.4, 0.35, 0.3), True, "f64", 5),
]
TOL = {"f64": 1e-12, "f32": 1e-5}


def _say(*a):
    print(*a, flush=True)


def _run(dg, torch, n, d, real_time, prec, steps, noalloc):
    dtype = torch.complex128 if prec == "f64" else torch.complex64
    cfg = W.Config("noalloc", n, d, 0.004, (1.0, 1.2, 1.6), 20.0, 8.0, not real_time, steps,
                   noise=1e-3, seed=21)
    plan = dg.Plan(n, d, cfg.dt, cfg.trap, cfg.g, cfg.gd, real_time=real_time, dtype=dtype,
                   noalloc=noalloc)
    psi = plan.new_state(W.noisy_gaussian(cfg))
    plan.step(psi, steps)
    obs = plan.observables(psi)
    return plan, psi.cpu().numpy().astype(np.complex128), obs


def test_noalloc_plans_match_workspace_plans_and_supersede():
    import torch
    import paper_1610_05329_amd as dg
    assert torch.cuda.is_available()
    dg.load()
    plans = []
    for n, d, real_time, prec, steps in CALLS:
        _say(f"noalloc plan {n} {'real' if real_time else 'imag'} {prec}")
        assert dg.workspace_bytes(n, real_time, prec == "f32") <= dg._lib.NOALLOC_MAX_BYTES
        ref_plan, ref, ref_obs = _run(dg, torch, n, d, real_time, prec, steps, noalloc=False)
        plan, got, obs = _run(dg, torch, n, d, real_time, prec, steps, noalloc=True)
        assert plan.workspace is None
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        _say(f"  rel L2 vs the workspace plan {err:.3e} (bitwise equal: {np.array_equal(got, ref)})")
        assert err <= TOL[prec]
        for k in ("norm", "mu", "energy"):
            assert abs(obs[k] - ref_obs[k]) <= TOL[prec] * abs(ref_obs[k]), k
        ref_plan.close()
        plans.append(plan)
    # the first allocation-free plan's tables were overwritten by the second
    first, second = plans
    psi = first.new_state()
    with pytest.raises(dg.DgpeError) as e:
        first.step(psi, 1)
    assert e.value.status == 6 and "superseded" in str(e.value)
    # the live one still steps
    n, d, real_time, prec, steps = CALLS[1]
    _, again, _ = _run(dg, torch, n, d, real_time, prec, steps, noalloc=False)
    psi2 = second.new_state(W.noisy_gaussian(W.Config("noalloc", n, d, 0.004, (1.0, 1.2, 1.6), 20.0,
                                                       8.0, not real_time, steps, noise=1e-3,
                                                       seed=21)))
    second.step(psi2, steps)
    got2 = psi2.cpu().numpy().astype(np.complex128)
    assert float(np.linalg.norm(got2 - again) / np.linalg.norm(again)) <= TOL[prec]
    first.close()
    second.close()
