"""Writes full-size oracle records for the GPU parity tests (calls only the
oracle and the seeded input module; minutes of CPU time each).

  imag_256cubed    256^3 imaginary time (dx 0.1, dt 0.001, trap (1, 1, 0.5), g 100, gd 60),
      20 steps from the seeded noisy Gaussian: observables and 512 sampled
      state values.  (These parameters collapse after about 90 steps; the
      record stays on the regular part of the trajectory.)
  quench_128cubed  128^3: the imaginary-time ground state at gd = 15 from the trap Gaussian
      (the driver: mu checked every 10 steps, stop when it changes by less
      than 1e-10 per step, at most 20000 steps), then the quench gd -> 20 and
      1000 real-time steps (dt 0.002): observables at the quench and at the
      end, and 512 sampled state values.
  adjoint_96cubed  96^3: 500 imaginary-time steps (dt 0.002, gd 15) from the trap Gaussian
      as psi0, then the adjoint of the final energy through 400 real-time
      steps with the trap amplitude on 40 seeded knots in [0.8, 1.2).

Usage: python tests/golden/make_fullsize_golden.py imag_256cubed|quench_128cubed|adjoint_96cubed
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import dgpe_oracle as O  # noqa: E402
import workloads as W  # noqa: E402

NSAMPLE = 512


def samples(psi, seed):
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, psi.size, size=NSAMPLE)
    flat = psi.reshape(-1)
    return {"index": idx.tolist(), "re": flat[idx].real.tolist(), "im": flat[idx].imag.tolist(),
            "max_abs": float(np.max(np.abs(psi)))}


def obs(p, psi, a=1.0):
    o = O.observables(p, psi, a)
    o["rms"] = [float(v) for v in o["rms"]]
    return o


def knot_amplitudes(knots, nsteps, dt):
    T = nsteps * dt
    h = T / (len(knots) - 1)
    out = np.empty(nsteps + 1)
    for n in range(nsteps + 1):
        t = n * dt
        k = min(int(np.floor(t / h)), len(knots) - 2)
        w = (t - k * h) / h
        out[n] = (1 - w) * knots[k] + w * knots[k + 1]
    return out


def make_imag_256cubed():
    cfg = W.CONFIGS["imag_256cubed"]
    steps = 20
    p = O.Params.from_config(cfg)
    psi = O.evolve(p, W.noisy_gaussian(cfg), steps)
    return {"config": "imag_256cubed", "steps": steps, "observables": obs(p, psi), "samples": samples(psi, 33)}


def make_quench_128cubed():
    cfg = W.CONFIGS["quench_128cubed"]
    tol, cap, every, steps = 1e-10, 20000, 10, 1000
    prep = O.Params.from_config(cfg, gd=15.0, imag=True)
    psi, prep_steps, rate, mu = O.ground_state(prep, W.gaussian_state(cfg.n, cfg.d, cfg.trap), tol, cap,
                                               every)
    p = O.Params.from_config(cfg, imag=False)
    o0 = obs(p, psi)
    psi = O.evolve(p, psi, steps)
    return {"config": "quench_128cubed", "prep": "ground_state", "prep_tol": tol, "prep_max_steps": cap,
            "prep_check_every": every, "prep_imag_steps": prep_steps, "prep_dmu_per_step": rate,
            "prep_mu": mu, "prep_gd": 15.0, "steps": steps,
            "observables_start": o0, "observables": obs(p, psi), "samples": samples(psi, 22)}


def make_adjoint_96cubed():
    cfg = W.CONFIGS["adjoint_96cubed"]
    prep_steps, steps = 500, cfg.steps
    prep = O.Params.from_config(cfg, imag=True)
    psi0 = O.evolve(prep, W.gaussian_state(cfg.n, cfg.d, cfg.trap), prep_steps)
    knots = W.knot_values(cfg.seed)
    amp = knot_amplitudes(knots, steps, cfg.dt)
    p = O.Params.from_config(cfg, imag=False)
    J, psiN, dJ_da, dJ_dt, lam0 = O.adjoint_evolve(p, psi0, amp)
    return {"config": "adjoint_96cubed", "prep_imag_steps": prep_steps, "steps": steps, "knots": knots.tolist(),
            "amp": amp.tolist(), "J": J, "dJ_damp": dJ_da.tolist(), "dJ_dtrap": dJ_dt.tolist(),
            "samples_psiN": samples(psiN, 44), "samples_lam0": samples(lam0, 45)}


def main():
    which = sys.argv[1]
    t = time.time()
    rec = {"imag_256cubed": make_imag_256cubed, "quench_128cubed": make_quench_128cubed,
           "adjoint_96cubed": make_adjoint_96cubed}[which]()
    rec["oracle_seconds"] = round(time.time() - t, 1)
    with open(os.path.join(HERE, f"{which}_oracle.json"), "w") as f:
        json.dump(rec, f)
    print(which, "done in", rec["oracle_seconds"], "s")


if __name__ == "__main__":
    main()
