"""Writes tests/golden/imag_32cubed_oracle.json: the FP64 oracle's observables for the
32^3 imaginary-time workload (isotropic trap, g = 20, gd = 5, R = 4, dt = 0.005,
200 steps from the seeded noisy Gaussian).  Calls only the oracle and the seeded
input module; the paper prints no such values, so this fixture is a regression
record of the oracle, not a pin of it."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import dgpe_oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def main():
    cfg = W.CONFIGS["imag_32cubed"]
    p = O.Params.from_config(cfg)
    psi = O.evolve(p, W.noisy_gaussian(cfg), cfg.steps)
    o = O.observables(p, psi)
    o["rms"] = [float(v) for v in o["rms"]]
    out = {"workload": "32^3 imaginary time, 200 steps", "config": "imag_32cubed", "observables": o}
    with open(os.path.join(os.path.dirname(__file__), "imag_32cubed_oracle.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
