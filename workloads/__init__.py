"""Seeded synthetic workloads for the 3D dipolar Gross-Pitaevskii time step.

This module holds the run configurations and the seeded initial states that both
the GPU library's callers (tests, benchmark) and the FP64 oracle consume.  It
contains none of the time-stepping arithmetic: only grid sizes, physical
parameters, the analytic Gaussian initial state and seeded random numbers.

The paper measures on "arbitrary grid sizes" (program summary, Testing results)
and ships no dataset; every input here is synthetic.  Units are trap units
(length sqrt(hbar/(m omega)), time 1/omega, energy hbar omega).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Tuple

import numpy as np

__all__ = [
    "Config", "CONFIGS", "grid_axes", "gaussian_state", "noisy_gaussian",
    "knot_values", "random_state",
]


@dataclass(frozen=True)
class Config:
    """One workload: grid, time step and physical parameters.

    n      -- (Nx, Ny, Nz); arrays are C-ordered [x][y][z] with Nx slowest
              (program summary, DBEC-GP-MPI package: distribution along NX,
              the first and slowest-changing dimension).
    d      -- (dx, dy, dz) grid spacings.
    dt     -- time step (imaginary or real time).
    trap   -- (nu, lambda, gamma): trap frequencies along (x, y, z).
    g, gd  -- contact and dipolar interaction strengths.
    R      -- spherical cut-off radius of the dipolar kernel; <= 0 selects
              min(N_i d_i) / 2.
    imag   -- True for imaginary-time propagation (ground state).
    steps  -- number of time steps of the workload.
    """

    name: str
    n: Tuple[int, int, int]
    d: Tuple[float, float, float]
    dt: float
    trap: Tuple[float, float, float]
    g: float
    gd: float
    imag: bool
    steps: int
    R: float = 0.0
    noise: float = 0.0
    seed: int = 0
    note: str = ""

    @property
    def npoints(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def cutoff(self) -> float:
        if self.R > 0:
            return float(self.R)
        return 0.5 * min(self.n[i] * self.d[i] for i in range(3))

    def with_(self, **kw) -> "Config":
        return replace(self, **kw)


# The five workloads of this project, named by time mode and grid.  Parameters
# the paper does not state are proposals (readings of the paper).
CONFIGS = {
    "imag_32cubed": Config("imag_32cubed", (32, 32, 32), (0.25, 0.25, 0.25), 0.005, (1.0, 1.0, 1.0),
                 20.0, 5.0, True, 200, R=4.0, noise=1e-3, seed=1,
                 note="imaginary time, FP64, isotropic; mu, energy, rms"),
    "quench_128cubed": Config("quench_128cubed", (128, 128, 128), (0.2, 0.2, 0.2), 0.002, (1.0, 1.0, 4.0),
                 50.0, 20.0, False, 1000, seed=2,
                 note="real time after a quench gd 15 -> 20; norm and energy drift"),
    "imag_256cubed": Config("imag_256cubed", (256, 256, 256), (0.1, 0.1, 0.1), 0.001, (1.0, 1.0, 0.5),
                 100.0, 60.0, True, 1000, noise=1e-3, seed=3,
                 note="imaginary time at 256^3; the throughput workload"),
    "adjoint_96cubed": Config("adjoint_96cubed", (96, 96, 96), (0.2, 0.2, 0.2), 0.002, (1.0, 1.0, 4.0),
                 50.0, 15.0, False, 400, seed=4,
                 note="real time, adjoint of the final energy; 40 trap-amplitude knots"),
    "real_512x512x256": Config("real_512x512x256", (512, 512, 256), (0.1, 0.1, 0.2), 0.001, (1.0, 1.0, 8.0),
                 200.0, 150.0, False, 200, seed=5,
                 note="large anisotropic real-time grid, FP32"),
}


def grid_axes(n, d):
    """Grid coordinates x_i = (i - N/2) d along each axis (the point x = 0 is on
    the grid; the box is [-N d / 2, N d / 2))."""
    return tuple((np.arange(n[a], dtype=np.float64) - n[a] // 2) * d[a] for a in range(3))


def gaussian_state(n, d, trap, widths=None):
    """Analytic Gaussian pi^{-3/4} (nu lam gam)^{1/4} exp(-(nu x^2 + lam y^2 + gam z^2)/2),
    the ground state of the non-interacting anisotropic harmonic trap, as complex128
    [Nx][Ny][Nz].  `widths` (per-axis inverse-width factors) replaces `trap` in the
    exponent and the prefactor when given."""
    w = trap if widths is None else widths
    x, y, z = grid_axes(n, d)
    fx = np.exp(-0.5 * w[0] * x * x)
    fy = np.exp(-0.5 * w[1] * y * y)
    fz = np.exp(-0.5 * w[2] * z * z)
    pref = np.pi ** -0.75 * (w[0] * w[1] * w[2]) ** 0.25
    psi = pref * fx[:, None, None] * fy[None, :, None] * fz[None, None, :]
    return psi.astype(np.complex128)


def _unit_norm(psi, d):
    dv = d[0] * d[1] * d[2]
    return psi / np.sqrt(np.sum(np.abs(psi) ** 2) * dv)


def noisy_gaussian(cfg: Config, seed=None, amplitude=None):
    """The trap Gaussian plus real uniform noise in [-a, a), rescaled to unit norm
    (sum |psi|^2 dV = 1).  The noise is drawn once on the host with numpy's
    default_rng(seed) so both sides of a comparison receive the same bytes."""
    a = cfg.noise if amplitude is None else amplitude
    s = cfg.seed if seed is None else seed
    psi = gaussian_state(cfg.n, cfg.d, cfg.trap)
    if a > 0:
        rng = np.random.default_rng(s)
        psi = psi + rng.uniform(-a, a, size=cfg.n)
    return _unit_norm(psi, cfg.d)


def random_state(n, d, seed, scale=1.0, envelope=True):
    """Seeded complex random field (uniform real and imaginary parts), optionally
    under a Gaussian envelope so it decays towards the box edge; unit norm."""
    rng = np.random.default_rng(seed)
    psi = rng.uniform(-1, 1, size=n) + 1j * rng.uniform(-1, 1, size=n)
    if envelope:
        x, y, z = grid_axes(n, d)
        L = [0.35 * n[a] * d[a] for a in range(3)]
        env = (np.exp(-(x / L[0]) ** 2)[:, None, None] * np.exp(-(y / L[1]) ** 2)[None, :, None]
               * np.exp(-(z / L[2]) ** 2)[None, None, :])
        psi = psi * env
    return scale * _unit_norm(psi, d)


def knot_values(seed=4, count=40, lo=0.8, hi=1.2):
    """Seeded trap-amplitude knots a_k, uniform in [lo, hi)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=count)
