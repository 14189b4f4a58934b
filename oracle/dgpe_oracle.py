"""FP64 CPU oracle for the split-step Crank-Nicolson time step of the 3D dipolar
Gross-Pitaevskii equation (GPE), in imaginary and real time, with its adjoint.

TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the
CPU-baseline leg of the benchmark may import or run this module.  It shares no
code with the GPU library: its own grid, kernel, FFT use (numpy's pocketfft as
the library primitive), Thomas solver and sums.  Everything is float64 /
complex128, written for readability, not speed.

What the paper fixes (program summary): the GPE with contact and dipolar
interaction in an anisotropic harmonic trap ("Nature of problem"); the
split-step Crank-Nicolson discretisation propagated in imaginary or real time,
with the dipolar term evaluated in momentum space through the convolution
theorem ("Solution method"); the real-to-complex transform of the real density
with its Hermitian half spectrum ("Summary of revisions", DBEC-GP-OMP package);
row-major [x][y][z] storage with NX slowest (DBEC-GP-MPI package).  The paper
prints no equations; the formulas below are the standard dimensionless dipolar
GPE in trap units and are readings of the paper where it is silent:

  i dpsi/dt = [-1/2 Lap + V + g |psi|^2 + gd Phi] psi     (real time)
    dpsi/dtau = -[...] psi                               (imaginary time)
  V = a(t)/2 (nu^2 x^2 + lam^2 y^2 + gam^2 z^2)
  Phi = IDFT[ U_R(k) DFT[|psi|^2] ],  dipoles along z,
  U_R(k) = (4 pi / 3)(3 kz^2/k^2 - 1)(1 + 3 cos(kR)/(kR)^2 - 3 sin(kR)/(kR)^3).

One step n -> n+1 (first-order Lie splitting, nonlinear part first):
  1. theta = dt (V(a_n) + g n + gd Phi[n]), n = |psi|^2 (the pre-step density);
     real time psi <- psi exp(-i theta), imaginary time psi <- psi exp(-theta).
  2. For each axis, along every line, Crank-Nicolson:
        (1 - A D) psi' = (1 + A D) psi,   D = [1, -2, 1],  zero ghost values,
     A = i dt/(4 d^2) in real time and dt/(4 d^2) in imaginary time; solved by
     Thomas elimination without pivoting.
  3. Imaginary time only: psi <- psi / sqrt(sum |psi|^2 dV).

Variants of the same method (the paper's programs use the form above):
  - the symmetric (Strang) step: nonlinear over dt/2, the three sweeps over dt,
    nonlinear over dt/2 from the new density, then step 3;
  - propagation to the ground state in imaginary time, stopped when the
    chemical potential changes by less than a tolerance per step ("Solution
    method": imaginary-time propagation to the stationary state);
  - the quasi-two-dimensional equation of the 2d programs (program title;
    "Nature of problem": one, two and three spatial dimensions), the tight
    axis integrated out over its trap's Gaussian ground state (section below).

Parity pins (tests/test_oracle_pins.py): brute-force DFT convolution, radial
quadrature of the cut-off kernel, the closed-form dipolar energy of an
anisotropic Gaussian, dense linear solves, exact separable non-interacting
evolution (Lie and Strang), the harmonic ground-state energy (1 + lam + gam)/2,
norm conservation, time reversal (and the exact symmetry of the Strang step),
the second order in dt of the Strang step, the virial theorem, finite
differences of the adjoint, and for the quasi-2D equation: quadrature of the
3D kernel over the tight axis, the 3D closed-form dipolar energy of axially
symmetric Gaussians (with the L^-3 image tail), the contact energy of the
product state and exact separable non-interacting steps.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import Optional, Sequence, Tuple

import numpy as np
from scipy import special

__all__ = [
    "Params", "grid", "trap_base", "cutoff_factor", "dipolar_kernel",
    "dipolar_potential", "cn_coefficient", "cn_solve_axis", "kinetic_step",
    "nonlinear_step", "step", "strang_step", "evolve", "ground_state", "norm", "observables",
    "hamiltonian_apply", "energy_total", "adjoint_evolve", "overlap_objective",
    "Params2D", "q2d_kernel", "q2d_potential", "q2d_step", "q2d_evolve", "q2d_observables",
]


@dataclass(frozen=True)
class Params:
    """Discretisation and physics of one run (trap units)."""

    n: Tuple[int, int, int]
    d: Tuple[float, float, float]
    dt: float
    trap: Tuple[float, float, float]
    g: float
    gd: float
    imag: bool
    R: float = 0.0  # <= 0: min(N_i d_i)/2

    @property
    def cutoff(self) -> float:
        if self.R > 0:
            return float(self.R)
        return 0.5 * min(self.n[i] * self.d[i] for i in range(3))

    @property
    def dV(self) -> float:
        return self.d[0] * self.d[1] * self.d[2]

    @classmethod
    def from_config(cls, cfg, **override):
        kw = dict(n=tuple(cfg.n), d=tuple(cfg.d), dt=cfg.dt, trap=tuple(cfg.trap),
                  g=cfg.g, gd=cfg.gd, imag=cfg.imag, R=cfg.R)
        kw.update(override)
        return cls(**kw)


# ----------------------------------------------------------------------------
# Grid and potentials
# ----------------------------------------------------------------------------

def grid(p: Params):
    """Axis coordinates x_i = (i - N/2) dx (likewise y, z)."""
    return tuple((np.arange(p.n[a], dtype=np.float64) - p.n[a] // 2) * p.d[a] for a in range(3))


def trap_base(p: Params):
    """V0 = (nu^2 x^2 + lam^2 y^2 + gam^2 z^2) / 2 on the grid; the trap at time t
    is a(t) V0 (a = 1 for a static trap)."""
    x, y, z = grid(p)
    nu, lam, gam = p.trap
    return 0.5 * ((nu * x) ** 2)[:, None, None] + 0.5 * ((lam * y) ** 2)[None, :, None] \
        + 0.5 * ((gam * z) ** 2)[None, None, :]


def cutoff_factor(u):
    """Spherical cut-off factor F(u) = 1 + 3 cos(u)/u^2 - 3 sin(u)/u^3 of the dipolar
    kernel truncated at |r| = R (u = kR).  F -> u^2/10 as u -> 0 (series below
    u = 0.1, where the closed form cancels) and F -> 1 as u -> infinity."""
    u = np.asarray(u, dtype=np.float64)
    out = np.empty_like(u)
    small = u < 0.1
    us = u[small]
    out[small] = us ** 2 / 10.0 - us ** 4 / 280.0 + us ** 6 / 15120.0
    ul = u[~small]
    out[~small] = 1.0 + 3.0 * np.cos(ul) / ul ** 2 - 3.0 * np.sin(ul) / ul ** 3
    return out


def dipolar_kernel(p: Params):
    """U_R(k) on the half spectrum [Nx][Ny][Nz/2+1] of the real-to-complex DFT along z.

    k_a = 2 pi m / (N_a d_a) with m the signed DFT frequency index.  U_R(0) = 0
    (the angular factor averages out and F(0) = 0)."""
    nx, ny, nz = p.n
    kx = 2.0 * np.pi * np.fft.fftfreq(nx, d=p.d[0])
    ky = 2.0 * np.pi * np.fft.fftfreq(ny, d=p.d[1])
    kz = 2.0 * np.pi * np.fft.rfftfreq(nz, d=p.d[2])
    k2 = kx[:, None, None] ** 2 + ky[None, :, None] ** 2 + kz[None, None, :] ** 2
    kz2 = np.broadcast_to(kz[None, None, :] ** 2, k2.shape)
    k = np.sqrt(k2)
    U = np.zeros(k2.shape)
    nz0 = k2 > 0
    U[nz0] = (4.0 * np.pi / 3.0) * (3.0 * kz2[nz0] / k2[nz0] - 1.0) * cutoff_factor(k[nz0] * p.cutoff)
    return U


def dipolar_potential(p: Params, field):
    """Phi = IDFT[U_R . DFT[field]] for a real field on the grid: unnormalised
    forward transform, 1/N_t in the inverse, real-to-complex along z."""
    spec = np.fft.rfftn(field, axes=(0, 1, 2))
    return np.fft.irfftn(dipolar_kernel(p) * spec, s=p.n, axes=(0, 1, 2))


# ----------------------------------------------------------------------------
# Crank-Nicolson kinetic step
# ----------------------------------------------------------------------------

def cn_coefficient(p: Params, axis: int, conjugate: bool = False):
    """A = i dt/(4 d^2) (real time) or dt/(4 d^2) (imaginary time); conjugate=True
    gives conj(A), the coefficient of the adjoint sweep."""
    a = p.dt / (4.0 * p.d[axis] ** 2)
    A = 1j * a if not p.imag else complex(a)
    return np.conj(A) if conjugate else A


def cn_solve_axis(psi, A, axis: int):
    """One Crank-Nicolson sweep along `axis`: solve (1 - A D) out = (1 + A D) psi on
    every line, D the second difference with zero ghosts psi_{-1} = psi_N = 0, by
    Thomas elimination of tridiag(-A, 1 + 2A, -A) without pivoting (the matrix is
    strictly diagonally dominant)."""
    u = np.moveaxis(np.asarray(psi, dtype=np.complex128), axis, 0)
    N = u.shape[0]
    r = (1.0 - 2.0 * A) * u
    r[1:] += A * u[:-1]
    r[:-1] += A * u[1:]
    sub, diag, sup = -A, 1.0 + 2.0 * A, -A
    cp = np.empty(N, dtype=np.complex128)
    dp = np.empty_like(r)
    cp[0] = sup / diag
    dp[0] = r[0] / diag
    for i in range(1, N):
        piv = diag - sub * cp[i - 1]
        cp[i] = sup / piv
        dp[i] = (r[i] - sub * dp[i - 1]) / piv
    out = np.empty_like(r)
    out[N - 1] = dp[N - 1]
    for i in range(N - 2, -1, -1):
        out[i] = dp[i] - cp[i] * out[i + 1]
    return np.moveaxis(out, 0, axis)


def kinetic_step(p: Params, psi, conjugate: bool = False):
    """The three Crank-Nicolson sweeps, x then y then z (they act on different
    tensor factors and commute exactly)."""
    for axis in (0, 1, 2):
        psi = cn_solve_axis(psi, cn_coefficient(p, axis, conjugate), axis)
    return psi


# ----------------------------------------------------------------------------
# Nonlinear step, full step
# ----------------------------------------------------------------------------

def phase_theta(p: Params, psi, a: float = 1.0, V0=None):
    """theta = dt (a V0 + g |psi|^2 + gd Phi[|psi|^2]) from the pre-step density."""
    if V0 is None:
        V0 = trap_base(p)
    dens = np.abs(psi) ** 2
    th = a * V0 + p.g * dens
    if p.gd != 0.0:
        th = th + p.gd * dipolar_potential(p, dens)
    return p.dt * th


def nonlinear_step(p: Params, psi, a: float = 1.0, V0=None):
    """psi exp(-i theta) in real time, psi exp(-theta) in imaginary time."""
    th = phase_theta(p, psi, a, V0)
    if p.imag:
        return psi * np.exp(-th)
    return psi * np.exp(-1j * th)


def norm(p: Params, psi) -> float:
    """sum |psi|^2 dV (rectangle rule)."""
    return float(np.sum(np.abs(psi) ** 2) * p.dV)


def step(p: Params, psi, a: float = 1.0, V0=None):
    """One split step: nonlinear, then the Crank-Nicolson sweeps, then (imaginary
    time) renormalisation to unit norm."""
    psi = nonlinear_step(p, psi, a, V0)
    psi = kinetic_step(p, psi)
    if p.imag:
        psi = psi / np.sqrt(norm(p, psi))
    return psi


def strang_step(p: Params, psi, a: float = 1.0, V0=None):
    """One symmetric (Strang) split step, the second-order variant of the same
    splitting: the nonlinear step over dt/2 from the density of the incoming
    state, the Crank-Nicolson sweeps over the full dt, the nonlinear step over
    dt/2 from the density after the sweeps; then (imaginary time)
    renormalisation to unit norm.  Both halves use the trap amplitude a of the
    step."""
    half = replace(p, dt=0.5 * p.dt)
    psi = nonlinear_step(half, psi, a, V0)
    psi = kinetic_step(p, psi)
    psi = nonlinear_step(half, psi, a, V0)
    if p.imag:
        psi = psi / np.sqrt(norm(p, psi))
    return psi


SCHEMES = {"lie": step, "strang": strang_step}


def evolve(p: Params, psi, nsteps: int, amp: Optional[Sequence[float]] = None,
           scheme: str = "lie"):
    """nsteps split steps; amp[n] is the trap amplitude a(t_n) of step n (1 if None).
    scheme: "lie" (first order, the paper's form) or "strang" (second order)."""
    one = SCHEMES[scheme]
    V0 = trap_base(p)
    psi = np.array(psi, dtype=np.complex128, copy=True)
    for n in range(nsteps):
        psi = one(p, psi, 1.0 if amp is None else float(amp[n]), V0)
    return psi


def ground_state(p: Params, psi0, tol: float, max_steps: int, check_every: int = 1,
                 scheme: str = "lie"):
    """Imaginary-time propagation to the stationary state, stopped on the change
    of the chemical potential.  mu is evaluated on psi0 and after every
    check_every steps; the run stops at the first evaluation where
    |mu_now - mu_before| / (steps between them) < tol, or after max_steps steps.

    Returns (psi, steps done, the last |delta mu| per step, mu of psi)."""
    assert p.imag and tol > 0 and max_steps >= 0 and check_every >= 1
    one = SCHEMES[scheme]
    V0 = trap_base(p)
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    mu = observables(p, psi)["mu"]
    done, rate = 0, float("inf")
    while done < max_steps:
        k = min(check_every, max_steps - done)
        for _ in range(k):
            psi = one(p, psi, 1.0, V0)
        done += k
        mu_new = observables(p, psi)["mu"]
        rate = abs(mu_new - mu) / k
        mu = mu_new
        if rate < tol:
            break
    return psi, done, rate, mu


# ----------------------------------------------------------------------------
# Observables
# ----------------------------------------------------------------------------

def _forward_differences(psi, axis):
    """psi_{i+1} - psi_i for i = -1 .. N-1 with zero ghosts (N + 1 differences)."""
    pad = [(0, 0)] * 3
    pad[axis] = (1, 1)
    return np.diff(np.pad(psi, pad), axis=axis)


def observables(p: Params, psi, a: float = 1.0):
    """Norm, chemical potential, energy (and parts) and rms sizes.

    E_kin = 1/2 sum_axes sum |psi_{i+1} - psi_i|^2 / d^2 dV (ghost zeros; equal to
    -1/2 <psi, D psi>/d^2 summed by parts), E_trap = sum a V0 |psi|^2 dV,
    E_c = g/2 sum |psi|^4 dV, E_dd = gd/2 sum Phi |psi|^2 dV.
    E = (E_kin + E_trap + E_c + E_dd)/norm, mu = (E_kin + E_trap + 2 E_c + 2 E_dd)/norm.
    rms sizes are second moments about the origin divided by the norm."""
    dV = p.dV
    dens = np.abs(psi) ** 2
    nrm = float(np.sum(dens) * dV)
    ekin = 0.0
    for axis in range(3):
        df = _forward_differences(psi, axis)
        ekin += 0.5 * float(np.sum(np.abs(df) ** 2)) / p.d[axis] ** 2 * dV
    etrap = float(np.sum(a * trap_base(p) * dens) * dV)
    ec = 0.5 * p.g * float(np.sum(dens * dens) * dV)
    edd = 0.5 * p.gd * float(np.sum(dipolar_potential(p, dens) * dens) * dV) if p.gd != 0.0 else 0.0
    x, y, z = grid(p)
    mx = float(np.sum(dens * (x ** 2)[:, None, None]) * dV) / nrm
    my = float(np.sum(dens * (y ** 2)[None, :, None]) * dV) / nrm
    mz = float(np.sum(dens * (z ** 2)[None, None, :]) * dV) / nrm
    return {
        "norm": nrm,
        "mu": (ekin + etrap + 2.0 * ec + 2.0 * edd) / nrm,
        "energy": (ekin + etrap + ec + edd) / nrm,
        "e_kin": ekin, "e_trap": etrap, "e_contact": ec, "e_dd": edd,
        "rms": (np.sqrt(mx), np.sqrt(my), np.sqrt(mz), np.sqrt(mx + my + mz)),
    }


def energy_total(p: Params, psi, a: float = 1.0) -> float:
    """E_kin + E_trap + E_c + E_dd, not divided by the norm (the real-time
    objective of the adjoint)."""
    o = observables(p, psi, a)
    return o["e_kin"] + o["e_trap"] + o["e_contact"] + o["e_dd"]


def laplacian(p: Params, psi):
    """Sum over axes of the 3-point second difference / d^2 with zero ghosts."""
    out = np.zeros_like(psi)
    for axis in range(3):
        u = np.moveaxis(psi, axis, 0)
        lap = -2.0 * u
        lap[1:] += u[:-1]
        lap[:-1] += u[1:]
        out += np.moveaxis(lap, 0, axis) / p.d[axis] ** 2
    return out


def hamiltonian_apply(p: Params, psi, a: float = 1.0):
    """H psi = (-1/2 Lap_D + a V0 + g |psi|^2 + gd Phi[|psi|^2]) psi."""
    dens = np.abs(psi) ** 2
    pot = a * trap_base(p) + p.g * dens
    if p.gd != 0.0:
        pot = pot + p.gd * dipolar_potential(p, dens)
    return -0.5 * laplacian(p, psi) + pot * psi


# ----------------------------------------------------------------------------
# Adjoint (real time)
# ----------------------------------------------------------------------------

def overlap_objective(p: Params, psi, target):
    """J = |sum conj(target) psi dV|^2 and its cotangent 2 dV c target."""
    c = complex(np.sum(np.conj(target) * psi) * p.dV)
    return abs(c) ** 2, 2.0 * p.dV * c * target


def adjoint_evolve(p: Params, psi0, amp: Sequence[float], objective: str = "energy",
                   target=None):
    """Reverse-mode derivative of a final-state objective through nsteps real-time
    split steps.

    amp has nsteps + 1 entries: amp[n] is a(t_n) for the step starting at t_n and
    amp[nsteps] is a(T), the amplitude in the final energy.  The inner product is
    <u, v> = Re sum conj(u) v (no dV), and the cotangent lam satisfies
    dJ = <lam, dpsi>.  For psi_{n+1} = C psi', psi' = exp(-i theta) psi_n:
      mu = C^H lam_{n+1}       (Crank-Nicolson with conj(A), sweeps commute)
      s  = Im(conj(mu) psi')
      w  = dt (g s + gd Phi[s])                (Phi is self-adjoint: real even U)
      lam_n = exp(+i theta) mu + 2 w psi_n
      dJ/da_n += dt sum s V0,  dJ/dtrap_j += dt sum s a_n trap_j x_j^2.
    Energy seed: lam_N = 2 dV H psi_N; dJ/da_N = dV sum V0 |psi_N|^2 and
    dJ/dtrap_j = dV sum a_N trap_j x_j^2 |psi_N|^2.

    Returns (J, psi_N, dJ/damp [nsteps+1], dJ/dtrap [3], lam_0 = dJ/dpsi0)."""
    if p.imag:
        raise ValueError("the adjoint is defined for real-time propagation")
    nsteps = len(amp) - 1
    V0 = trap_base(p)
    x, y, z = grid(p)
    coord2 = ((x ** 2)[:, None, None], (y ** 2)[None, :, None], (z ** 2)[None, None, :])
    states = [np.array(psi0, dtype=np.complex128, copy=True)]
    for n in range(nsteps):
        states.append(step(p, states[-1], float(amp[n]), V0))
    psiN = states[-1]
    dJ_da = np.zeros(nsteps + 1)
    dJ_dtrap = np.zeros(3)
    aN = float(amp[nsteps])
    if objective == "energy":
        J = energy_total(p, psiN, aN)
        lam = 2.0 * p.dV * hamiltonian_apply(p, psiN, aN)
        densN = np.abs(psiN) ** 2
        dJ_da[nsteps] = p.dV * float(np.sum(V0 * densN))
        for j in range(3):
            dJ_dtrap[j] = p.dV * aN * p.trap[j] * float(np.sum(coord2[j] * densN))
    elif objective == "overlap":
        J, lam = overlap_objective(p, psiN, target)
    else:
        raise ValueError(objective)
    for n in range(nsteps - 1, -1, -1):
        an = float(amp[n])
        mu = kinetic_step(p, lam, conjugate=True)
        psin = states[n]
        th = phase_theta(p, psin, an, V0)
        psip = np.exp(-1j * th) * psin
        s = np.imag(np.conj(mu) * psip)
        w = p.g * s
        if p.gd != 0.0:
            w = w + p.gd * dipolar_potential(p, s)
        w = p.dt * w
        lam = np.exp(1j * th) * mu + 2.0 * w * psin
        dJ_da[n] += p.dt * float(np.sum(s * V0))
        for j in range(3):
            dJ_dtrap[j] += p.dt * an * p.trap[j] * float(np.sum(s * coord2[j]))
    return J, psiN, dJ_da, dJ_dtrap, lam


# ----------------------------------------------------------------------------
# Quasi-two-dimensional programs (the paper's 2d programs)
# ----------------------------------------------------------------------------
#
# A condensate held by a tight harmonic trap of frequency nu_t along one axis
# stays in that trap's Gaussian ground state phi(t) = exp(-t^2/(2 l^2)) /
# (pi l^2)^(1/4), l = 1/sqrt(nu_t); integrating the 3D equation over that axis
# leaves a 2D equation for psi(a, b) on the plane (axes a = first, b = second,
# [Na][Nb] with b contiguous):
#   contact  g2 = g int phi^4 dt = g / (sqrt(2 pi) l)
#   dipolar  U2(q) = int dk_t/(2 pi) U(q, k_t) exp(-k_t^2 l^2 / 2) with the 3D
#            kernel U(k) = (4 pi/3)(3 cos^2 - 1) of dipoles along a fixed axis
#            (no spherical cut-off; the plane's own sum has none either):
#     dipoles along the tight axis ("perp", the XY programs):
#       U2(q) = (4 pi/3) / (sqrt(2 pi) l) [2 - 3 F(q l / sqrt 2)]
#     dipoles along the plane's axis b ("inplane", the XZ programs):
#       U2(q) = (4 pi/3) / (sqrt(2 pi) l) [-1 + 3 (q_b^2/q^2) F(q l / sqrt 2)]
#     with F(u) = sqrt(pi) u exp(u^2) erfc(u) (F(0) = 0, F -> 1 as u -> inf).
#   trap V = a/2 (nu_a^2 a^2 + nu_b^2 b^2); the tight axis' constant energy
#   nu_t/2 is left out of every reported energy.
# One step is the 3D step with two Crank-Nicolson sweeps (a and b).

@dataclass(frozen=True)
class Params2D:
    """Quasi-2D run: plane grid n = (Na, Nb), spacings d, in-plane trap
    (nu_a, nu_b), tight-axis frequency nu_t, 3D couplings g, gd, and the dipole
    orientation "perp" (along the tight axis) or "inplane" (along axis b)."""

    n: Tuple[int, int]
    d: Tuple[float, float]
    dt: float
    trap: Tuple[float, float]
    nu_t: float
    g: float
    gd: float
    imag: bool
    dipoles: str = "perp"

    @property
    def ell(self) -> float:
        return 1.0 / np.sqrt(self.nu_t)

    @property
    def g2(self) -> float:
        return self.g / (np.sqrt(2.0 * np.pi) * self.ell)

    @property
    def dA(self) -> float:
        return self.d[0] * self.d[1]


def q2d_grid(p: Params2D):
    return tuple((np.arange(p.n[a], dtype=np.float64) - p.n[a] // 2) * p.d[a] for a in range(2))


def q2d_trap(p: Params2D):
    xa, xb = q2d_grid(p)
    return 0.5 * ((p.trap[0] * xa) ** 2)[:, None] + 0.5 * ((p.trap[1] * xb) ** 2)[None, :]


def q2d_kernel(p: Params2D):
    """U2 on the half spectrum [Na][Nb/2+1] of the real-to-complex DFT along b."""
    qa = 2.0 * np.pi * np.fft.fftfreq(p.n[0], d=p.d[0])
    qb = 2.0 * np.pi * np.fft.rfftfreq(p.n[1], d=p.d[1])
    q2 = qa[:, None] ** 2 + qb[None, :] ** 2
    u = np.sqrt(q2) * p.ell / np.sqrt(2.0)
    F = np.sqrt(np.pi) * u * special.erfcx(u)
    pre = (4.0 * np.pi / 3.0) / (np.sqrt(2.0 * np.pi) * p.ell)
    if p.dipoles == "perp":
        return pre * (2.0 - 3.0 * F)
    if p.dipoles == "inplane":
        ratio = np.zeros_like(q2)
        nz = q2 > 0
        ratio[nz] = np.broadcast_to(qb[None, :] ** 2, q2.shape)[nz] / q2[nz]
        return pre * (-1.0 + 3.0 * ratio * F)
    raise ValueError(p.dipoles)


def q2d_potential(p: Params2D, field):
    spec = np.fft.rfftn(field, axes=(0, 1))
    return np.fft.irfftn(q2d_kernel(p) * spec, s=p.n, axes=(0, 1))


def q2d_step(p: Params2D, psi, a: float = 1.0):
    """Nonlinear step (pre-step density), Crank-Nicolson along a and b, then
    (imaginary time) renormalisation to sum |psi|^2 dA = 1."""
    dens = np.abs(psi) ** 2
    th = a * q2d_trap(p) + p.g2 * dens
    if p.gd != 0.0:
        th = th + p.gd * q2d_potential(p, dens)
    th = p.dt * th
    psi = psi * (np.exp(-th) if p.imag else np.exp(-1j * th))
    for axis in (0, 1):
        c = p.dt / (4.0 * p.d[axis] ** 2)
        psi = cn_solve_axis(psi, complex(c) if p.imag else 1j * c, axis)
    if p.imag:
        psi = psi / np.sqrt(np.sum(np.abs(psi) ** 2) * p.dA)
    return psi


def q2d_evolve(p: Params2D, psi, nsteps: int):
    psi = np.array(psi, dtype=np.complex128, copy=True)
    for _ in range(nsteps):
        psi = q2d_step(p, psi)
    return psi


def q2d_observables(p: Params2D, psi, a: float = 1.0):
    """As observables() on the plane: E_kin over the two axes (ghost zeros),
    E_trap, E_c = g2/2 sum n^2, E_dd = gd/2 sum Phi n, all times dA; rms sizes
    along a and b and in the plane."""
    dA = p.dA
    dens = np.abs(psi) ** 2
    nrm = float(np.sum(dens) * dA)
    ekin = 0.0
    for axis in range(2):
        pad = [(0, 0)] * 2
        pad[axis] = (1, 1)
        df = np.diff(np.pad(psi, pad), axis=axis)
        ekin += 0.5 * float(np.sum(np.abs(df) ** 2)) / p.d[axis] ** 2 * dA
    etrap = float(np.sum(a * q2d_trap(p) * dens) * dA)
    ec = 0.5 * p.g2 * float(np.sum(dens * dens) * dA)
    edd = 0.5 * p.gd * float(np.sum(q2d_potential(p, dens) * dens) * dA) if p.gd != 0.0 else 0.0
    xa, xb = q2d_grid(p)
    ma = float(np.sum(dens * (xa ** 2)[:, None]) * dA) / nrm
    mb = float(np.sum(dens * (xb ** 2)[None, :]) * dA) / nrm
    return {
        "norm": nrm,
        "mu": (ekin + etrap + 2.0 * ec + 2.0 * edd) / nrm,
        "energy": (ekin + etrap + ec + edd) / nrm,
        "e_kin": ekin, "e_trap": etrap, "e_contact": ec, "e_dd": edd,
        "rms": (np.sqrt(ma), np.sqrt(mb), np.sqrt(ma + mb)),
    }
