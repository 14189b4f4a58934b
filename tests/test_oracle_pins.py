"""Pins of the FP64 oracle against facts other than itself.

Each test checks the oracle against a closed form, an invariant, a dense linear
solve, a brute-force sum or a quadrature, chosen so that a plausible mistake in
the oracle (a dropped term, a wrong sign or index, a transposed axis, a wrong
normalisation) fails at least one of them.  No GPU is needed.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import dgpe_oracle as O
import workloads as W


def _params(n, d, dt=0.01, trap=(1.0, 1.0, 1.0), g=0.0, gd=0.0, imag=False, R=0.0):
    return O.Params(n=tuple(n), d=tuple(d), dt=dt, trap=tuple(trap), g=g, gd=gd, imag=imag, R=R)


# ---------------------------------------------------------------------------
# Dipolar kernel and potential
# ---------------------------------------------------------------------------

def _cutoff_by_quadrature(u):
    """3 * integral_0^u j2(t)/t dt: the radial part of the Fourier transform of
    (1 - 3 cos^2)/r^3 restricted to r < R, written through the partial-wave
    expansion of exp(-i k.r) (a route independent of the closed form)."""
    val, _ = integrate.quad(lambda t: special.spherical_jn(2, t) / t, 0.0, u, limit=400,
                            epsabs=1e-15, epsrel=1e-13)
    return 3.0 * val


@pytest.mark.parametrize("u", [0.02, 0.09, 0.11, 0.5, 1.0, math.pi, 7.3, 40.0])
def test_cutoff_factor_matches_radial_quadrature(u):
    got = float(O.cutoff_factor(np.array([u]))[0])
    ref = _cutoff_by_quadrature(u)
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)) + 1e-15


def test_cutoff_factor_limits():
    # F -> u^2/10 for small u, F -> 1 for large u
    assert abs(float(O.cutoff_factor(np.array([1e-3]))[0]) / 1e-7 - 1.0) < 1e-5
    assert abs(float(O.cutoff_factor(np.array([1e4]))[0]) - 1.0) < 1e-7


def _bruteforce_potential(n, d, R, field):
    """Circular convolution through an explicit O(N^2) DFT along each axis, with the
    kernel evaluated on the full (not half) spectrum from the quadrature form."""
    mats, ks = [], []
    for a in range(3):
        m = np.arange(n[a])
        mats.append(np.exp(-2j * np.pi * np.outer(m, m) / n[a]))
        signed = np.where(m <= n[a] // 2, m, m - n[a])
        ks.append(2 * np.pi * signed / (n[a] * d[a]))
    spec = np.einsum("ai,bj,ck,ijk->abc", mats[0], mats[1], mats[2], field)
    U = np.zeros(n)
    for i in range(n[0]):
        for j in range(n[1]):
            for l in range(n[2]):
                k2 = ks[0][i] ** 2 + ks[1][j] ** 2 + ks[2][l] ** 2
                if k2 == 0:
                    continue
                ang = 3.0 * ks[2][l] ** 2 / k2 - 1.0
                U[i, j, l] = 4 * np.pi / 3 * ang * _cutoff_by_quadrature(math.sqrt(k2) * R)
    back = np.einsum("ai,bj,ck,ijk->abc", mats[0].conj(), mats[1].conj(), mats[2].conj(), U * spec)
    return (back / field.size).real


@pytest.mark.parametrize("n", [(4, 6, 8), (6, 4, 5)])
def test_potential_matches_bruteforce_dft(n):
    d = (0.7, 0.5, 0.4)
    R = 1.1
    rng = np.random.default_rng(11)
    field = rng.uniform(0.0, 1.0, size=n)
    p = _params(n, d, R=R, gd=1.0)
    got = O.dipolar_potential(p, field)
    ref = _bruteforce_potential(n, d, R, field)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [(4, 6, 8), (6, 4, 5)])
def test_potential_default_cutoff_is_half_the_shortest_box_side(n):
    """With R left at its default (R <= 0), the potential equals the brute-force
    convolution with R = min_i(N_i d_i)/2, the written reading of the default
    cut-off.  On (4, 6, 8) the shortest side is x, on (6, 4, 5) it is y and z,
    so a default taken from one fixed axis fails one of the two."""
    d = (0.7, 0.5, 0.4)
    R_ref = 0.5 * min(n[a] * d[a] for a in range(3))
    rng = np.random.default_rng(12)
    field = rng.uniform(0.0, 1.0, size=n)
    got = O.dipolar_potential(_params(n, d, gd=1.0), field)
    ref = _bruteforce_potential(n, d, R_ref, field)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    # and a different radius gives a measurably different potential
    other = _bruteforce_potential(n, d, 0.5 * n[0] * d[0] * 1.5, field)
    assert np.max(np.abs(other - ref)) > 1e-3 * np.max(np.abs(ref))


def test_isotropic_density_has_zero_dipolar_energy():
    # A spherically symmetric density on a cubic grid: the angular factor
    # 3 kz^2/k^2 - 1 averages to zero over the x<->y<->z permutations of k.
    n, d = (32, 32, 32), (0.4, 0.4, 0.4)
    p = _params(n, d, gd=1.0)
    psi = W.gaussian_state(n, d, (1.0, 1.0, 1.0))
    dens = np.abs(psi) ** 2
    edd = 0.5 * np.sum(O.dipolar_potential(p, dens) * dens) * p.dV
    assert abs(edd) < 1e-15


def _edd_gaussian_closed(sr, sz):
    """Dipolar energy (gd = 1, no cut-off) of the unit-norm density
    exp(-rho^2/sr^2 - z^2/sz^2)/(pi^1.5 sr^2 sz): by Parseval,
    E = 1/2 (2 pi)^-3 int (4 pi/3)(3 cos^2 a - 1) |n~(k)|^2 d^3k with
    |n~|^2 = exp(-k^2 (sr^2 sin^2 a + sz^2 cos^2 a)/2); the radial integral is
    sqrt(pi/2) s^-3 and the angular one is done by quadrature."""
    ang, _ = integrate.quad(lambda u: (3 * u * u - 1) / (sr ** 2 + (sz ** 2 - sr ** 2) * u * u) ** 1.5,
                            -1.0, 1.0, epsabs=1e-15, epsrel=1e-13)
    return 0.5 * (2 * np.pi) ** -3 * (4 * np.pi / 3) * (2 * np.pi) * math.sqrt(np.pi / 2) * ang


def _edd_gaussian_kappa(sr, sz):
    """The same energy through the elementary closed form in kappa = sr/sz:
    E = -f(kappa) / (3 sqrt(2 pi) sr^2 sz), f = (1 + 2k^2)/(1 - k^2)
    - 3 k^2 artanh(sqrt(1 - k^2))/(1 - k^2)^1.5 (analytic continuation for k > 1)."""
    k = sr / sz
    if k < 1:
        s = math.sqrt(1 - k * k)
        f = (1 + 2 * k * k) / (1 - k * k) - 3 * k * k * math.atanh(s) / (1 - k * k) ** 1.5
    else:
        s = math.sqrt(k * k - 1)
        f = (1 + 2 * k * k) / (1 - k * k) - 3 * k * k * math.atan(s) / ((1 - k * k) * s)
    return -f / (3 * math.sqrt(2 * np.pi) * sr * sr * sz)


@pytest.mark.parametrize("sr,sz", [(1.0, 0.6), (1.0, 1.6), (0.8, 2.0), (1.5, 0.5)])
def test_dipolar_energy_of_anisotropic_gaussian(sr, sz):
    closed = _edd_gaussian_closed(sr, sz)
    assert abs(_edd_gaussian_kappa(sr, sz) - closed) < 1e-12 * abs(closed)
    # box L = 32 and cut-off R = 16: both the cut-off and the periodic images are
    # far outside the density's autocorrelation, so the grid value must reach the
    # uncut closed form to near rounding
    n, d = (128, 128, 256), (0.25, 0.25, 0.125)
    p = _params(n, d, gd=1.0)
    x, y, z = O.grid(p)
    rho2 = (x ** 2)[:, None, None] + (y ** 2)[None, :, None]
    dens = np.exp(-rho2 / sr ** 2 - (z ** 2)[None, None, :] / sz ** 2) / (np.pi ** 1.5 * sr * sr * sz)
    psi = np.sqrt(dens).astype(np.complex128)
    edd = O.observables(p, psi)["e_dd"]
    assert abs(edd - closed) < 1e-11 * abs(closed)


# ---------------------------------------------------------------------------
# Crank-Nicolson sweeps
# ---------------------------------------------------------------------------

def _dense_cn(u, A, axis):
    N = u.shape[axis]
    D = -2 * np.eye(N) + np.eye(N, k=1) + np.eye(N, k=-1)
    lhs = np.eye(N) - A * D
    rhs_op = np.eye(N) + A * D
    v = np.moveaxis(u, axis, 0).reshape(N, -1)
    out = np.linalg.solve(lhs, rhs_op @ v)
    return np.moveaxis(out.reshape(np.moveaxis(u, axis, 0).shape), 0, axis)


@pytest.mark.parametrize("imag", [False, True])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_cn_sweep_matches_dense_solve(imag, axis):
    n, d = (5, 6, 7), (0.3, 0.2, 0.25)
    p = _params(n, d, dt=0.03, imag=imag)
    rng = np.random.default_rng(3 + axis)
    u = rng.normal(size=n) + 1j * rng.normal(size=n)
    A = O.cn_coefficient(p, axis)
    assert (A.imag == 0) == imag
    assert abs(abs(A) - 0.03 / (4 * d[axis] ** 2)) < 1e-15
    got = O.cn_solve_axis(u, A, axis)
    ref = _dense_cn(u, A, axis)
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))


def test_cn_real_time_is_unitary_and_commutes():
    n, d = (9, 10, 11), (0.2, 0.25, 0.3)
    p = _params(n, d, dt=0.05)
    psi = W.random_state(n, d, seed=5)
    out = O.kinetic_step(p, psi)
    assert abs(O.norm(p, out) - O.norm(p, psi)) < 1e-14
    ax = [O.cn_coefficient(p, a) for a in range(3)]
    zyx = O.cn_solve_axis(O.cn_solve_axis(O.cn_solve_axis(psi, ax[2], 2), ax[1], 1), ax[0], 0)
    assert np.max(np.abs(zyx - out)) < 1e-14


# ---------------------------------------------------------------------------
# Whole steps
# ---------------------------------------------------------------------------

def _axis_transfer(p, axis, a=1.0):
    """Dense one-axis transfer matrix C_axis diag(exp(-i dt a V_axis)) (real time) or
    C_axis diag(exp(-dt a V_axis)) (imaginary time), V_axis = trap^2 x^2 / 2."""
    N = p.n[axis]
    x = (np.arange(N) - N // 2) * p.d[axis]
    v = 0.5 * (p.trap[axis] * x) ** 2
    phase = np.exp(-p.dt * a * v) if p.imag else np.exp(-1j * p.dt * a * v)
    A = p.dt / (4 * p.d[axis] ** 2) * (1.0 if p.imag else 1j)
    D = -2 * np.eye(N) + np.eye(N, k=1) + np.eye(N, k=-1)
    C = np.linalg.solve(np.eye(N) - A * D, np.eye(N) + A * D)
    return C @ np.diag(phase)


@pytest.mark.parametrize("imag", [False, True])
def test_noninteracting_step_is_exactly_separable(imag):
    n, d = (10, 12, 14), (0.4, 0.3, 0.35)
    p = _params(n, d, dt=0.02, trap=(1.0, 1.3, 2.1), imag=imag)
    rng = np.random.default_rng(7)
    f = [rng.normal(size=n[a]) + 1j * rng.normal(size=n[a]) for a in range(3)]
    psi0 = np.einsum("i,j,k->ijk", *f)
    steps = 15
    got = O.evolve(p, psi0, steps)
    g = [np.linalg.matrix_power(_axis_transfer(p, a), steps) @ f[a] for a in range(3)]
    ref = np.einsum("i,j,k->ijk", *g)
    if imag:
        ref = ref / math.sqrt(np.sum(np.abs(ref) ** 2) * p.dV)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_noninteracting_ground_state_energy():
    # Imaginary-time fixed point of the non-interacting step: the product of the
    # dominant eigenvectors of the one-axis transfer matrices.  Its energy tends to
    # (nu + lam + gam)/2 with O(dx^2) + O(dt) error.
    trap = (1.0, 1.5, 2.0)
    errs = []
    for h, dt in [(0.2, 0.004), (0.1, 0.001)]:
        n = (int(round(12 / h)),) * 3
        p = _params(n, (h, h, h), dt=dt, trap=trap, imag=True)
        vecs = []
        for a in range(3):
            w, v = np.linalg.eig(_axis_transfer(p, a))
            vecs.append(v[:, np.argmax(np.abs(w))])
        psi = np.einsum("i,j,k->ijk", *vecs)
        psi = psi / math.sqrt(O.norm(p, psi))
        # the fixed point is invariant under one more oracle step
        assert np.max(np.abs(np.abs(O.step(p, psi)) - np.abs(psi))) < 1e-10 * np.max(np.abs(psi))
        obs = O.observables(p, psi)
        errs.append(abs(obs["energy"] - sum(trap) / 2))
        for a in range(3):
            assert abs(obs["rms"][a] - 1 / math.sqrt(2 * trap[a])) < 5 * h * h
    assert errs[0] < 1.5e-2 and errs[1] < 4e-3 and errs[1] < errs[0] / 3


def test_gaussian_observables_closed_forms():
    trap = (1.0, 1.4, 0.7)
    n, d = (64, 64, 80), (0.2, 0.2, 0.25)
    p = _params(n, d, trap=trap)
    psi = W.gaussian_state(n, d, trap)
    o = O.observables(p, psi)
    assert abs(o["norm"] - 1) < 1e-12
    assert abs(o["e_trap"] - sum(trap) / 4) < 1e-10
    # the 3-point kinetic energy of a Gaussian is (nu+lam+gam)/4 up to O(d^2)
    exact_kin = sum(trap) / 4
    assert abs(o["e_kin"] - exact_kin) < 0.02 * exact_kin
    for a in range(3):
        assert abs(o["rms"][a] - 1 / math.sqrt(2 * trap[a])) < 1e-10
    assert abs(o["rms"][3] - math.sqrt(sum(1 / (2 * t) for t in trap))) < 1e-10


def test_real_time_conserves_norm_and_reverses():
    n, d = (16, 16, 20), (0.35, 0.35, 0.3)
    p = _params(n, d, dt=0.004, trap=(1.0, 1.0, 2.0), g=30.0, gd=12.0)
    psi0 = W.random_state(n, d, seed=9)
    psi = O.evolve(p, psi0, 25)
    assert abs(O.norm(p, psi) - 1.0) < 1e-13
    # The inverse step: Crank-Nicolson with -dt, then the phase with -dt, which
    # sees the same density because the phase preserves |psi|.
    back = _params(n, d, dt=-0.004, trap=(1.0, 1.0, 2.0), g=30.0, gd=12.0)
    for _ in range(25):
        psi = O.nonlinear_step(back, O.kinetic_step(back, psi))
    assert np.max(np.abs(psi - psi0)) < 1e-12 * np.max(np.abs(psi0))


def test_real_time_energy_drift_is_first_order_in_dt():
    # With consistent signs of the kinetic, trap and interaction parts the split
    # step conserves the energy up to the splitting error, which shrinks with dt.
    n, d = (20, 20, 20), (0.4, 0.4, 0.4)
    cfg = W.Config("t", n, d, 0.0, (1.0, 1.0, 1.5), 25.0, 10.0, True, 0)
    psi0 = W.gaussian_state(n, d, (0.8, 0.8, 1.0))
    drifts = []
    for dt in (0.004, 0.002):
        p = O.Params.from_config(cfg, dt=dt, imag=False)
        e0 = O.observables(p, psi0)["energy"]
        psi = O.evolve(p, psi0, int(round(0.2 / dt)))
        drifts.append(abs(O.observables(p, psi)["energy"] - e0))
    assert drifts[0] < 2e-3
    assert drifts[1] < 0.7 * drifts[0]


def test_interacting_ground_state_virial_and_eigen_residual():
    # For the ground state of the dipolar GPE, 2 E_kin - 2 E_trap + 3 E_c + 3 E_dd = 0
    # (dilation of the state), and H psi = mu psi.
    n, d = (24, 24, 24), (0.45, 0.45, 0.45)
    p = _params(n, d, dt=0.002, trap=(1.0, 1.0, 1.4), g=20.0, gd=8.0, imag=True)
    psi = W.gaussian_state(n, d, p.trap)
    psi = O.evolve(p, psi, 1500)
    o = O.observables(p, psi)
    scale = o["e_kin"] + o["e_trap"] + o["e_contact"] + abs(o["e_dd"])
    vir = 2 * o["e_kin"] - 2 * o["e_trap"] + 3 * o["e_contact"] + 3 * o["e_dd"]
    assert abs(vir) < 0.02 * scale
    res = O.hamiltonian_apply(p, psi) - o["mu"] * psi
    assert np.linalg.norm(res) < 0.02 * o["mu"] * np.linalg.norm(psi)
    assert o["e_dd"] < 0  # elongated along the dipoles (gam < lam): attractive


# ---------------------------------------------------------------------------
# Strang splitting and the ground-state driver
# ---------------------------------------------------------------------------

def _axis_transfer_strang(p, axis, a=1.0):
    """Dense one-axis transfer matrix of the symmetric step: half the trap phase,
    the Crank-Nicolson solve, the other half of the trap phase."""
    N = p.n[axis]
    x = (np.arange(N) - N // 2) * p.d[axis]
    v = 0.5 * (p.trap[axis] * x) ** 2
    half = np.exp(-0.5 * p.dt * a * v) if p.imag else np.exp(-0.5j * p.dt * a * v)
    A = p.dt / (4 * p.d[axis] ** 2) * (1.0 if p.imag else 1j)
    D = -2 * np.eye(N) + np.eye(N, k=1) + np.eye(N, k=-1)
    C = np.linalg.solve(np.eye(N) - A * D, np.eye(N) + A * D)
    return np.diag(half) @ C @ np.diag(half)


@pytest.mark.parametrize("imag", [False, True])
def test_strang_noninteracting_step_is_exactly_separable(imag):
    n, d = (10, 12, 14), (0.4, 0.3, 0.35)
    p = _params(n, d, dt=0.02, trap=(1.0, 1.3, 2.1), imag=imag)
    rng = np.random.default_rng(8)
    f = [rng.normal(size=n[a]) + 1j * rng.normal(size=n[a]) for a in range(3)]
    psi0 = np.einsum("i,j,k->ijk", *f)
    steps = 15
    got = O.evolve(p, psi0, steps, scheme="strang")
    g = [np.linalg.matrix_power(_axis_transfer_strang(p, a), steps) @ f[a] for a in range(3)]
    ref = np.einsum("i,j,k->ijk", *g)
    if imag:
        ref = ref / math.sqrt(np.sum(np.abs(ref) ** 2) * p.dV)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
    # and it differs from the first-order step by more than rounding
    lie = O.evolve(p, psi0, steps)
    assert np.max(np.abs(got - lie)) > 1e-6 * np.max(np.abs(ref))


def _interacting_real(dt):
    n, d = (16, 16, 16), (0.45, 0.45, 0.45)
    return _params(n, d, dt=dt, trap=(1.0, 1.2, 1.6), g=25.0, gd=10.0)


def test_strang_step_is_second_order_in_dt():
    """At a fixed final time, halving dt shrinks the change of the final state
    about fourfold for the symmetric step and about twofold for the
    first-order one."""
    psi0 = W.random_state((16, 16, 16), (0.45,) * 3, seed=17)
    T = 0.08
    ratios = {}
    for scheme in ("strang", "lie"):
        finals = []
        for dt in (0.008, 0.004, 0.002):
            p = _interacting_real(dt)
            finals.append(O.evolve(p, psi0, int(round(T / dt)), scheme=scheme))
        e1 = np.linalg.norm(finals[0] - finals[1])
        e2 = np.linalg.norm(finals[1] - finals[2])
        ratios[scheme] = e1 / e2
    assert 3.6 < ratios["strang"] < 4.4, ratios
    assert 1.6 < ratios["lie"] < 2.4, ratios


def test_strang_real_time_step_is_its_own_reverse():
    """S(-dt) S(dt) = 1: the symmetric step run backwards undoes itself (each
    half phase sees the same density forwards and backwards, and the
    Crank-Nicolson solve with -dt inverts the one with dt).  The first-order
    step run backwards does not."""
    p, back = _interacting_real(0.006), _interacting_real(-0.006)
    psi0 = W.random_state(p.n, p.d, seed=18)
    psi = O.evolve(p, psi0, 10, scheme="strang")
    assert abs(O.norm(p, psi) - O.norm(p, psi0)) < 1e-13
    again = O.evolve(back, psi, 10, scheme="strang")
    assert np.max(np.abs(again - psi0)) < 1e-12 * np.max(np.abs(psi0))
    lie_back = O.evolve(back, O.evolve(p, psi0, 10), 10)
    assert np.max(np.abs(lie_back - psi0)) > 1e-6 * np.max(np.abs(psi0))


@pytest.mark.parametrize("scheme", ["lie", "strang"])
def test_ground_state_driver_reaches_the_noninteracting_fixed_point(scheme):
    """Without interactions the stationary state of either step is the product
    of the dominant eigenvectors of the one-axis transfer matrices; the driver
    stops near it, on the first check whose mu change per step is below tol,
    and its state is exactly that many plain steps from psi0."""
    n, d = (24, 20, 28), (0.45, 0.5, 0.4)
    p = _params(n, d, dt=0.02, trap=(1.0, 1.5, 2.0), imag=True)
    psi0 = W.gaussian_state(n, d, (0.7, 1.0, 1.2))
    tol, every = 1e-11, 7
    psi, steps, rate, mu = O.ground_state(p, psi0, tol, 5000, every, scheme=scheme)
    assert rate < tol and 0 < steps < 5000 and steps % every == 0
    transfer = _axis_transfer_strang if scheme == "strang" else _axis_transfer
    vecs = []
    for a in range(3):
        w, v = np.linalg.eig(transfer(p, a))
        e = v[:, np.argmax(np.abs(w))]
        vecs.append(e * np.sign(e[np.argmax(np.abs(e))].real))
    ref = np.einsum("i,j,k->ijk", *vecs)
    ref = ref / math.sqrt(O.norm(p, ref))
    assert np.max(np.abs(psi - ref)) < 2e-5 * np.max(np.abs(ref))
    assert abs(mu - O.observables(p, ref)["mu"]) < 1e-9
    # the stopping rule: mu along the plain trajectory, one check at a time
    traj = O.evolve(p, psi0, steps - every, scheme=scheme)
    before = O.observables(p, traj)["mu"]
    if steps > every:
        older = O.observables(p, O.evolve(p, psi0, steps - 2 * every, scheme=scheme))["mu"]
        assert abs(before - older) / every >= tol
    np.testing.assert_array_equal(psi, O.evolve(p, traj, every, scheme=scheme))
    assert abs(abs(mu - before) / every - rate) < 1e-15


def test_ground_state_driver_interacting_virial():
    # the dipolar ground state reached by the driver satisfies the virial
    # theorem 2 E_kin - 2 E_trap + 3 E_c + 3 E_dd = 0 and H psi = mu psi
    n, d = (24, 24, 24), (0.45, 0.45, 0.45)
    p = _params(n, d, dt=0.004, trap=(1.0, 1.0, 1.4), g=20.0, gd=8.0, imag=True)
    psi, steps, rate, mu = O.ground_state(p, W.gaussian_state(n, d, p.trap), 1e-9, 4000, 10,
                                          scheme="strang")
    assert rate < 1e-9 and steps < 4000
    o = O.observables(p, psi)
    assert o["mu"] == mu
    scale = o["e_kin"] + o["e_trap"] + o["e_contact"] + abs(o["e_dd"])
    vir = 2 * o["e_kin"] - 2 * o["e_trap"] + 3 * o["e_contact"] + 3 * o["e_dd"]
    assert abs(vir) < 0.02 * scale
    res = O.hamiltonian_apply(p, psi) - o["mu"] * psi
    assert np.linalg.norm(res) < 0.01 * o["mu"] * np.linalg.norm(psi)


# ---------------------------------------------------------------------------
# Quasi-two-dimensional programs
# ---------------------------------------------------------------------------

def _q2d(n=(32, 48), d=(0.3, 0.25), dt=0.004, trap=(1.0, 1.3), nu_t=8.0, g=20.0, gd=6.0, imag=True,
         dipoles="perp"):
    return O.Params2D(tuple(n), tuple(d), dt, tuple(trap), nu_t, g, gd, imag, dipoles)


@pytest.mark.parametrize("dipoles", ["perp", "inplane"])
def test_q2d_kernel_is_the_tight_axis_average_of_the_3d_kernel(dipoles):
    """U2(q) against direct quadrature of int dk_t/(2 pi) U(q, k_t)
    exp(-k_t^2 l^2/2) with the 3D kernel (4 pi/3)(3 cos^2 - 1) of dipoles along
    the tight axis or along the plane's axis b."""
    p = _q2d(nu_t=5.0, dipoles=dipoles)
    U2 = O.q2d_kernel(p)
    qa = 2 * np.pi * np.fft.fftfreq(p.n[0], d=p.d[0])
    qb = 2 * np.pi * np.fft.rfftfreq(p.n[1], d=p.d[1])
    ell = 1 / math.sqrt(p.nu_t)
    for ia, ib in [(1, 0), (0, 1), (3, 5), (7, 2), (16, 24), (5, 0), (0, 20)]:
        q2 = qa[ia] ** 2 + qb[ib] ** 2

        def f(kt):
            k2 = q2 + kt * kt
            c2 = kt * kt / k2 if dipoles == "perp" else qb[ib] ** 2 / k2
            return (4 * np.pi / 3) * (3 * c2 - 1) * math.exp(-kt * kt * ell * ell / 2) / (2 * np.pi)
        val = 2 * integrate.quad(f, 0, np.inf, epsabs=1e-13, epsrel=1e-12, limit=400)[0]
        assert abs(U2[ia, ib] - val) < 1e-9 * max(1.0, abs(val)), (ia, ib, U2[ia, ib], val)
    # q = 0: (4 pi/3)/(sqrt(2 pi) l) times 2 (perp) or -1 (in plane)
    pre = (4 * np.pi / 3) / (math.sqrt(2 * np.pi) * ell)
    assert abs(U2[0, 0] - pre * (2.0 if dipoles == "perp" else -1.0)) < 1e-12 * pre


@pytest.mark.parametrize("dipoles,sa,sb", [("perp", 1.1, 1.1), ("perp", 0.7, 0.7), ("inplane", None, 1.6),
                                            ("inplane", None, 0.6)])
def test_q2d_dipolar_energy_of_gaussian_equals_the_3d_closed_form(dipoles, sa, sb):
    """The quasi-2D state psi(a, b) phi(t) of a Gaussian in the plane is a 3D
    Gaussian; when it is axially symmetric about the dipole axis its dipolar
    energy has the closed form of the 3D pin (gd = 1, unit norm, no cut-off).
    perp: axis t, widths (sigma_rho, l); in plane: axis b, sigma_a = l.  The
    periodic plane adds the images' 1/r^3 tail, so the grid value approaches
    the closed form as L^-3: eightfold per doubling of the box."""
    nu_t = 4.0
    ell = 1 / math.sqrt(nu_t)
    if dipoles == "inplane":
        sa = ell
    ref = _edd_gaussian_closed(sa, ell) if dipoles == "perp" else _edd_gaussian_closed(ell, sb)
    errs = []
    for n in (320, 640, 1280):  # L = 28.8, 57.6, 115.2
        p = _q2d(n=(n, n), d=(0.09, 0.09), nu_t=nu_t, g=0.0, gd=1.0, dipoles=dipoles)
        xa, xb = O.q2d_grid(p)
        dens = np.exp(-(xa[:, None] / sa) ** 2 - (xb[None, :] / sb) ** 2)
        dens /= np.sum(dens) * p.dA
        errs.append(abs(O.q2d_observables(p, np.sqrt(dens).astype(complex))["e_dd"] - ref) / abs(ref))
    assert errs[-1] < 3e-5, errs
    for e0, e1 in zip(errs, errs[1:]):
        assert 6.5 < e0 / e1 < 9.5, errs


def test_q2d_contact_coupling_is_the_tight_axis_average():
    """E_c of psi(a, b) equals the 3D contact energy g/2 int |psi phi|^4 of the
    product state, with phi the tight trap's ground state sampled on a fine
    grid along t."""
    p = _q2d(n=(24, 30), d=(0.35, 0.3), nu_t=6.0, g=17.0, gd=0.0)
    psi = W.random_state((p.n[0], 1, p.n[1]), (p.d[0], 1.0, p.d[1]), seed=41)[:, 0, :]
    ec2 = O.q2d_observables(p, psi)["e_contact"]
    t = np.linspace(-6, 6, 4001)
    dt_ = t[1] - t[0]
    phi2 = np.exp(-t ** 2 * p.nu_t) * math.sqrt(p.nu_t / np.pi)  # |phi|^2, unit norm
    ec3 = 0.5 * p.g * float(np.sum(np.abs(psi) ** 4) * p.dA) * float(np.sum(phi2 ** 2) * dt_)
    assert abs(ec2 - ec3) < 1e-9 * ec3


@pytest.mark.parametrize("imag", [False, True])
def test_q2d_noninteracting_step_is_exactly_separable(imag):
    p = _q2d(n=(12, 14), d=(0.4, 0.35), dt=0.02, trap=(1.0, 1.7), g=0.0, gd=0.0, imag=imag)
    rng = np.random.default_rng(42)
    f = [rng.normal(size=p.n[a]) + 1j * rng.normal(size=p.n[a]) for a in range(2)]
    psi0 = np.einsum("i,j->ij", *f)
    steps = 12
    got = O.q2d_evolve(p, psi0, steps)
    p3 = _params((p.n[0], p.n[1], 4), (p.d[0], p.d[1], 1.0), dt=p.dt, trap=(p.trap[0], p.trap[1], 0.0),
                 imag=imag)
    g = [np.linalg.matrix_power(_axis_transfer(p3, a), steps) @ f[a] for a in range(2)]
    ref = np.einsum("i,j->ij", *g)
    if imag:
        ref = ref / math.sqrt(np.sum(np.abs(ref) ** 2) * p.dA)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("dipoles", ["perp", "inplane"])
def test_q2d_real_time_conserves_norm_and_reverses(dipoles):
    p = _q2d(n=(20, 24), d=(0.35, 0.3), dt=0.004, g=25.0, gd=10.0, imag=False, dipoles=dipoles)
    back = _q2d(n=(20, 24), d=(0.35, 0.3), dt=-0.004, g=25.0, gd=10.0, imag=False, dipoles=dipoles)
    psi0 = W.random_state((p.n[0], 1, p.n[1]), (p.d[0], 1.0, p.d[1]), seed=43)[:, 0, :]
    psi = O.q2d_evolve(p, psi0, 20)
    n0 = np.sum(np.abs(psi0) ** 2)
    assert abs(np.sum(np.abs(psi) ** 2) - n0) < 1e-13 * n0
    for _ in range(20):  # the inverse step: sweeps with -dt, then the phase with -dt
        for axis in (1, 0):
            c = back.dt / (4.0 * back.d[axis] ** 2)
            psi = O.cn_solve_axis(psi, 1j * c, axis)
        dens = np.abs(psi) ** 2
        th = back.dt * (O.q2d_trap(back) + back.g2 * dens + back.gd * O.q2d_potential(back, dens))
        psi = psi * np.exp(-1j * th)
    assert np.max(np.abs(psi - psi0)) < 1e-12 * np.max(np.abs(psi0))


# ---------------------------------------------------------------------------
# Adjoint
# ---------------------------------------------------------------------------

def _small_real_params():
    n, d = (8, 10, 12), (0.5, 0.45, 0.4)
    return _params(n, d, dt=0.01, trap=(1.0, 1.2, 1.7), g=15.0, gd=9.0, imag=False)


def _forward_J(p, psi0, amp, objective="energy", target=None):
    psi = O.evolve(p, psi0, len(amp) - 1, amp)
    if objective == "energy":
        return O.energy_total(p, psi, amp[-1])
    return O.overlap_objective(p, psi, target)[0]


@pytest.mark.parametrize("objective", ["energy", "overlap"])
def test_adjoint_matches_central_differences(objective):
    p = _small_real_params()
    psi0 = W.random_state(p.n, p.d, seed=21)
    target = W.random_state(p.n, p.d, seed=22) if objective == "overlap" else None
    amp = np.random.default_rng(23).uniform(0.8, 1.2, size=7)
    J, psiN, dJ_da, dJ_dtrap, lam0 = O.adjoint_evolve(p, psi0, amp, objective, target)
    assert abs(J - _forward_J(p, psi0, amp, objective, target)) < 1e-14 * abs(J)
    h = 1e-4
    fd = np.zeros(len(amp))
    for i in range(len(amp)):
        ap, am = amp.copy(), amp.copy()
        ap[i] += h
        am[i] -= h
        fd[i] = (_forward_J(p, psi0, ap, objective, target) - _forward_J(p, psi0, am, objective, target)) / (2 * h)
    scale = max(np.max(np.abs(fd)), 1e-3 * abs(J))
    assert np.max(np.abs(dJ_da - fd)) < 1e-6 * scale
    for j in range(3):
        tp, tm = list(p.trap), list(p.trap)
        tp[j] += h
        tm[j] -= h
        pp = O.Params(p.n, p.d, p.dt, tuple(tp), p.g, p.gd, p.imag, p.R)
        pm = O.Params(p.n, p.d, p.dt, tuple(tm), p.g, p.gd, p.imag, p.R)
        fdj = (_forward_J(pp, psi0, amp, objective, target) - _forward_J(pm, psi0, amp, objective, target)) / (2 * h)
        assert abs(dJ_dtrap[j] - fdj) < 1e-6 * max(abs(fdj), 1e-3 * abs(J))
    v = W.random_state(p.n, p.d, seed=24)
    fdv = (_forward_J(p, psi0 + h * v, amp, objective, target)
           - _forward_J(p, psi0 - h * v, amp, objective, target)) / (2 * h)
    adj = float(np.real(np.sum(np.conj(lam0) * v)))
    assert abs(adj - fdv) < 1e-6 * max(abs(fdv), 1e-3 * abs(J))


def test_adjoint_sweep_is_conjugate_transpose():
    # <lam, C u> = <C^H lam, u> with C^H the sweep with conj(A)
    p = _small_real_params()
    u = W.random_state(p.n, p.d, seed=31)
    lam = W.random_state(p.n, p.d, seed=32)
    lhs = np.vdot(lam, O.kinetic_step(p, u))
    rhs = np.vdot(O.kinetic_step(p, lam, conjugate=True), u)
    assert abs(lhs - rhs) < 1e-14 * abs(lhs) + 1e-16
