"""MI355X split-step Crank-Nicolson solver for the 3D dipolar Gross-Pitaevskii
equation: Python binding of libdgpe (include/dgpe.h).

PyTorch supplies device memory and the current HIP stream; every step of the
method runs in libdgpe's HIP kernels.  The binding only marshals arguments.

    plan = Plan((256, 256, 256), (0.1,) * 3, dt=1e-3, trap=(1, 1, 0.5), g=100, gd=60,
                real_time=False, dtype=torch.complex64)
    plan.step(psi, 100)                 # psi: cuda complex tensor [Nx][Ny][Nz], in place
    obs = plan.observables(psi)         # norm, mu, energy, parts, rms
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import DgpeError, check, load

__all__ = ["Plan", "DgpeError", "DgpeEvolve", "knot_matrix", "load", "workspace_bytes"]


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def workspace_bytes(n, real_time=False, f32=False, q2d=None):
    n_arr = (ctypes.c_int32 * 3)(*n)
    mode = ((_lib.DGPE_REAL if real_time else _lib.DGPE_IMAG) | (_lib.DGPE_F32 if f32 else _lib.DGPE_F64)
            | _lib.Q2D[q2d])
    return int(load().dgpe_workspace_bytes(n_arr, mode))


class Plan:
    """A libdgpe plan bound to a torch-allocated device workspace.

    n, d      grid sizes (Nx, Ny, Nz) and spacings
    dt        time step; trap (nu, lambda, gamma); g, gd interaction strengths
    cutoff    dipolar cut-off radius (<= 0: min(N_i d_i)/2)
    real_time False: imaginary time (renormalised every step); True: real time
    dtype     torch.complex128 (FP64 path) or torch.complex64 (FP32 path)
    noalloc   True: no workspace tensor; the plan uses the library's static
              device scratch (dgpe_plan_create_noalloc, at most 64 MiB; a later
              such plan on the same device supersedes this one)
    q2d       None (3D), or "perp" / "inplane" for a quasi-2D plan on an
              (N1, 1, N2) grid whose middle axis is the tight trap trap[1]
              (dipoles along the tight axis, or along z in the plane)
    """

    def __init__(self, n, d, dt, trap, g, gd, cutoff=0.0, real_time=False, dtype=None,
                 device="cuda", stream=None, noalloc=False, q2d=None):
        torch = _torch()
        dtype = torch.complex128 if dtype is None else dtype
        if dtype not in (torch.complex128, torch.complex64):
            raise ValueError("dtype must be torch.complex128 or torch.complex64")
        self.lib = load()
        self.n = tuple(int(v) for v in n)
        self.d = tuple(float(v) for v in d)
        self.dt = float(dt)
        self.trap = [float(v) for v in trap]
        self.g, self.gd = float(g), float(gd)
        self.real_time = bool(real_time)
        self.dtype = dtype
        self.rdtype = torch.float64 if dtype == torch.complex128 else torch.float32
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        f32 = dtype == torch.complex64
        self.q2d = q2d
        self.mode = ((_lib.DGPE_REAL if real_time else _lib.DGPE_IMAG) | (_lib.DGPE_F32 if f32 else _lib.DGPE_F64)
                     | _lib.Q2D[q2d])
        n_arr = (ctypes.c_int32 * 3)(*self.n)
        nbytes = int(self.lib.dgpe_workspace_bytes(n_arr, self.mode))
        if nbytes == 0:
            raise DgpeError(2, f"unsupported grid {self.n}")
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        handle = ctypes.c_void_p()
        d_arr = (ctypes.c_double * 3)(*self.d)
        t_arr = (ctypes.c_double * 3)(*self.trap)
        self.noalloc = bool(noalloc)
        if self.noalloc:
            self.workspace = None
            with torch.cuda.device(self.device):
                check(self.lib.dgpe_plan_create_noalloc(
                    ctypes.byref(handle), n_arr, d_arr, self.dt, t_arr, self.g, self.gd,
                    float(cutoff), self.mode, ctypes.c_void_p(stream.cuda_stream)))
        else:
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            check(self.lib.dgpe_plan_create(ctypes.byref(handle), n_arr, d_arr, self.dt, t_arr,
                                            self.g, self.gd, float(cutoff), self.mode,
                                            _ptr(self.workspace), nbytes,
                                            ctypes.c_void_p(stream.cuda_stream)))
        self.handle = handle

    # -- helpers ------------------------------------------------------------
    def _check_state(self, psi, name="psi"):
        torch = _torch()
        if not isinstance(psi, torch.Tensor) or psi.dtype != self.dtype or psi.device != self.device:
            raise TypeError(f"{name} must be a {self.dtype} tensor on {self.device}")
        if tuple(psi.shape) != self.n or not psi.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {self.n}")

    def new_state(self, array=None):
        """A device state of this plan's dtype, optionally copied from numpy."""
        torch = _torch()
        if array is None:
            return torch.zeros(self.n, dtype=self.dtype, device=self.device)
        return torch.from_numpy(np.ascontiguousarray(array)).to(self.dtype).to(self.device).contiguous()

    @property
    def fused_y(self):
        """True when step() runs the fused y schedule (the z pass starts the y
        solve in 16-line segments, a carry pass joins them)."""
        return self.lib.dgpe_plan_fused_y(self.handle) == 1

    def set(self, name, value):
        """Change one parameter: g, gd, nu, lambda, gamma, dt, real_time,
        fast_fft (0/1), fused_y (0/1) or scheme ("lie"/"strang" or 0/1)."""
        if name == "scheme" and isinstance(value, str):
            value = _lib.SCHEME[value]
        check(self.lib.dgpe_plan_set(self.handle, _lib.PARAM[name], float(value)))
        if name == "g":
            self.g = float(value)
        elif name == "gd":
            self.gd = float(value)
        elif name in ("nu", "lambda", "gamma"):
            self.trap[("nu", "lambda", "gamma").index(name)] = float(value)
        elif name == "dt":
            self.dt = float(value)
        elif name == "real_time":
            self.real_time = bool(value)

    # -- the method -----------------------------------------------------------
    def step(self, psi, nsteps=1, amp=None):
        """Advance psi in place by nsteps split steps (asynchronous).  amp: per-step
        trap amplitudes (length nsteps) or None."""
        self._check_state(psi)
        amp_p = None
        if amp is not None:
            a = np.ascontiguousarray(np.asarray(amp, dtype=np.float64))
            if a.shape != (nsteps,):
                raise ValueError("amp must have nsteps entries")
            amp_p = a.ctypes.data_as(_lib.P_double)
        check(self.lib.dgpe_step(self.handle, _ptr(psi), int(nsteps), amp_p))
        return psi

    def ground_state(self, psi, tol=1e-10, max_steps=20000, check_every=10):
        """Imaginary-time steps on psi (in place) until mu changes by less than
        tol per step between checks every check_every steps, or max_steps.
        Returns dict(steps, dmu_per_step, converged, observables)."""
        self._check_state(psi)
        steps = ctypes.c_int32()
        rate = ctypes.c_double()
        o = _lib.DgpeObs()
        check(self.lib.dgpe_ground_state(self.handle, _ptr(psi), float(tol), int(max_steps),
                                         int(check_every), ctypes.byref(steps), ctypes.byref(rate),
                                         ctypes.byref(o)))
        return {"steps": steps.value, "dmu_per_step": rate.value, "converged": rate.value < tol,
                "observables": _obs_dict(o)}

    def potential(self, psi, out=None):
        """Dipolar potential Phi of |psi|^2 on the grid (real, plan precision)."""
        torch = _torch()
        self._check_state(psi)
        if out is None:
            out = torch.empty(self.n, dtype=self.rdtype, device=self.device)
        check(self.lib.dgpe_potential(self.handle, _ptr(psi), _ptr(out)))
        return out

    def density(self, psi, out=None):
        """|psi|^2 on the grid (real, plan precision)."""
        torch = _torch()
        self._check_state(psi)
        if out is None:
            out = torch.empty(self.n, dtype=self.rdtype, device=self.device)
        check(self.lib.dgpe_density(self.handle, _ptr(psi), _ptr(out)))
        return out

    def write_density(self, psi, path):
        """Write |psi|^2 as a binary file of Nx*Ny*Nz float64 values, row-major
        [x][y][z] (read back with numpy.fromfile(path).reshape(n))."""
        self._check_state(psi)
        check(self.lib.dgpe_write_density(self.handle, _ptr(psi), str(path).encode()))

    def observables(self, psi, amp=1.0):
        """Norm, chemical potential, energy and parts, rms sizes (synchronises)."""
        self._check_state(psi)
        o = _lib.DgpeObs()
        check(self.lib.dgpe_energy_mu_rms(self.handle, _ptr(psi), float(amp), ctypes.byref(o)))
        return _obs_dict(o)

    def adjoint(self, psi0, amp, ckpt_every=20, objective="energy", target=None,
                want_psi_final=True, want_dpsi0=True):
        """Gradient of a final-state objective through len(amp)-1 real-time steps.

        Returns dict(J, dJ_damp [nsteps+1], dJ_dtrap [3], psi_final, dJ_dpsi0)."""
        torch = _torch()
        self._check_state(psi0, "psi0")
        a = np.ascontiguousarray(np.asarray(amp, dtype=np.float64))
        nsteps = a.shape[0] - 1
        if objective == "overlap":
            self._check_state(target, "target")
        nbytes = int(self.lib.dgpe_adjoint_workspace_bytes(self.handle, nsteps, int(ckpt_every)))
        if nbytes == 0:
            raise DgpeError(1, "invalid adjoint sizes")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        psi_f = torch.empty_like(psi0) if want_psi_final else None
        lam0 = torch.empty_like(psi0) if want_dpsi0 else None
        J = ctypes.c_double()
        dJ_da = np.zeros(nsteps + 1)
        dJ_dt = np.zeros(3)
        check(self.lib.dgpe_step_adjoint(
            self.handle, _ptr(psi0), nsteps, a.ctypes.data_as(_lib.P_double), int(ckpt_every),
            _lib.OBJECTIVE[objective], _ptr(target) if target is not None else None, _ptr(ws),
            nbytes, _ptr(psi_f) if psi_f is not None else None, ctypes.byref(J),
            dJ_da.ctypes.data_as(_lib.P_double), dJ_dt.ctypes.data_as(_lib.P_double),
            _ptr(lam0) if lam0 is not None else None))
        return {"J": J.value, "dJ_damp": dJ_da, "dJ_dtrap": dJ_dt, "psi_final": psi_f,
                "dJ_dpsi0": lam0}

    def pass_bytes(self):
        """Algorithmic HBM bytes per launch of each pass (dict by pass name)."""
        b = np.zeros(_lib.NPASS)
        check(self.lib.dgpe_pass_bytes(self.handle, b.ctypes.data_as(_lib.P_double)))
        return dict(zip(_lib.PASS_NAMES, b.tolist()))

    def step_profiled(self, psi, nsteps=1, amp=None):
        """dgpe_step with HIP events around every pass; returns (mean ms per launch
        by pass name, total ms).  Synchronises."""
        self._check_state(psi)
        amp_p = None
        if amp is not None:
            a = np.ascontiguousarray(np.asarray(amp, dtype=np.float64))
            if a.shape != (nsteps,):
                raise ValueError("amp must have nsteps entries")
            amp_p = a.ctypes.data_as(_lib.P_double)
        ms = np.zeros(_lib.NPASS)
        tot = ctypes.c_double()
        check(self.lib.dgpe_step_profiled(self.handle, _ptr(psi), int(nsteps), amp_p,
                                          ms.ctypes.data_as(_lib.P_double), ctypes.byref(tot)))
        return dict(zip(_lib.PASS_NAMES, ms.tolist())), tot.value

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.dgpe_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _obs_dict(o):
    return {"norm": o.norm, "mu": o.mu, "energy": o.energy, "e_kin": o.e_kin,
            "e_trap": o.e_trap, "e_contact": o.e_contact, "e_dd": o.e_dd,
            "rms": tuple(o.rms[i] for i in range(4))}


def knot_matrix(nknots, nsteps, dt):
    """W [(nsteps+1) x nknots]: a(t_n) = sum_k W[n, k] a_k for a piecewise-linear
    a(t) on knots t_k = k T/(nknots - 1), T = nsteps dt, sampled at t_n = n dt."""
    T = nsteps * dt
    W = np.zeros((nsteps + 1, nknots))
    h = T / (nknots - 1)
    for n in range(nsteps + 1):
        t = n * dt
        k = min(int(np.floor(t / h)), nknots - 2)
        w = (t - k * h) / h
        W[n, k] += 1.0 - w
        W[n, k + 1] += w
    return W


class DgpeEvolve:
    """torch.autograd.Function: J = objective(psi_N) after real-time evolution with
    a trap amplitude a(t) interpolated from knots and trap (lambda, gamma).

        J = DgpeEvolve.apply(knots, lam_gam, psi0, plan, nsteps, ckpt_every, objective, target)

    knots, lam_gam: float64 CPU tensors.  The forward pass runs libdgpe's
    checkpointed adjoint once and keeps the gradients; backward returns
    (W^T dJ/da, dJ/d(lambda, gamma), dJ/dpsi0) scaled by the incoming gradient."""

    _fn = None

    @classmethod
    def _function(cls):
        if cls._fn is None:
            torch = _torch()

            class _Evolve(torch.autograd.Function):
                @staticmethod
                def forward(ctx, knots, lam_gam, psi0, plan, nsteps, ckpt_every=20,
                            objective="energy", target=None):
                    if not plan.real_time:
                        raise DgpeError(6, "DgpeEvolve needs a real-time plan")
                    W = knot_matrix(knots.numel(), nsteps, plan.dt)
                    amp = W @ knots.detach().cpu().numpy().astype(np.float64)
                    # the trap (lambda, gamma) of this evaluation; the plan's own
                    # values are restored afterwards, also when the call fails
                    saved = (plan.trap[1], plan.trap[2])
                    try:
                        plan.set("lambda", float(lam_gam[0]))
                        plan.set("gamma", float(lam_gam[1]))
                        out = plan.adjoint(psi0.detach(), amp, ckpt_every, objective, target)
                    finally:
                        plan.set("lambda", saved[0])
                        plan.set("gamma", saved[1])
                    ctx.gk = torch.from_numpy(W.T @ out["dJ_damp"])
                    ctx.gt = torch.from_numpy(out["dJ_dtrap"][1:3].copy())
                    ctx.gpsi = out["dJ_dpsi0"]
                    return torch.tensor(out["J"], dtype=torch.float64)

                @staticmethod
                def backward(ctx, gJ):
                    g = float(gJ)
                    return (g * ctx.gk, g * ctx.gt, g * ctx.gpsi, None, None, None, None, None)

            cls._fn = _Evolve
        return cls._fn

    @classmethod
    def apply(cls, *args):
        return cls._function().apply(*args)
