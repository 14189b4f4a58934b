/*
 * dgpe.h -- C ABI of libdgpe, the MI355X (gfx950) split-step Crank-Nicolson
 * time step of the three-dimensional dipolar Gross-Pitaevskii equation (GPE).
 *
 * Method (paper, program summary, "Nature of problem" and "Solution method";
 * "Summary of revisions" for the real-to-complex transform of the density):
 * the GPE with contact and dipolar interaction in an anisotropic harmonic trap,
 * discretised in space and time and propagated over small steps in imaginary
 * time (ground state) or real time (dynamics); the dipolar term is evaluated in
 * momentum space through the convolution theorem.  In trap units:
 *
 *   real time       i dpsi/dt  =  [-1/2 Lap + V + g|psi|^2 + gd Phi] psi
 *   imaginary time    dpsi/dtau = -[...] psi
 *   V   = a(t)/2 (nu^2 x^2 + lam^2 y^2 + gam^2 z^2)
 *   Phi = IDFT[ U_R(k) DFT[|psi|^2] ],  dipoles along z,
 *   U_R = (4 pi/3)(3 kz^2/k^2 - 1)(1 + 3 cos(kR)/(kR)^2 - 3 sin(kR)/(kR)^3), U_R(0) = 0.
 *
 * One step: theta = dt (V + g n + gd Phi[n]) from the pre-step density n;
 * psi <- psi exp(-i theta) (real) or psi exp(-theta) (imaginary); then the
 * Crank-Nicolson solve (1 - A D) psi' = (1 + A D) psi along x, y and z with
 * D = [1, -2, 1], zero ghost values, A = i dt/(4 d^2) (real) or dt/(4 d^2)
 * (imaginary); in imaginary time psi is then rescaled to sum |psi|^2 dV = 1.
 * Grid: x_i = (i - Nx/2) dx (likewise y, z).
 *
 * Layout: every grid array is C-ordered [Nx][Ny][Nz] with z contiguous and x
 * slowest (paper, DBEC-GP-MPI package, data distribution along NX).  Complex
 * values are interleaved (re, im): complex128 for DGPE_F64 plans, complex64
 * for DGPE_F32 plans.  Real arrays (Phi) have the plan's real type.
 *
 * Ownership: the caller allocates every device buffer (state, workspace,
 * adjoint workspace) and keeps it alive while the plan or call uses it; the
 * library allocates no device memory.  The plan owns only host metadata.
 * Device pointers must be 256-byte aligned.
 *
 * Streams: all work is enqueued on the plan's HIP stream.  dgpe_step and
 * dgpe_potential are asynchronous and report only argument and launch errors;
 * dgpe_energy_mu_rms and dgpe_step_adjoint synchronise the stream and report
 * deferred errors.  A plan is not re-entrant; distinct plans are independent.
 *
 * Errors: every call returns a dgpe_status; dgpe_last_error() gives a
 * thread-local message for the last failure.  Grid sizes must be even, have no
 * prime factor other than 2 and 3 (the paper's FFT-friendly sizes restricted to
 * the radices implemented here) and lie in [4, 2048], with at most 2^30 points
 * in all (the kernels index points with 32-bit integers); invalid arguments are
 * rejected before any work is enqueued (the library's counterpart of the
 * paper's input checks, "Additional comments").
 */
#ifndef DGPE_H
#define DGPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dgpe_plan_s* dgpe_plan;

typedef enum {
    DGPE_OK = 0,
    DGPE_EINVAL = 1,             /* an argument is out of range or inconsistent   */
    DGPE_EUNSUPPORTED_SIZE = 2,  /* a grid size has a factor other than 2 and 3  */
    DGPE_EWORKSPACE = 3,         /* workspace missing, misaligned or too small   */
    DGPE_EHIP = 4,               /* the HIP runtime reported an error            */
    DGPE_ENONFINITE = 5,         /* a reduction met NaN or Inf                   */
    DGPE_ESTATE = 6              /* the call does not fit the plan's mode        */
} dgpe_status;

/* mode = time | precision [| quasi-2D] */
#define DGPE_IMAG 0u
#define DGPE_REAL 1u
#define DGPE_F64 0u
#define DGPE_F32 2u
/* Quasi-two-dimensional plans (the paper's 2d programs: the GPE in two spatial
 * dimensions, "Nature of problem"): the grid is (N1, 1, N2) and its middle axis
 * is a tight harmonic trap of frequency trap[1] whose ground state
 * phi(t) = exp(-t^2/(2 l^2))/(pi l^2)^(1/4), l = 1/sqrt(trap[1]), is integrated
 * out.  The plane's equation has the contact coupling g/(sqrt(2 pi) l) and the
 * dipolar kernel of the 3D one averaged over phi^2 along the tight axis (no
 * cut-off; u = q l/sqrt 2, F(u) = sqrt(pi) u exp(u^2) erfc(u)):
 *   DGPE_Q2D_PERP     dipoles along the tight axis (the XY programs):
 *                     U(q) = (4 pi/3)/(sqrt(2 pi) l) (2 - 3 F(u))
 *   DGPE_Q2D_INPLANE  dipoles along the plane's second axis (z; the XZ
 *                     programs): U(q) = (4 pi/3)/(sqrt(2 pi) l)(-1 + 3 qz^2/q^2 F(u))
 * g and gd are the 3D couplings; d[1] is ignored (dV = d[0] d[2]); the trap is
 * a/2 (nu^2 x^2 + gamma^2 z^2) in the plane, and reported energies leave out
 * the tight axis' constant trap[1]/2 (no kinetic term along it; rms[1] = 0,
 * rms[3] the in-plane radius).  No y transforms and no y sweep run; the
 * adjoint is not available.  Changing TRAP_LAMBDA rebuilds the kernel table
 * (synchronous). */
#define DGPE_Q2D_PERP 4u
#define DGPE_Q2D_INPLANE 8u

/* dgpe_plan_set parameters */
#define DGPE_PARAM_G 0
#define DGPE_PARAM_GD 1
#define DGPE_PARAM_TRAP_NU 2
#define DGPE_PARAM_TRAP_LAMBDA 3
#define DGPE_PARAM_TRAP_GAMMA 4
#define DGPE_PARAM_DT 5
#define DGPE_PARAM_REAL_TIME 6 /* value 1: real time, 0: imaginary time */
#define DGPE_PARAM_FAST_FFT 7  /* 1 (default): compiled two-factor FFT passes where available; 0: generic passes only */
#define DGPE_PARAM_FUSED_Y 8   /* 1 (default): in imaginary time, the fused z pass also solves the y axis
                                  in 16-line segments and pass 5 joins them (see the pass list); 0: the
                                  separate y sweep.  Same result to rounding either way */
#define DGPE_PARAM_SCHEME 9    /* 0 (default): the first-order (Lie) step of the paper's method;
                                  1: the symmetric (Strang) step, see dgpe_step (3D plans only:
                                  DGPE_ESTATE for quasi-2D ones) */

/* adjoint objectives */
#define DGPE_OBJ_ENERGY 0
#define DGPE_OBJ_OVERLAP 1

/* Observables: the diagnostics this library evaluates after a run of steps
 * (its own choice of reported quantities; the paper prints no formulas for
 * them).  Sums are FP64 over the grid times dV:
 *   e_kin  = 1/2 sum_axes sum_{i=-1}^{N-1} |psi_{i+1} - psi_i|^2 / d^2 (ghost zeros)
 *   e_trap = sum a V0 |psi|^2,  e_contact = g/2 sum |psi|^4,  e_dd = gd/2 sum Phi |psi|^2
 *   energy = (e_kin + e_trap + e_contact + e_dd)/norm
 *   mu     = (e_kin + e_trap + 2 e_contact + 2 e_dd)/norm
 *   rms    = sqrt(<x^2>), sqrt(<y^2>), sqrt(<z^2>), sqrt(<r^2>) about the origin. */
typedef struct {
    double norm, mu, energy, e_kin, e_trap, e_contact, e_dd;
    double rms[4];
} dgpe_obs;

/* Bytes of device workspace a plan of grid n[3] and mode needs (0 if the
 * arguments are invalid). */
size_t dgpe_workspace_bytes(const int32_t n[3], uint32_t mode);

/* Create a plan.
 *   n[3]        Nx, Ny, Nz (each even, 2^a 3^b, 4..2048, at most 2^30 points;
 *               Ny = 1 for quasi-2D)
 *   d[3]        grid spacings > 0
 *   dt          time step > 0
 *   trap[3]     nu, lambda, gamma (trap frequencies along x, y, z), finite
 *   g, gd       contact and dipolar strengths, finite
 *   cutoff_R    kernel cut-off radius; <= 0 selects min(N_i d_i)/2 (3D only)
 *   mode        DGPE_IMAG | DGPE_REAL, combined with DGPE_F64 | DGPE_F32 and
 *               optionally DGPE_Q2D_PERP or DGPE_Q2D_INPLANE
 *   workspace   device buffer of workspace_bytes >= dgpe_workspace_bytes()
 *   hip_stream  hipStream_t for all work (NULL: the default stream)
 * Fills the workspace's constant tables (dipolar kernel, twiddles, Thomas
 * factors) and synchronises the stream once.  On failure *out is NULL. */
dgpe_status dgpe_plan_create(dgpe_plan* out, const int32_t n[3], const double d[3], double dt,
                             const double trap[3], double g, double gd, double cutoff_R,
                             uint32_t mode, void* workspace, size_t workspace_bytes,
                             void* hip_stream);

/* Largest workspace an allocation-free plan can use (64 MiB: grids up to
 * 128^3 in FP64 and 192^3 in FP32). */
#define DGPE_NOALLOC_MAX_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * plan as dgpe_plan_create, with the library's own device scratch array as
 * the workspace instead of a caller buffer.  The array is a static device
 * array of DGPE_NOALLOC_MAX_BYTES, one per device, held until the process
 * ends; this call allocates no device memory (only the plan's host metadata).
 * Arguments as for dgpe_plan_create; the plan lives on the current device.
 *   DGPE_EWORKSPACE if dgpe_workspace_bytes(n, mode) > DGPE_NOALLOC_MAX_BYTES.
 * Every allocation-free plan on a device shares that device's one array and
 * fills it with its tables: creating another one overwrites them, so every
 * earlier allocation-free plan on the device is superseded and its calls then
 * return DGPE_ESTATE (destroy it as usual).  No part of the array needs to
 * start at zero (each call writes what it reads).  Calls on allocation-free
 * plans of one device that overlap in time (other streams or threads) race
 * on the array.  The adjoint's own workspace is still the caller's. */
dgpe_status dgpe_plan_create_noalloc(dgpe_plan* out, const int32_t n[3], const double d[3],
                                     double dt, const double trap[3], double g, double gd,
                                     double cutoff_R, uint32_t mode, void* hip_stream);

/* Change one parameter (DGPE_PARAM_*).  DT and REAL_TIME rebuild the Thomas
 * tables (synchronous); the others take effect at the next launch. */
dgpe_status dgpe_plan_set(dgpe_plan plan, int32_t param, double value);

/* Redirect subsequent work to another HIP stream. */
dgpe_status dgpe_plan_set_stream(dgpe_plan plan, void* hip_stream);

/* 1 if dgpe_step on this plan, as it is now set, runs the fused y schedule
 * (DGPE_PARAM_FUSED_Y and the conditions in the pass list below), 0 if it
 * runs the separate y sweep, -1 for a NULL plan.  Host only. */
int32_t dgpe_plan_fused_y(dgpe_plan plan);

/* Advance psi (device, [Nx][Ny][Nz] complex of the plan precision, in place) by
 * nsteps split steps.  amp: host array of nsteps trap amplitudes a(t_n) (NULL:
 * all 1); it is read during the call only.  In imaginary time the returned
 * state has unit norm.  Asynchronous.
 * With DGPE_PARAM_SCHEME = 1 each step is the symmetric (Strang) step: the
 * nonlinear step over dt/2 from the incoming density, the three sweeps over
 * dt, the nonlinear step over dt/2 from the density after the sweeps, then the
 * renormalisation (imaginary time); both halves use a(t_n).  Second order in
 * dt, against first order for the default step; the paper's programs use the
 * default step.  The fused y schedule is not used with it. */
dgpe_status dgpe_step(dgpe_plan plan, void* psi, int32_t nsteps, const double* amp);

/* Imaginary-time propagation to the stationary state (paper, "Solution
 * method": propagation in imaginary time yields the ground state), stopped on
 * the change of the chemical potential.  mu (as in dgpe_energy_mu_rms, trap
 * amplitude 1) is evaluated on the incoming psi and after every check_every
 * steps; the run stops at the first evaluation where
 * |mu_now - mu_before| / (steps between them) < tol, or after max_steps steps.
 *   psi           device state (in place); returned with unit norm
 *   steps_done    steps taken; dmu_per_step: the last |delta mu| per step
 *                 (+inf if no step ran); converged iff *dmu_per_step < tol
 *   obs           observables of the returned state
 * Imaginary-time plans only (DGPE_ESTATE otherwise).  Uses the plan's scheme.
 * Synchronises the stream at every check. */
dgpe_status dgpe_ground_state(dgpe_plan plan, void* psi, double tol, int32_t max_steps,
                              int32_t check_every, int32_t* steps_done, double* dmu_per_step,
                              dgpe_obs* obs);

/* Dipolar potential Phi = IDFT[U_R DFT[|psi|^2]] of a state (paper, "Solution
 * method": the dipolar term through the convolution theorem).  phi: device
 * [Nx][Ny][Nz] real of the plan precision.  Asynchronous. */
dgpe_status dgpe_potential(dgpe_plan plan, const void* psi, void* phi);

/* Density |psi|^2 of a state (FP64 products rounded once): out is device
 * [Nx][Ny][Nz] real of the plan precision.  Asynchronous. */
dgpe_status dgpe_density(dgpe_plan plan, const void* psi, void* out);

/* Write the density of psi to the file at path in binary form (paper,
 * "Summary of revisions", MPI output format: binary density output into one
 * file, each part at its offset): Nx*Ny*Nz IEEE float64 values in the host's
 * byte order (little-endian here), row-major [x][y][z] with x slowest, no
 * header; the part of x-planes [x0, x1) starts at byte 8*x0*Ny*Nz.  The
 * density passes through the plan's workspace (its Phi buffer) and a bounded
 * host buffer.  Synchronises the stream.  DGPE_EINVAL if the file cannot be
 * written. */
dgpe_status dgpe_write_density(dgpe_plan plan, const void* psi, const char* path);

/* Norm, chemical potential, energy and its parts, rms sizes of psi with trap
 * amplitude amp.  Synchronises the stream; DGPE_ENONFINITE if any sum is not
 * finite. */
dgpe_status dgpe_energy_mu_rms(dgpe_plan plan, const void* psi, double amp, dgpe_obs* out);

/* Bytes of adjoint workspace for dgpe_step_adjoint(nsteps, ckpt_every). */
size_t dgpe_adjoint_workspace_bytes(dgpe_plan plan, int32_t nsteps, int32_t ckpt_every);

/* Reverse-mode gradient of a final-state objective through nsteps real-time
 * steps from psi0 (the hand-written adjoint of the split step; its equations
 * are the transpose of the forward step's linearisation):
 *   amp       host, nsteps+1 amplitudes: a(t_n) for step n, amp[nsteps] = a(T)
 *   objective DGPE_OBJ_ENERGY: J = e_kin + e_trap + e_contact + e_dd of psi_N
 *             (not divided by the norm, which real time conserves), trap
 *             amplitude amp[nsteps];
 *             DGPE_OBJ_OVERLAP: J = |sum conj(target) psi_N dV|^2 (target:
 *             device state of the plan precision).
 *   adj_ws    device buffer of >= dgpe_adjoint_workspace_bytes(); holds the
 *             checkpoints (every ckpt_every steps), one segment of recomputed
 *             states and the dipolar potential of each of them.  ckpt_every = 1
 *             keeps every state psi_1..psi_N and the potential of every state
 *             psi_0..psi_{N-1} from the forward sweep, so that nothing is
 *             recomputed (nsteps states and nsteps real arrays: at 256^3 FP32
 *             192 MiB per step, for a memory of 288 GB).  The result does not
 *             depend on ckpt_every (bitwise).
 * Outputs (host unless stated): J; dJ_damp[nsteps+1]; dJ_dtrap[3] for
 * (nu, lambda, gamma); psi_final (device, nullable) = psi_N; dJ_dpsi0 (device,
 * nullable) = the cotangent lam_0 with dJ = Re sum conj(lam_0) dpsi0.
 * Real-time plans only (DGPE_ESTATE otherwise).  Synchronises the stream. */
dgpe_status dgpe_step_adjoint(dgpe_plan plan, const void* psi0, int32_t nsteps, const double* amp,
                              int32_t ckpt_every, int32_t objective, const void* target,
                              void* adj_ws, size_t adj_ws_bytes, void* psi_final, double* J,
                              double* dJ_damp, double dJ_dtrap[3], void* dJ_dpsi0);

/* Pass kinds of one step, in launch order (indices of the arrays below):
 *   0 density + R2C along z      1 FFT along y
 *   2 FFT along x, U_R multiply, inverse FFT along x
 *   3 inverse FFT along y        4 C2R along z + nonlinear phase + CN along z
 *   5 CN along y                 6 CN along x (+ norm partials, imaginary time)
 *   7 norm reduction (imaginary time)
 * With DGPE_PARAM_FUSED_Y in effect (imaginary time, compiled fused pass,
 * Ny a multiple of 16 up to 256, state under 4 GiB): pass 4 also solves y in 16-line
 * segments with zero carries, pass 5 is the segment carry pass, and pass 6
 * adds the carries before the x solve; the norm of one step is then reduced
 * inside pass 1 of the next (pass 7 runs once, after the last step). */
#define DGPE_NPASS 8

/* Algorithmic HBM bytes of one launch of each pass for this plan: every array
 * a pass must read or write, counted once (state 2s bytes per point, half
 * spectrum 2s per complex value, kernel table s per entry, s = real size).
 * Host only; no device work. */
dgpe_status dgpe_pass_bytes(dgpe_plan plan, double bytes[DGPE_NPASS]);

/* Same work as dgpe_step, with a HIP event pair around every pass on the
 * plan's stream; synchronises and writes the mean milliseconds per launch of
 * each pass kind into ms[DGPE_NPASS] (0 for passes that did not run) and the
 * wall time of the whole call into *total_ms (nullable).  For measurement. */
dgpe_status dgpe_step_profiled(dgpe_plan plan, void* psi, int32_t nsteps, const double* amp,
                               double ms[DGPE_NPASS], double* total_ms);

/* Release the plan's host metadata (the workspace stays with the caller). */
void dgpe_plan_destroy(dgpe_plan plan);

const char* dgpe_status_string(dgpe_status status);
const char* dgpe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DGPE_H */
