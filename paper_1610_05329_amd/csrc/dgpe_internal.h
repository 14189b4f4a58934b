// Internal declarations shared by the libdgpe host code and kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dgpe {

constexpr int kMaxStages = 12;

// Factorisation of one FFT length into radices 8/4/2 (first) and 3 (last).
struct FftDesc {
    int L;
    int nstages;
    int radix[kMaxStages];
};

// n / d as umulhi(n, m) with m = ceil(2^32 / d); exact for n * d < 2^32.
struct FastDiv {
    uint32_t d;
    uint32_t m;
};

// Per-axis Crank-Nicolson tables (complex, plan precision), each of length N,
// stored back to back, for (1 - A D) x = (1 + A D) u with zero ghosts:
//   alpha_i = A m_i with Thomas pivots m_0 = 1/(1 + 2A), m_i = 1/(1 + 2A - A^2 m_{i-1})
//   P_i = prod_{j = seg start}^{i} alpha_j,  Q_i = prod_{j = i}^{seg end - 1} alpha_j
//   PEND[k] = P at the last point of segment k, QBEG[k] = Q at its first point,
//   E_i = P_i + alpha_i E_{i+1} (E = 0 past the segment end): the response of
//   the back substitution to a unit forward carry entering the segment.
//   G_i = prod_{j = seg start}^{i - 1} alpha_j (1 at the start): the weight of
//   d_i in the segment's first x of a back substitution from a zero right
//   carry, x_first = sum_i G_i d_i; H[k] = sum over segment k of G_i P_i.
enum {
    TAB_ALPHA = 0, TAB_P = 1, TAB_Q = 2, TAB_PEND = 3, TAB_QBEG = 4, TAB_E = 5, TAB_G = 6,
    TAB_H = 7, TAB_COUNT = 8
};

// Launch parameters of the seven passes for one plan (host side).
struct Launch {
    int threads;  // block size of FFT passes
    int logB_z;   // lines per block in the z passes (r2c / c2r)
    int logB_y;   // rows per block in the y pass
    int logB_x;   // columns per block in the x pass
    int seg[3];   // Thomas segment length per axis
    int logZB[3]; // columns per block of the strided sweeps (x, y)
    int gtab[3];  // strided sweeps: Thomas tables read from global memory, not
                  // staged in LDS (lines whose tables would crowd out the columns)
};

struct Plan {
    int n[3];
    double d[3];
    double dt;
    double dt_nl;  // time step of the nonlinear phase in the fused z pass (dt, or dt/2
                   // in the first step of the symmetric scheme)
    int scheme;    // 0: first-order (Lie) step; 1: symmetric (Strang) step
    int q2d;       // 0: 3D; quasi-2D on an (N1, 1, N2) grid with dipoles along the
                   // tight axis (1) or along the plane's second axis (2)
    double g_in;   // the caller's contact coupling (g holds the one the kernels use)
    double trap[3];
    double g, gd, R;
    bool imag, f32;
    hipStream_t stream;
    int device;
    // workspace carve-up (device pointers)
    char* ws;
    size_t ws_bytes;
    void* spec;         // [Nz/2+1][Nx][Ny] complex
    void* phi;          // [Nx][Ny][Nz] real (observables / adjoint scratch)
    void* ukern;        // [Nz/2+1][Nx/2+1][Ny/2+1] real, U_R / Nt (even in kx and ky)
    void* tw[3];        // twiddles W_L^m for the x, y FFTs (L = Nx, Ny) and the z FFT (L = Nz/2)
    void* twr2c;        // W_Nz^k, k = 0..Nz/2
    void* cntab[3][2];  // per axis: [0] forward A, [1] conj(A) (adjoint)
    double* red;        // reduction partials
    double* scal;       // device scalars: [0] sigma (pending 1/norm), [1..] spare
    size_t red_count;
    FftDesc fx, fy, fz;
    Launch lc;
    bool fast;  // use the two-factor register FFT passes where compiled
    bool fuse_y;  // let the fused z pass start the y solve where it can
    bool static_ws;   // the workspace is the library's allocation-free scratch array
    uint64_t ws_gen;  // that array's generation when this plan was created
};

size_t workspace_layout(const int n[3], bool f32, size_t* offs /* [16] or null */);

// ---- kernel launchers (templated on precision in the .hip files) ----------
// Each returns hipSuccess or the launch error.
template <typename T>
hipError_t launch_r2c_density(const Plan& p, const void* psi, const double* sigma);
template <typename T>
hipError_t launch_r2c_adjoint_s(const Plan& p, const void* mu, const void* psin, const void* phin,
                                double amp, double* partials, int* nblocks);
// npart (forward, compiled pass only): block 0 also reduces nnpart FP64 norm
// partials into *sigma_out = 1 / (sum dV)
template <typename T>
hipError_t launch_rows(const Plan& p, bool inverse, const double* npart = nullptr, int nnpart = 0,
                       double* sigma_out = nullptr);
template <typename T>
hipError_t launch_xmul(const Plan& p);
template <typename T>
// P5 from psi_in to psi_out (may be the same buffer); phi_out (optional)
// receives Phi of psi_in's density; ycar (optional, imaginary time, the
// compiled pass only): also solve the y axis in 16-line segments with zero
// carries, writing the three carry inputs [3][Nx][Ny/16][Nz] there;
// phi_sigma (compiled pass only): the spectrum holds the unscaled density and
// Phi is multiplied by sigma here
hipError_t launch_c2r_step(const Plan& p, const void* psi_in, void* psi_out, const double* sigma,
                           double amp, void* phi_out = nullptr, void* ycar = nullptr,
                           bool phi_sigma = false);
template <typename T>
hipError_t launch_c2r_phi(const Plan& p, void* phi_out);
template <typename T>
hipError_t launch_cn_z(const Plan& p, void* f, bool conjugate);
template <typename T>
// ycar (x axis, imaginary time): add the y segment carries c_d, c_x (the
// pairs launch_cn_ycarry writes after the three input arrays) to the values
// as they are loaded
hipError_t launch_cn_strided(const Plan& p, void* f, int axis, bool conjugate, double* norm_partials,
                             const void* ycar = nullptr);
// (c_d, c_x) pairs of the y segments, tiled for the x sweep, at car + 3
// arrays, from the three carry inputs written by the fused z pass
template <typename T>
hipError_t launch_cn_ycarry(const Plan& p, void* car);
template <typename T>
hipError_t launch_scale(const Plan& p, void* psi, const double* sigma);
template <typename T>
hipError_t launch_ukern(const Plan& p);
template <typename T>
hipError_t launch_observables(const Plan& p, const void* psi, const void* phi, double amp,
                              double* partials, int* nblocks);
template <typename T>
hipError_t launch_adj_update(const Plan& p, void* lam, const void* psin, const void* phin,
                             const void* phis, double amp);
template <typename T>
hipError_t launch_adj_seed(const Plan& p, void* lam, const void* psi, const void* phi, double amp,
                           double* partials, int* nblocks);
template <typename T>
hipError_t launch_overlap(const Plan& p, const void* target, const void* psi, double* partials,
                          int* nblocks);
template <typename T>
hipError_t launch_overlap_seed(const Plan& p, void* lam, const void* target, const double* coef);
template <typename T>
hipError_t launch_copy(const Plan& p, void* dst, const void* src);
// |psi|^2 into out (real, plan precision)
template <typename T>
hipError_t launch_density(const Plan& p, const void* psi, void* out);
// the nonlinear step alone over time dt with potential phi (a real grid array
// of Phi[|psi|^2]); imaginary time: per-block sums of |psi'|^2 into partials
template <typename T>
hipError_t launch_nonlinear(const Plan& p, void* psi, const void* phi, double dt, double amp,
                            double* partials, int* nblocks);

// Deterministic fixed-order reduction of partials[nblocks][width] into
// out[width] (FP64, Neumaier-compensated); optional 1/(sum[0] dV) into sigma.
hipError_t launch_reduce(const Plan& p, const double* partials, int nblocks, int width, double* out,
                         double* sigma_out, int nsets = 1, size_t set_stride = 0);
// sigma = 1 / (sum of norm partials * dV)
hipError_t launch_norm_finalize(const Plan& p, const double* partials, int nblocks, double* sigma);

// columns per block (log2) and block count of the strided sweep; ycarry: the
// variant that completes the y carries (at most 512 threads per block)
int cn_strided_logzb(const Plan& p, int axis, bool ycarry = false);
int cn_strided_blocks(const Plan& p, int axis, bool ycarry = false);

// Two-factor register FFT passes (k_fft2.hip); false when the length has no
// compiled fast path (the caller then uses the generic Stockham kernel).
template <typename T>
bool fast_rows(const Plan& p, bool inverse, const double* npart, int nnpart, double* sigma_out);
// the compiled forward rows pass can reduce the norm partials (whole waves)
template <typename T>
bool fast_rows_sigma_ok(const Plan& p);
template <typename T>
bool fast_xmul(const Plan& p);
template <typename T>
bool fast_r2c(const Plan& p, const void* psi, const double* sigma);
template <typename T>
bool fast_r2c_adj(const Plan& p, const void* mu, const void* psin, const void* phin, double amp,
                  double* partials, int* nblocks);
// fused C2R of Phi_s + adjoint nonlinear update (false: no compiled split)
template <typename T>
// zsweep: also apply the conjugate z sweep of the next reverse step where the
// fused form exists; *zdone tells whether it ran
bool fast_c2r_adjupd(const Plan& p, void* lam, const void* psin, const void* phin, double amp,
                     bool zsweep, bool* zdone);
template <typename T>
bool fast_c2r_phi(const Plan& p, void* phi);
// the C2R of Phi fused with the pointwise half step of the symmetric scheme
// (psi in place, over dt; imaginary time: block norm partials); false when the
// grid has no compiled pass (the caller then runs the C2R and the pointwise pass)
template <typename T>
bool fast_c2r_nl(const Plan& p, void* psi, double dt, double amp, double* partials, int* nblocks);
template <typename T>
bool fast_c2r_step(const Plan& p, const void* psi_in, void* psi_out, const double* sigma,
                   double amp, void* phi_out, void* ycar, bool phi_sigma);
// the compiled fused z pass can start the y solve for this plan (blocks of whole
// 16-line y segments, imaginary time)
template <typename T>
bool fast_c2r_step_yfused_ok(const Plan& p);

// kappa = 1/A - 2 of the scaled Crank-Nicolson right-hand side (conj(A) for the adjoint)
struct cx_coef {
    double re, im;
};
cx_coef cn_kappa(const Plan& p, int axis, bool conjugate);
int observables_blocks(const Plan& p);
int r2c_blocks(const Plan& p);

}  // namespace dgpe
