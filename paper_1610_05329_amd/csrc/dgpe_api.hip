// libdgpe C ABI: plan creation (validation, constant tables, launch shapes),
// the split-step time loop, the dipolar potential, the observables and the
// checkpointed adjoint.  All device memory belongs to the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "dgpe.h"
#include "dgpe_internal.h"

using namespace dgpe;

// Workspace of the allocation-free plans (dgpe_plan_create_noalloc): one array
// per device, held until the process ends.  Host code never passes this name
// to a kernel or a copy: it uses the device address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[DGPE_NOALLOC_MAX_BYTES];

// The opaque handle of the C ABI is the plan itself.
struct dgpe_plan_s : public dgpe::Plan {};

namespace {

thread_local std::string g_last_error;

dgpe_status fail(dgpe_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

#define DGPE_HIP(expr)                                                                         \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(DGPE_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));         \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kThreads = 256;
constexpr int kEmax = 16;
// LDS per block: the block shapes are chosen within 64 KB where they can be
// (several blocks per CU); a pass whose one-line block needs more takes up to
// the 160 KB a gfx950 workgroup may hold (one block per CU)
constexpr size_t kLdsBudget = 64 * 1024;
constexpr size_t kLdsMax = 160 * 1024;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// a quasi-2D plan's grid is (N1, 1, N2): the middle axis is the tight one
bool q2d_mode(uint32_t mode) { return (mode & (DGPE_Q2D_PERP | DGPE_Q2D_INPLANE)) != 0; }

bool size_ok(int n);

// at most 2^30 points (the kernels index points and lines with 32-bit integers)
constexpr int kMaxAxis = 2048;
constexpr int64_t kMaxPoints = int64_t(1) << 30;

bool points_ok(const int32_t n[3]) { return (int64_t)n[0] * n[1] * n[2] <= kMaxPoints; }

bool grid_ok(const int32_t n[3], uint32_t mode) {
    if (!points_ok(n)) return false;
    if (q2d_mode(mode)) return n[1] == 1 && size_ok(n[0]) && size_ok(n[2]);
    return size_ok(n[0]) && size_ok(n[1]) && size_ok(n[2]);
}

bool size_ok(int n) {
    if (n < 4 || n > kMaxAxis || (n & 1)) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

FftDesc factor(int L) {
    FftDesc f{};
    f.L = L;
    int r = L;
    std::vector<int> rad;
    while (r % 8 == 0) { rad.push_back(8); r /= 8; }
    if (r % 4 == 0) { rad.push_back(4); r /= 4; }
    if (r % 2 == 0) { rad.push_back(2); r /= 2; }
    while (r % 3 == 0) { rad.push_back(3); r /= 3; }
    f.nstages = (int)rad.size();
    for (int i = 0; i < f.nstages; ++i) f.radix[i] = rad[i];
    return f;
}

int ilog2(int v) {
    int l = 0;
    while ((1 << (l + 1)) <= v) ++l;
    return l;
}

// upper bound of the fused z pass's LDS (16-point segments, FP64 carries)
size_t c2r_step_lds(int Nz, int B, size_t csz) {
    const int M = Nz / 2, es = B == 1 ? 1 : B + 1, nseg = (Nz + 15) / 16;
    const size_t fcap = std::max<size_t>((size_t)(M + 1) * es, ((size_t)2 * nseg * B * 16 + csz - 1) / csz);
    return (fcap + (size_t)Nz * es + M + M + 1) * csz + 16 + (size_t)2 * nseg * 16;
}

// Block shapes for a grid; false if no shape fits the LDS budget.
bool choose_launch(const int n[3], bool f32, bool imag, Launch* lc) {
    const size_t csz = f32 ? 8 : 16;
    lc->threads = kThreads;
    const int cap = kEmax * kThreads;
    const int Nx = n[0], Ny = n[1], Nz = n[2];
    const int M = Nz / 2;
    // z passes: B lines, B | Ny, B*M <= cap, LDS within budget
    int Bz = f32 ? 16 : 8;
    while (Bz > 1 && (Ny % Bz || Bz * M > cap || c2r_step_lds(Nz, Bz, csz) > kLdsBudget)) Bz >>= 1;
    if (Bz * M > cap || c2r_step_lds(Nz, Bz, csz) > kLdsMax) return false;
    lc->logB_z = ilog2(Bz);
    // z segments (16 or 32 points): B * nseg <= threads
    int sz = 16;
    if (Bz * ((Nz + sz - 1) / sz) > kThreads) sz = 32;
    if (Bz * ((Nz + sz - 1) / sz) > kThreads) return false;
    lc->seg[2] = sz;
    // y rows
    int By = f32 ? 16 : 8;
    while (By > 1 && (By * Ny > cap || (size_t)(Ny * (By + 1) + Ny) * csz > kLdsBudget)) By >>= 1;
    if ((size_t)(Ny * (By + 1) + Ny) * csz > kLdsMax || By * Ny > cap) return false;
    lc->logB_y = ilog2(By);
    // x columns: B | Ny
    int Bx = f32 ? 16 : 8;
    while (Bx > 1 && (Ny % Bx || Bx * Nx > cap || (size_t)(Nx * (Bx + 1) + Nx) * csz > kLdsBudget))
        Bx >>= 1;
    if (Bx * Nx > cap || (size_t)(Nx * (Bx + 1) + Nx) * csz > kLdsMax) return false;
    lc->logB_x = ilog2(Bx);
    // strided sweeps: columns C, segments S, ZB | C; FP32 blocks up to 1024
    // threads, FP64 up to 512 (register budget of the segment arrays)
    for (int axis = 0; axis < 2; ++axis) {
        const int L = n[axis];
        const int C = axis == 1 ? Nz : Ny * Nz;
        const int S = 16;
        const int nseg = (L + S - 1) / S;
        // FP32 imaginary time keeps FP32 recurrences (1024-thread blocks); FP64
        // and real-time recurrences are FP64
        const bool narrow = f32 && imag;
        // FP64 states hold ~140 VGPRs (3 waves per SIMD): blocks of at most 256
        // threads keep 3 blocks per CU resident.  FP32 states in real time hold
        // the line in FP32 between the FP64 recurrences (~114 VGPRs): blocks of
        // up to 512 threads, so that 512-point lines (32 segments) still get 16
        // columns, 128-byte runs (8 columns: 264 us, 16: 230 us, 32 in
        // 1024-thread blocks: 315 us at 512 x 512 x 256)
        const int tmax = narrow ? 1024 : f32 ? 512 : 256;
        const size_t asz = narrow ? 8 : 16;
        // measured at 256^3: 32 columns per block (FP32 recurrences) and 16
        // (FP64 recurrences) overlap loads and solves better than 64
        int zb = narrow ? 32 : 16;
        while (zb > 1 && (C % zb || nseg * zb > tmax)) zb >>= 1;
        // the tables in LDS where they leave room for these columns; long lines
        // read them from global memory (L1/L2 resident) instead of giving up
        // columns (at 2048 points, FP64: 104 KB of tables left one 128-thread
        // block of one column per CU)
        auto lds = [&](int z, bool gt) {
            return (size_t)(2 * nseg * z + (gt ? 0 : 3 * nseg * (S + 1)) + 3 * nseg) * asz;
        };
        const bool gt = lds(zb, false) > kLdsBudget;
        while (zb > 1 && lds(zb, gt) > kLdsBudget) zb >>= 1;
        if (C % zb || nseg * zb > tmax || lds(zb, gt) > kLdsMax) return false;
        lc->seg[axis] = S;
        lc->logZB[axis] = ilog2(zb);
        lc->gtab[axis] = gt ? 1 : 0;
    }
    return true;
}

enum {
    OFF_SPEC, OFF_PHI, OFF_UK, OFF_TWX, OFF_TWY, OFF_TWZ, OFF_TWR, OFF_CN0, /* 6 tables */
    OFF_RED = OFF_CN0 + 6, OFF_SCAL, OFF_END
};

size_t red_count_for(const int n[3], const Launch& lc) {
    const size_t nx = n[0], ny = n[1], nz = n[2];
    size_t r = 10 * 2048;
    r = std::max(r, ny * nz);                       // x-sweep blocks (>= 1 column each)
    r = std::max(r, nx * nz);                       // y-sweep blocks
    r = std::max(r, 4 * nx * (ny >> lc.logB_z));    // adjoint r2c partials
    return r;
}

// Computes the workspace carve-up; offs[OFF_END] is the total.
bool layout(const int n[3], bool f32, size_t offs[OFF_END + 1], Launch* lc_out,
            bool imag = true) {
    Launch lc{};
    if (!choose_launch(n, f32, imag, &lc)) return false;
    Launch other;  // the workspace serves both time modes (dgpe_plan_set)
    if (!choose_launch(n, f32, !imag, &other)) return false;
    if (lc_out) *lc_out = lc;
    const size_t csz = f32 ? 8 : 16, rsz = f32 ? 4 : 8;
    const size_t nx = n[0], ny = n[1], nz = n[2];
    size_t sz[OFF_END];
    sz[OFF_SPEC] = (nz / 2 + 1) * nx * ny * csz;
    sz[OFF_PHI] = nx * ny * nz * rsz;
    sz[OFF_UK] = (nz / 2 + 1) * (ny / 2 + 1) * (nx / 2 + 1) * rsz;
    sz[OFF_TWX] = nx * csz;
    sz[OFF_TWY] = ny * csz;
    sz[OFF_TWZ] = (nz / 2) * csz;
    sz[OFF_TWR] = (nz / 2 + 1) * csz;
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 2; ++c) sz[OFF_CN0 + 2 * a + c] = TAB_COUNT * (size_t)n[a] * 16;
    sz[OFF_RED] = red_count_for(n, lc) * sizeof(double);
    sz[OFF_SCAL] = 16 * sizeof(double);
    size_t o = 0;
    for (int i = 0; i < OFF_END; ++i) {
        offs[i] = o;
        o += align_up(sz[i]);
    }
    offs[OFF_END] = o;
    return true;
}

// W_L^m = exp(-2 pi i m / L) in extended precision, rounded once.
template <typename T>
std::vector<T> twiddles(int L, int count) {
    std::vector<T> out(2 * (size_t)count);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int m = 0; m < count; ++m) {
        const long double a = -2.0L * pi * (long double)m / (long double)L;
        out[2 * m] = (T)cosl(a);
        out[2 * m + 1] = (T)sinl(a);
    }
    return out;
}

// Thomas factors of tridiag(-A, 1 + 2A, -A) and the segment carry products:
// alpha_i = A m_i with m_0 = 1/(1 + 2A), m_i = 1/(1 + 2A - A^2 m_{i-1}).
template <typename T>
std::vector<T> cn_tables(int N, std::complex<long double> A, int S) {
    using C = std::complex<long double>;
    std::vector<C> al(N), P(N), Q(N), E(N), G(N), pend(N, C(0)), qbeg(N, C(0)), H(N, C(0));
    const C diag = C(1) + C(2) * A;
    C m = C(1) / diag;
    for (int i = 0; i < N; ++i) {
        if (i > 0) m = C(1) / (diag - A * A * m);
        al[i] = A * m;
    }
    for (int s0 = 0, k = 0; s0 < N; s0 += S, ++k) {
        const int s1 = std::min(s0 + S, N);
        C acc = 1;
        for (int i = s0; i < s1; ++i) { acc *= al[i]; P[i] = acc; }
        pend[k] = acc;
        acc = 1;
        for (int i = s1 - 1; i >= s0; --i) { acc *= al[i]; Q[i] = acc; }
        qbeg[k] = acc;
        acc = 0;
        for (int i = s1 - 1; i >= s0; --i) { acc = P[i] + al[i] * acc; E[i] = acc; }
        acc = 1;
        for (int i = s0; i < s1; ++i) { G[i] = acc; acc *= al[i]; }
        acc = 0;
        for (int i = s0; i < s1; ++i) acc += G[i] * P[i];
        H[k] = acc;
    }
    std::vector<T> out(2 * TAB_COUNT * (size_t)N);
    const std::vector<C>* tabs[TAB_COUNT];
    tabs[TAB_ALPHA] = &al;
    tabs[TAB_P] = &P;
    tabs[TAB_Q] = &Q;
    tabs[TAB_PEND] = &pend;
    tabs[TAB_QBEG] = &qbeg;
    tabs[TAB_E] = &E;
    tabs[TAB_G] = &G;
    tabs[TAB_H] = &H;
    for (int t = 0; t < TAB_COUNT; ++t)
        for (int i = 0; i < N; ++i) {
            out[2 * ((size_t)t * N + i)] = (T)(*tabs[t])[i].real();
            out[2 * ((size_t)t * N + i) + 1] = (T)(*tabs[t])[i].imag();
        }
    return out;
}

template <typename T>
dgpe_status upload(void* dst, const std::vector<T>& v) {
    DGPE_HIP(hipMemcpy(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return DGPE_OK;
}

template <typename T>
dgpe_status build_cn_tables(Plan& p) {
    for (int a = 0; a < 3; ++a) {
        const long double c = (long double)p.dt / (4.0L * (long double)p.d[a] * (long double)p.d[a]);
        for (int cj = 0; cj < 2; ++cj) {
            std::complex<long double> A = p.imag ? std::complex<long double>(c, 0)
                                                 : std::complex<long double>(0, cj ? -c : c);
            dgpe_status s = upload(p.cntab[a][cj], cn_tables<double>(p.n[a], A, p.lc.seg[a]));
            if (s != DGPE_OK) return s;
        }
    }
    return DGPE_OK;
}

template <typename T>
dgpe_status build_tables(Plan& p) {
    dgpe_status s;
    if ((s = upload(p.tw[0], twiddles<T>(p.n[0], p.n[0]))) != DGPE_OK) return s;
    if ((s = upload(p.tw[1], twiddles<T>(p.n[1], p.n[1]))) != DGPE_OK) return s;
    if ((s = upload(p.tw[2], twiddles<T>(p.n[2] / 2, p.n[2] / 2))) != DGPE_OK) return s;
    if ((s = upload(p.twr2c, twiddles<T>(p.n[2], p.n[2] / 2 + 1))) != DGPE_OK) return s;
    if ((s = build_cn_tables<T>(p)) != DGPE_OK) return s;
    DGPE_HIP(launch_ukern<T>(p));
    DGPE_HIP(hipStreamSynchronize(p.stream));
    return DGPE_OK;
}

bool finite3(const double* v) {
    return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

dgpe_status check_ptr(const void* ptr, const char* what) {
    if (!ptr) return fail(DGPE_EINVAL, std::string(what) + " is NULL");
    if (reinterpret_cast<uintptr_t>(ptr) % kAlign)
        return fail(DGPE_EINVAL, std::string(what) + " is not 256-byte aligned");
    return DGPE_OK;
}

// ---- the time loop ---------------------------------------------------------

// A grid with one point along y (the quasi-2D plans) has no y transform and
// no y sweep.
bool has_y(const Plan& p) { return p.n[1] > 1; }

template <typename T>
dgpe_status convolve_density(Plan& p, const void* psi, const double* sigma) {
    DGPE_HIP(launch_r2c_density<T>(p, psi, sigma));
    if (has_y(p)) DGPE_HIP(launch_rows<T>(p, false));
    DGPE_HIP(launch_xmul<T>(p));
    if (has_y(p)) DGPE_HIP(launch_rows<T>(p, true));
    return DGPE_OK;
}

// Optional per-pass event pairs (measurement only).
struct PassTimer {
    std::vector<hipEvent_t> ev;  // [launch][2]
    std::vector<int> kind;
    hipStream_t stream = nullptr;
    bool on = false;
    hipError_t begin(int k) {
        if (!on) return hipSuccess;
        hipEvent_t a, b;
        hipError_t e = hipEventCreate(&a);
        if (e != hipSuccess) return e;
        if ((e = hipEventCreate(&b)) != hipSuccess) {
            (void)hipEventDestroy(a);
            return e;
        }
        ev.push_back(a);
        ev.push_back(b);
        kind.push_back(k);
        return hipEventRecord(a, stream);
    }
    hipError_t end() { return on ? hipEventRecord(ev.back(), stream) : hipSuccess; }
    ~PassTimer() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

#define DGPE_PASS(timer, k, expr)       \
    do {                                \
        DGPE_HIP((timer).begin(k));     \
        DGPE_HIP(expr);                 \
        DGPE_HIP((timer).end());        \
    } while (0)

// The y solve starts inside the fused z pass (16-line segments, zero carries),
// a carry pass joins the segments and the x sweep adds the carries while it
// loads: imaginary time, compiled fused pass, Ny / 16 <= 16 segments, state
// under 4 GiB (32-bit offsets in the x sweep).  The carry inputs
// ([3][Nx][Ny/16][Nz] complex) and the carry pairs (the same count times 2),
// together 5/16 of the state's bytes, live in the Phi buffer (half the
// state's bytes), which stepping does not otherwise use in imaginary time.
template <typename T>
bool use_fused_y(const Plan& p) {
    const size_t state = (size_t)p.n[0] * p.n[1] * p.n[2] * 2 * sizeof(T);
    return p.fuse_y && p.fast && p.imag && p.n[1] / 16 <= 16 &&
           state < (size_t(1) << 32) && fast_c2r_step_yfused_ok<T>(p);
}

bool fused_y(const Plan& p) { return p.f32 ? use_fused_y<float>(p) : use_fused_y<double>(p); }

// the fused y schedule also folds the norm reduction into the forward y FFT
// when that pass is compiled with whole waves
template <typename T>
bool use_folded_norm(const Plan& p) {
    return use_fused_y<T>(p) && p.scheme == 0 && fast_rows_sigma_ok<T>(p);
}

// The nonlinear phase of the fused z pass runs over dt_nl instead of dt while
// this guard lives.
struct NonlinearStep {
    Plan& p;
    NonlinearStep(Plan& plan, double dt_nl) : p(plan) { p.dt_nl = dt_nl; }
    ~NonlinearStep() { p.dt_nl = p.dt; }
};

// nsteps symmetric (Strang) steps in place: nonlinear over dt/2 from the
// density of the incoming state, the three sweeps over dt, nonlinear over dt/2
// from the density after the sweeps, then (imaginary time) renormalisation.
// The leading half runs inside the fused z pass.  In real time the phase
// keeps |psi|, so the trailing half of one step and the leading half of the
// next see the same density and run as one phase over dt (trap amplitude the
// mean of the two steps'); the last step's trailing half is a pass of its own.
// In imaginary time each trailing half convolves the density after the sweeps
// and reduces the norm of its result (applied lazily by the next step); the
// sweeps take the fused y schedule where the plan has it (the y solve started
// in the fused z pass, completed by the carry pass and the x sweep).
template <typename T>
dgpe_status run_steps_strang(Plan& p, void* psi, int nsteps, const double* amp, PassTimer& t) {
    double* sigma = p.scal;
    void* car = use_fused_y<T>(p) ? p.phi : nullptr;
    const size_t car_bytes = (size_t)p.n[0] * (p.n[1] / 16) * p.n[2] * 2 * sizeof(T);  // one array
    for (int s = 0; s < nsteps; ++s) {
        const double a = amp ? amp[s] : 1.0;
        const double* sg = (p.imag && s > 0) ? sigma : nullptr;
        const bool merged = !p.imag && s > 0;
        const double a_nl = merged ? 0.5 * ((amp ? amp[s - 1] : 1.0) + a) : a;
        DGPE_PASS(t, 0, (launch_r2c_density<T>(p, psi, sg)));
        if (has_y(p)) DGPE_PASS(t, 1, (launch_rows<T>(p, false)));
        DGPE_PASS(t, 2, (launch_xmul<T>(p)));
        if (has_y(p)) DGPE_PASS(t, 3, (launch_rows<T>(p, true)));
        {
            NonlinearStep half(p, merged ? p.dt : 0.5 * p.dt);
            DGPE_PASS(t, 4, (launch_c2r_step<T>(p, psi, psi, sg, a_nl, nullptr, car)));
        }
        if (car) {
            DGPE_PASS(t, 5, (launch_cn_ycarry<T>(p, car)));
            DGPE_PASS(t, 6, (launch_cn_strided<T>(p, psi, 0, false, nullptr, (char*)car + 3 * car_bytes)));
        } else {
            if (has_y(p)) DGPE_PASS(t, 5, (launch_cn_strided<T>(p, psi, 1, false, nullptr)));
            DGPE_PASS(t, 6, (launch_cn_strided<T>(p, psi, 0, false, nullptr)));
        }
        if (p.imag || s + 1 == nsteps) {  // the trailing half as a pass of its own
            dgpe_status st = convolve_density<T>(p, psi, nullptr);
            if (st != DGPE_OK) return st;
            int nb = 0;
            // the C2R of Phi fused with the pointwise step where compiled
            if (!(p.fast && fast_c2r_nl<T>(p, psi, 0.5 * p.dt, a, p.red, &nb))) {
                DGPE_HIP(launch_c2r_phi<T>(p, p.phi));
                DGPE_HIP(launch_nonlinear<T>(p, psi, p.phi, 0.5 * p.dt, a, p.red, &nb));
            }
            DGPE_HIP(hipGetLastError());
            if (p.imag) DGPE_PASS(t, 7, (launch_norm_finalize(p, p.red, nb, sigma)));
        }
    }
    if (p.imag && nsteps > 0) DGPE_HIP(launch_scale<T>(p, psi, sigma));
    return DGPE_OK;
}

// nsteps steps in place on psi; with psi_in, the first step reads psi_in
// instead (out of place) and, with phi_out, also writes Phi of psi_in's density.
template <typename T>
dgpe_status run_steps(Plan& p, void* psi, int nsteps, const double* amp, PassTimer* tm = nullptr,
                      const void* psi_in = nullptr, void* phi_out = nullptr) {
    PassTimer none;
    PassTimer& t = tm ? *tm : none;
    if (p.scheme == 1 && !psi_in && !phi_out) return run_steps_strang<T>(p, psi, nsteps, amp, t);
    double* sigma = p.scal;
    void* car = use_fused_y<T>(p) ? p.phi : nullptr;
    const size_t car_bytes = (size_t)p.n[0] * (p.n[1] / 16) * p.n[2] * 2 * sizeof(T);  // one array
    const int nb_x = cn_strided_blocks(p, 0, car != nullptr);
    // with the fused y schedule the previous step's norm is reduced inside the
    // forward y FFT (block 0) and applied to Phi in the fused z pass; P1 then
    // transforms the unscaled density
    const bool fold = car && use_folded_norm<T>(p);
    for (int s = 0; s < nsteps; ++s) {
        const double a = amp ? amp[s] : 1.0;
        const double* sg = (p.imag && s > 0) ? sigma : nullptr;
        const void* src = (s == 0 && psi_in) ? psi_in : psi;
        void* phs = s == 0 ? phi_out : nullptr;
        DGPE_PASS(t, 0, (launch_r2c_density<T>(p, src, fold ? nullptr : sg)));
        if (fold && sg)
            DGPE_PASS(t, 1, (launch_rows<T>(p, false, p.red, nb_x, sigma)));
        else if (has_y(p))
            DGPE_PASS(t, 1, (launch_rows<T>(p, false)));
        DGPE_PASS(t, 2, (launch_xmul<T>(p)));
        if (has_y(p)) DGPE_PASS(t, 3, (launch_rows<T>(p, true)));
        if (car && !phs) {
            DGPE_PASS(t, 4, (launch_c2r_step<T>(p, src, psi, sg, a, nullptr, car, fold && sg)));
            DGPE_PASS(t, 5, (launch_cn_ycarry<T>(p, car)));
            DGPE_PASS(t, 6, (launch_cn_strided<T>(p, psi, 0, false, p.red,
                                                  (char*)car + 3 * car_bytes)));
        } else {
            DGPE_PASS(t, 4, (launch_c2r_step<T>(p, src, psi, sg, a, phs)));
            if (has_y(p)) DGPE_PASS(t, 5, (launch_cn_strided<T>(p, psi, 1, false, nullptr)));
            DGPE_PASS(t, 6, (launch_cn_strided<T>(p, psi, 0, false, p.imag ? p.red : nullptr)));
        }
        if (p.imag && (!fold || s + 1 == nsteps))
            DGPE_PASS(t, 7, (launch_norm_finalize(p, p.red, nb_x, sigma)));
    }
    if (p.imag && nsteps > 0) DGPE_HIP(launch_scale<T>(p, psi, sigma));
    return DGPE_OK;
}

void pass_bytes(const Plan& p, double b[DGPE_NPASS]) {
    const double s = p.f32 ? 4.0 : 8.0;
    const double nt = (double)p.n[0] * p.n[1] * p.n[2];
    const double state = 2.0 * s * nt;
    const double spec = 2.0 * s * (double)p.n[0] * p.n[1] * (p.n[2] / 2 + 1);
    const double uk = s * (double)(p.n[0] / 2 + 1) * (p.n[1] / 2 + 1) * (p.n[2] / 2 + 1);
    b[0] = state + spec;         // read psi, write S
    b[1] = 2.0 * spec;           // S in place
    b[2] = 2.0 * spec + uk;      // S in place + kernel table
    b[3] = 2.0 * spec;
    b[4] = spec + 2.0 * state;   // read S and psi, write psi
    b[5] = 2.0 * state;          // psi in place
    b[6] = 2.0 * state;
    if (!has_y(p)) b[1] = b[3] = b[5] = 0.0;  // no y passes
    if (fused_y(p)) {
        const bool fold = p.f32 ? use_folded_norm<float>(p) : use_folded_norm<double>(p);
        if (fold) b[1] += 8.0 * cn_strided_blocks(p, 0, true);  // the norm partials
        const double car = state / 16.0;  // one carry array [Nx][Ny/16][Nz]
        b[4] += 3.0 * car;                // + the three carry inputs
        b[5] = 5.0 * car;                 // carry pass: read 3, write the (c_d, c_x) pairs
        b[6] += 2.0 * car;                // x sweep: + c_d, c_x
    }
    b[7] = p.imag ? 8.0 * cn_strided_blocks(p, 0, fused_y(p)) + 8.0 : 0.0;
}

template <typename T>
dgpe_status observables_impl(Plan& p, const void* psi, double amp, dgpe_obs* out) {
    dgpe_status st = convolve_density<T>(p, psi, nullptr);
    if (st != DGPE_OK) return st;
    DGPE_HIP(launch_c2r_phi<T>(p, p.phi));
    int nb = 0;
    DGPE_HIP(launch_observables<T>(p, psi, p.phi, amp, p.red, &nb));
    DGPE_HIP(launch_reduce(p, p.red, nb, 10, p.scal + 2, nullptr));
    double h[10];
    DGPE_HIP(hipMemcpyAsync(h, p.scal + 2, sizeof(h), hipMemcpyDeviceToHost, p.stream));
    DGPE_HIP(hipStreamSynchronize(p.stream));
    const double dV = p.d[0] * p.d[1] * p.d[2];
    const double nrm = h[0] * dV;
    // (a quasi-2D plan has no kinetic energy along its tight axis)
    const double ky = p.q2d ? 0.0 : h[2] / (p.d[1] * p.d[1]);
    const double ekin = 0.5 * (h[1] / (p.d[0] * p.d[0]) + ky + h[3] / (p.d[2] * p.d[2])) * dV;
    const double etrap = amp * h[4] * dV;
    const double ec = 0.5 * p.g * h[5] * dV;
    const double edd = 0.5 * p.gd * h[6] * dV;
    out->norm = nrm;
    out->e_kin = ekin;
    out->e_trap = etrap;
    out->e_contact = ec;
    out->e_dd = edd;
    out->energy = (ekin + etrap + ec + edd) / nrm;
    out->mu = (ekin + etrap + 2.0 * ec + 2.0 * edd) / nrm;
    const double mx = h[7] * dV / nrm, my = h[8] * dV / nrm, mz = h[9] * dV / nrm;
    out->rms[0] = std::sqrt(mx);
    out->rms[1] = std::sqrt(my);
    out->rms[2] = std::sqrt(mz);
    out->rms[3] = std::sqrt(mx + my + mz);
    for (int i = 0; i < 10; ++i)
        if (!std::isfinite(h[i])) return fail(DGPE_ENONFINITE, "observables: non-finite sum");
    return DGPE_OK;
}

// ---- adjoint ---------------------------------------------------------------

struct AdjLayout {
    size_t ckpt, seg, lam, phin, phis, sums, part, scratch, end;
    int nckpt;
};

// K > 1: a checkpoint every K steps and one segment of K recomputed states
// with their Phi.  K = 1: every state psi_1..psi_N and the Phi of every state
// psi_0..psi_{N-1}, kept from the forward sweep (no recompute).
AdjLayout adj_layout(const Plan& p, int nsteps, int K) {
    AdjLayout L{};
    const size_t nt = (size_t)p.n[0] * p.n[1] * p.n[2];
    const size_t csz = p.f32 ? 8 : 16, rsz = p.f32 ? 4 : 8;
    const size_t st = align_up(nt * csz);
    const bool all = K == 1;
    const int nphi = all ? nsteps : K;  // Phi slots and partial sets
    L.nckpt = (nsteps + K - 1) / K;
    size_t o = 0;
    L.ckpt = o;
    o += st * (size_t)std::max(L.nckpt, 1);
    L.seg = o;
    o += st * (size_t)(all ? 0 : K);
    L.lam = o;
    o += st;
    L.phin = o;  // Phi of the states, one slot per step
    o += align_up(nt * rsz) * (size_t)nphi;
    L.phis = o;
    o += align_up(nt * rsz);
    L.sums = o;
    o += align_up((size_t)(nsteps + 1) * 4 * sizeof(double));
    L.part = o;  // partials: one set per step of a segment (of the run for K = 1)
    o += align_up(red_count_for(p.n, p.lc) * sizeof(double)) * (size_t)nphi;
    L.scratch = o;
    o += align_up(16 * sizeof(double));
    L.end = o;
    return L;
}

template <typename T>
dgpe_status adjoint_impl(Plan& p, const void* psi0, int nsteps, const double* amp, int K,
                         int objective, const void* target, char* ws, void* psi_final, double* J,
                         double* dJ_damp, double* dJ_dtrap, void* dJ_dpsi0) {
    const AdjLayout L = adj_layout(p, nsteps, K);
    const size_t nt = (size_t)p.n[0] * p.n[1] * p.n[2];
    const size_t st = align_up(nt * sizeof(T) * 2);
    auto state = [&](size_t base, int i) { return (void*)(ws + base + st * (size_t)i); };
    void* lam = ws + L.lam;
    const size_t phi_bytes = align_up(nt * sizeof(T));
    auto phi_slot = [&](int i) { return (void*)(ws + L.phin + phi_bytes * (size_t)i); };
    void* phis = ws + L.phis;
    double* sums = (double*)(ws + L.sums);
    double* part = (double*)(ws + L.part);
    const size_t set_stride = align_up(red_count_for(p.n, p.lc) * sizeof(double)) / sizeof(double);
    int nbs = 0;  // partial blocks of the adjoint source pass (the same for every step)
    double* scratch = (double*)(ws + L.scratch);
    // K = 1: psi_n for n >= 1 in checkpoint slot n - 1, psi_0 the caller's
    const bool all = K == 1;
    auto kept = [&](int n) -> const void* { return n == 0 ? psi0 : state(L.ckpt, n - 1); };
    // forward sweep, storing the state at the start of every segment (K = 1:
    // every state, stepping out of place, and the Phi each step starts from)
    void* cur = nullptr;
    if (all) {
        for (int n = 0; n < nsteps; ++n) {
            dgpe_status stt = run_steps<T>(p, state(L.ckpt, n), 1, amp + n, nullptr, kept(n), phi_slot(n));
            if (stt != DGPE_OK) return stt;
        }
        cur = state(L.ckpt, nsteps - 1);
    } else {
        cur = state(L.seg, 0);
        DGPE_HIP(launch_copy<T>(p, cur, psi0));
        for (int s = 0; s < L.nckpt; ++s) {
            const int n0 = s * K, len = std::min(K, nsteps - n0);
            DGPE_HIP(launch_copy<T>(p, state(L.ckpt, s), cur));
            dgpe_status stt = run_steps<T>(p, cur, len, amp + n0);
            if (stt != DGPE_OK) return stt;
        }
    }
    if (psi_final) DGPE_HIP(launch_copy<T>(p, psi_final, cur));
    const double dV = p.d[0] * p.d[1] * p.d[2];
    const double aN = amp[nsteps];
    std::vector<double> hs((size_t)(nsteps + 1) * 4, 0.0);
    double seed4[4] = {0, 0, 0, 0};
    // seed
    if (objective == DGPE_OBJ_ENERGY) {
        dgpe_obs o;
        dgpe_status stt = observables_impl<T>(p, cur, aN, &o);
        if (stt != DGPE_OK) return stt;
        *J = o.e_kin + o.e_trap + o.e_contact + o.e_dd;
        // p.phi holds Phi[|psi_N|^2] from the observables
        int nb = 0;
        DGPE_HIP(launch_adj_seed<T>(p, lam, cur, p.phi, aN, part, &nb));
        DGPE_HIP(launch_reduce(p, part, nb, 4, scratch, nullptr));
        DGPE_HIP(hipMemcpyAsync(seed4, scratch, sizeof(seed4), hipMemcpyDeviceToHost, p.stream));
    } else {
        int nb = 0;
        DGPE_HIP(launch_overlap<T>(p, target, cur, part, &nb));
        DGPE_HIP(launch_reduce(p, part, nb, 2, scratch, nullptr));
        double c2[2];
        DGPE_HIP(hipMemcpyAsync(c2, scratch, sizeof(c2), hipMemcpyDeviceToHost, p.stream));
        DGPE_HIP(hipStreamSynchronize(p.stream));
        const double cr = c2[0] * dV, ci = c2[1] * dV;
        *J = cr * cr + ci * ci;
        const double coef[2] = {2.0 * dV * cr, 2.0 * dV * ci};
        DGPE_HIP(launch_overlap_seed<T>(p, lam, target, coef));
    }
    // one reverse step: the conjugate sweeps, the adjoint source and its
    // convolution, the nonlinear adjoint update; source sums into partial set i.
    // The reverse steps run n = nsteps - 1 down to 0 on lam, recomputation
    // between them touching other buffers; the compiled update of step n > 0
    // also applies the conjugate z sweep that opens step n - 1 (zpre).
    bool zpre = false;
    auto reverse_step = [&](int n, const void* psin, const void* phin, int i) -> dgpe_status {
        if (!zpre) DGPE_HIP(launch_cn_z<T>(p, lam, true));
        DGPE_HIP(launch_cn_strided<T>(p, lam, 1, true, nullptr));
        DGPE_HIP(launch_cn_strided<T>(p, lam, 0, true, nullptr));
        DGPE_HIP(launch_r2c_adjoint_s<T>(p, lam, psin, phin, amp[n], part + set_stride * i, &nbs));
        DGPE_HIP(launch_rows<T>(p, false));
        DGPE_HIP(launch_xmul<T>(p));
        DGPE_HIP(launch_rows<T>(p, true));
        zpre = false;
        if (!(p.fast && fast_c2r_adjupd<T>(p, lam, psin, phin, amp[n], n > 0, &zpre))) {
            DGPE_HIP(launch_c2r_phi<T>(p, phis));
            DGPE_HIP(launch_adj_update<T>(p, lam, psin, phin, phis, amp[n]));
        }
        DGPE_HIP(hipGetLastError());
        return DGPE_OK;
    };
    if (all) {
        // every state and its Phi kept: no recompute; the source sums of all
        // steps reduced in one launch (one block per step)
        for (int n = nsteps - 1; n >= 0; --n) {
            dgpe_status stt = reverse_step(n, kept(n), phi_slot(n), n);
            if (stt != DGPE_OK) return stt;
        }
        DGPE_HIP(launch_reduce(p, part, nbs, 4, sums, nullptr, nsteps, set_stride));
    }
    // reverse sweep over segments
    for (int s = all ? -1 : L.nckpt - 1; s >= 0; --s) {
        const int n0 = s * K, len = std::min(K, nsteps - n0);
        DGPE_HIP(launch_copy<T>(p, state(L.seg, 0), state(L.ckpt, s)));
        // recompute the segment out of place; each step also leaves Phi of
        // the state it started from
        for (int i = 1; i < len; ++i) {
            dgpe_status stt = run_steps<T>(p, state(L.seg, i), 1, amp + n0 + i - 1, nullptr,
                                           state(L.seg, i - 1), phi_slot(i - 1));
            if (stt != DGPE_OK) return stt;
        }
        for (int i = len - 1; i >= 0; --i) {
            void* psin = state(L.seg, i);
            void* phin = phi_slot(i);
            if (i == len - 1) {  // the last state of the segment was never stepped from
                dgpe_status stt = convolve_density<T>(p, psin, nullptr);
                if (stt != DGPE_OK) return stt;
                DGPE_HIP(launch_c2r_phi<T>(p, phin));
            }
            dgpe_status stt = reverse_step(n0 + i, psin, phin, i);
            if (stt != DGPE_OK) return stt;
        }
        // the segment's source sums, one reduction block per step
        DGPE_HIP(launch_reduce(p, part, nbs, 4, sums + (size_t)n0 * 4, nullptr, len, set_stride));
    }
    if (dJ_dpsi0) DGPE_HIP(launch_copy<T>(p, dJ_dpsi0, lam));
    DGPE_HIP(hipMemcpyAsync(hs.data(), sums, (size_t)nsteps * 4 * sizeof(double),
                            hipMemcpyDeviceToHost, p.stream));
    DGPE_HIP(hipStreamSynchronize(p.stream));
    for (int j = 0; j < 3; ++j) dJ_dtrap[j] = 0.0;
    for (int n = 0; n < nsteps; ++n) {
        dJ_damp[n] = p.dt * hs[(size_t)n * 4];
        for (int j = 0; j < 3; ++j) dJ_dtrap[j] += p.dt * amp[n] * p.trap[j] * hs[(size_t)n * 4 + 1 + j];
    }
    dJ_damp[nsteps] = 0.0;
    if (objective == DGPE_OBJ_ENERGY) {
        dJ_damp[nsteps] = dV * seed4[0];
        for (int j = 0; j < 3; ++j) dJ_dtrap[j] += dV * aN * p.trap[j] * seed4[1 + j];
    }
    for (int n = 0; n <= nsteps; ++n)
        if (!std::isfinite(dJ_damp[n])) return fail(DGPE_ENONFINITE, "adjoint: non-finite gradient");
    if (!std::isfinite(*J)) return fail(DGPE_ENONFINITE, "adjoint: non-finite objective");
    return DGPE_OK;
}


// ---- plan creation ---------------------------------------------------------

dgpe_status check_plan_args(const int32_t n[3], const double d[3], double dt, const double trap[3],
                            double g, double gd, double cutoff_R, uint32_t mode) {
    if (!n || !d || !trap) return fail(DGPE_EINVAL, "n, d and trap must be non-NULL");
    if (mode & ~(DGPE_REAL | DGPE_F32 | DGPE_Q2D_PERP | DGPE_Q2D_INPLANE))
        return fail(DGPE_EINVAL, "unknown mode bits");
    if ((mode & DGPE_Q2D_PERP) && (mode & DGPE_Q2D_INPLANE))
        return fail(DGPE_EINVAL, "DGPE_Q2D_PERP and DGPE_Q2D_INPLANE exclude each other");
    if (q2d_mode(mode) && n[1] != 1)
        return fail(DGPE_EUNSUPPORTED_SIZE, "a quasi-2D grid is (N1, 1, N2)");
    for (int a = 0; a < 3; ++a)
        if (!(q2d_mode(mode) && a == 1) && !size_ok(n[a]))
            return fail(DGPE_EUNSUPPORTED_SIZE,
                        "grid size " + std::to_string(n[a]) +
                            " must be even, of the form 2^a 3^b, and in [4, 2048]");
    if (!points_ok(n)) return fail(DGPE_EUNSUPPORTED_SIZE, "the grid has more than 2^30 points");
    for (int a = 0; a < 3; ++a)
        if (!(d[a] > 0) || !std::isfinite(d[a])) return fail(DGPE_EINVAL, "spacings must be finite and > 0");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(DGPE_EINVAL, "dt must be finite and > 0");
    if (!finite3(trap) || !std::isfinite(g) || !std::isfinite(gd) || !std::isfinite(cutoff_R))
        return fail(DGPE_EINVAL, "trap, g, gd and cutoff must be finite");
    if (q2d_mode(mode) && !(trap[1] > 0))
        return fail(DGPE_EINVAL, "a quasi-2D plan needs the tight trap frequency trap[1] > 0");
    return DGPE_OK;
}

// Generation of the allocation-free scratch per device: each allocation-free
// plan records the value its creation set; a later creation on the same
// device overwrites the tables, and the older plan is then refused.
constexpr int kMaxDevices = 64;
std::atomic<uint64_t> g_scratch_gen[kMaxDevices];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each device

// Contact coupling the kernels use: g, or for a quasi-2D plan g int phi^4 =
// g / (sqrt(2 pi) l) over the tight trap's ground state phi, l = 1/sqrt(trap[1]).
double contact_coupling(const Plan& p) {
    return p.q2d ? p.g_in * std::sqrt(p.trap[1] / (2.0 * M_PI)) : p.g_in;
}

dgpe_status create_plan(dgpe_plan* out, const int32_t n[3], const double d[3], double dt,
                        const double trap[3], double g, double gd, double cutoff_R, uint32_t mode,
                        void* workspace, size_t workspace_bytes, hipStream_t stream,
                        bool static_ws) {
    const bool f32 = (mode & DGPE_F32) != 0;
    int nn[3] = {n[0], n[1], n[2]};
    size_t offs[OFF_END + 1];
    Launch lc{};
    if (!layout(nn, f32, offs, &lc, (mode & DGPE_REAL) == 0))
        return fail(DGPE_EUNSUPPORTED_SIZE, "no launch shape fits this grid");
    dgpe_status st = check_ptr(workspace, "workspace");
    if (st != DGPE_OK) return fail(DGPE_EWORKSPACE, dgpe_last_error());
    if (workspace_bytes < offs[OFF_END])
        return fail(DGPE_EWORKSPACE, "workspace too small: need " + std::to_string(offs[OFF_END]) +
                                         " bytes");
    int dev = 0;
    DGPE_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(DGPE_EINVAL, "device index out of range");
    dgpe_plan_s* p = new (std::nothrow) dgpe_plan_s();
    if (!p) return fail(DGPE_EINVAL, "out of host memory");
    for (int a = 0; a < 3; ++a) {
        p->n[a] = n[a];
        p->d[a] = d[a];
        p->trap[a] = trap[a];
    }
    p->dt = dt;
    p->dt_nl = dt;
    p->scheme = 0;
    p->q2d = (mode & DGPE_Q2D_PERP) ? 1 : (mode & DGPE_Q2D_INPLANE) ? 2 : 0;
    if (p->q2d) p->d[1] = 1.0;  // no spacing along the tight axis: dV = d1 d2
    p->g_in = g;
    p->g = contact_coupling(*p);
    p->gd = gd;
    p->R = cutoff_R > 0 ? cutoff_R
           : p->q2d   ? 0.5 * std::min(n[0] * d[0], n[2] * d[2])
                      : 0.5 * std::min({n[0] * d[0], n[1] * d[1], n[2] * d[2]});
    p->imag = (mode & DGPE_REAL) == 0;
    p->f32 = f32;
    p->stream = stream;
    p->lc = lc;
    p->device = dev;
    p->static_ws = static_ws;
    p->ws_gen = static_ws ? g_scratch_gen[p->device].load() : 0;
    char* ws = (char*)workspace;
    p->ws = ws;
    p->ws_bytes = workspace_bytes;
    p->spec = ws + offs[OFF_SPEC];
    p->phi = ws + offs[OFF_PHI];
    p->ukern = ws + offs[OFF_UK];
    p->tw[0] = ws + offs[OFF_TWX];
    p->tw[1] = ws + offs[OFF_TWY];
    p->tw[2] = ws + offs[OFF_TWZ];
    p->twr2c = ws + offs[OFF_TWR];
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 2; ++c) p->cntab[a][c] = ws + offs[OFF_CN0 + 2 * a + c];
    p->red = (double*)(ws + offs[OFF_RED]);
    p->scal = (double*)(ws + offs[OFF_SCAL]);
    p->red_count = red_count_for(nn, lc);
    p->fx = factor(n[0]);
    p->fy = factor(n[1]);
    p->fz = factor(n[2] / 2);
    p->fast = true;
    p->fuse_y = true;
    st = f32 ? build_tables<float>(*p) : build_tables<double>(*p);
    if (st != DGPE_OK) {
        delete p;
        return st;
    }
    *out = p;
    return DGPE_OK;
}

// A plan on the allocation-free scratch is usable until the next
// allocation-free plan is created on its device.
dgpe_status plan_live(const Plan& p) {
    if (p.static_ws && g_scratch_gen[p.device].load() != p.ws_gen)
        return fail(DGPE_ESTATE,
                    "this allocation-free plan was superseded by a later one on the same device "
                    "(they share one scratch array)");
    return DGPE_OK;
}

// Device address of the scratch array on device dev, looked up once per
// device with that device current (the host-side name is not a device address).
dgpe_status scratch_for_device(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(DGPE_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        DGPE_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(DGPE_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return DGPE_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================

// A fixed sequence of launches on the plan's stream, captured as a HIP graph
// on its first run and replayed afterwards (plain launches if capture is not
// possible).  The capture runs on a private stream that stands in for the
// plan's (the legacy default stream cannot be captured); the replays go to the
// plan's stream, in order with its other work.  The sequence must record no
// memset and call nothing that synchronises.  Plans that must not allocate
// (static workspace) keep plain launches: instantiating a graph allocates.
struct ChunkGraph {
    Plan& p;
    hipStream_t cs = nullptr;
    hipGraphExec_t exec = nullptr;
    bool eager = false;
    explicit ChunkGraph(Plan& plan) : p(plan), eager(plan.static_ws) {}
    ~ChunkGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (cs) (void)hipStreamDestroy(cs);
    }
    template <typename F>
    dgpe_status run(F launches) {
        if (!exec && !eager) {
            eager = true;  // unless everything below succeeds
            hipGraph_t g = nullptr;
            if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess &&
                hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
                const hipStream_t own = p.stream;
                p.stream = cs;
                const dgpe_status st = launches();
                p.stream = own;
                const hipError_t e = hipStreamEndCapture(cs, &g);
                if (st == DGPE_OK && e == hipSuccess && g &&
                    hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess)
                    eager = false;
                else
                    exec = nullptr;
            }
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
        }
        if (exec) {
            DGPE_HIP(hipGraphLaunch(exec, p.stream));
            return DGPE_OK;
        }
        return launches();
    }
};

extern "C" {

const char* dgpe_status_string(dgpe_status s) {
    switch (s) {
        case DGPE_OK: return "DGPE_OK";
        case DGPE_EINVAL: return "DGPE_EINVAL";
        case DGPE_EUNSUPPORTED_SIZE: return "DGPE_EUNSUPPORTED_SIZE";
        case DGPE_EWORKSPACE: return "DGPE_EWORKSPACE";
        case DGPE_EHIP: return "DGPE_EHIP";
        case DGPE_ENONFINITE: return "DGPE_ENONFINITE";
        case DGPE_ESTATE: return "DGPE_ESTATE";
    }
    return "DGPE_UNKNOWN";
}

const char* dgpe_last_error(void) { return g_last_error.c_str(); }

size_t dgpe_workspace_bytes(const int32_t n[3], uint32_t mode) {
    if (!n) return 0;
    int nn[3] = {n[0], n[1], n[2]};
    if (mode & ~(DGPE_REAL | DGPE_F32 | DGPE_Q2D_PERP | DGPE_Q2D_INPLANE)) return 0;
    if ((mode & DGPE_Q2D_PERP) && (mode & DGPE_Q2D_INPLANE)) return 0;
    if (!grid_ok(n, mode)) return 0;
    size_t offs[OFF_END + 1];
    if (!layout(nn, (mode & DGPE_F32) != 0, offs, nullptr)) return 0;
    return offs[OFF_END];
}

dgpe_status dgpe_plan_create(dgpe_plan* out, const int32_t n[3], const double d[3], double dt,
                             const double trap[3], double g, double gd, double cutoff_R,
                             uint32_t mode, void* workspace, size_t workspace_bytes,
                             void* hip_stream) {
    if (!out) return fail(DGPE_EINVAL, "out is NULL");
    *out = nullptr;
    dgpe_status st = check_plan_args(n, d, dt, trap, g, gd, cutoff_R, mode);
    if (st != DGPE_OK) return st;
    return create_plan(out, n, d, dt, trap, g, gd, cutoff_R, mode, workspace, workspace_bytes,
                       (hipStream_t)hip_stream, false);
}

dgpe_status dgpe_plan_create_noalloc(dgpe_plan* out, const int32_t n[3], const double d[3],
                                     double dt, const double trap[3], double g, double gd,
                                     double cutoff_R, uint32_t mode, void* hip_stream) {
    if (!out) return fail(DGPE_EINVAL, "out is NULL");
    *out = nullptr;
    dgpe_status st = check_plan_args(n, d, dt, trap, g, gd, cutoff_R, mode);
    if (st != DGPE_OK) return st;
    const size_t need = dgpe_workspace_bytes(n, mode);
    if (need > DGPE_NOALLOC_MAX_BYTES)
        return fail(DGPE_EWORKSPACE, "grid needs " + std::to_string(need) +
                                         " bytes of workspace; the allocation-free plan holds at most " +
                                         std::to_string((size_t)DGPE_NOALLOC_MAX_BYTES));
    int dev = -1;
    DGPE_HIP(hipGetDevice(&dev));
    void* ws = nullptr;
    if ((st = scratch_for_device(dev, &ws)) != DGPE_OK) return st;
    // every plan created here before on this device is superseded from now on
    g_scratch_gen[dev].fetch_add(1);
    return create_plan(out, n, d, dt, trap, g, gd, cutoff_R, mode, ws, DGPE_NOALLOC_MAX_BYTES,
                       (hipStream_t)hip_stream, true);
}

dgpe_status dgpe_plan_set(dgpe_plan plan, int32_t param, double value) {
    if (!plan) return fail(DGPE_EINVAL, "plan is NULL");
    if (plan_live(*plan) != DGPE_OK) return DGPE_ESTATE;
    if (!std::isfinite(value)) return fail(DGPE_EINVAL, "value must be finite");
    Plan& p = *plan;
    switch (param) {
        case DGPE_PARAM_G:
            p.g_in = value;
            p.g = contact_coupling(p);
            return DGPE_OK;
        case DGPE_PARAM_GD: p.gd = value; return DGPE_OK;
        case DGPE_PARAM_TRAP_NU: p.trap[0] = value; return DGPE_OK;
        case DGPE_PARAM_TRAP_LAMBDA:
            if (!p.q2d) {
                p.trap[1] = value;
                return DGPE_OK;
            }
            // quasi-2D: the tight axis sets the contact coupling and the kernel
            if (!(value > 0)) return fail(DGPE_EINVAL, "the tight trap frequency must be > 0");
            p.trap[1] = value;
            p.g = contact_coupling(p);
            DGPE_HIP(hipStreamSynchronize(p.stream));
            DGPE_HIP(p.f32 ? launch_ukern<float>(p) : launch_ukern<double>(p));
            DGPE_HIP(hipStreamSynchronize(p.stream));
            return DGPE_OK;
        case DGPE_PARAM_TRAP_GAMMA: p.trap[2] = value; return DGPE_OK;
        case DGPE_PARAM_FAST_FFT:
            if (value != 0.0 && value != 1.0) return fail(DGPE_EINVAL, "FAST_FFT takes 0 or 1");
            p.fast = value == 1.0;
            return DGPE_OK;
        case DGPE_PARAM_FUSED_Y:
            if (value != 0.0 && value != 1.0) return fail(DGPE_EINVAL, "FUSED_Y takes 0 or 1");
            p.fuse_y = value == 1.0;
            return DGPE_OK;
        case DGPE_PARAM_SCHEME:
            if (value != 0.0 && value != 1.0) return fail(DGPE_EINVAL, "SCHEME takes 0 or 1");
            if (value == 1.0 && p.q2d)
                return fail(DGPE_ESTATE, "the symmetric step is for three-dimensional plans");
            p.scheme = (int)value;
            return DGPE_OK;
        case DGPE_PARAM_DT:
            if (!(value > 0)) return fail(DGPE_EINVAL, "dt must be > 0");
            p.dt = value;
            p.dt_nl = value;
            break;
        case DGPE_PARAM_REAL_TIME: {
            if (value != 0.0 && value != 1.0) return fail(DGPE_EINVAL, "REAL_TIME takes 0 or 1");
            Launch lc{};
            if (!choose_launch(p.n, p.f32, value == 0.0, &lc))
                return fail(DGPE_EUNSUPPORTED_SIZE, "no launch shape for this mode");
            p.imag = value == 0.0;
            p.lc = lc;
            break;
        }
        default: return fail(DGPE_EINVAL, "unknown parameter");
    }
    DGPE_HIP(hipStreamSynchronize(p.stream));
    return p.f32 ? build_cn_tables<float>(p) : build_cn_tables<double>(p);
}

dgpe_status dgpe_plan_set_stream(dgpe_plan plan, void* hip_stream) {
    if (!plan) return fail(DGPE_EINVAL, "plan is NULL");
    plan->stream = (hipStream_t)hip_stream;
    return DGPE_OK;
}

int32_t dgpe_plan_fused_y(dgpe_plan plan) {
    if (!plan) return -1;
    return fused_y(*plan) ? 1 : 0;
}

dgpe_status dgpe_step(dgpe_plan plan, void* psi, int32_t nsteps, const double* amp) {
    if (!plan) return fail(DGPE_EINVAL, "plan is NULL");
    if (plan_live(*plan) != DGPE_OK) return DGPE_ESTATE;
    dgpe_status st = check_ptr(psi, "psi");
    if (st != DGPE_OK) return st;
    if (nsteps < 0) return fail(DGPE_EINVAL, "nsteps must be >= 0");
    if (amp)
        for (int i = 0; i < nsteps; ++i)
            if (!std::isfinite(amp[i])) return fail(DGPE_EINVAL, "amp must be finite");
    return plan->f32 ? run_steps<float>(*plan, psi, nsteps, amp)
                     : run_steps<double>(*plan, psi, nsteps, amp);
}

dgpe_status dgpe_ground_state(dgpe_plan plan, void* psi, double tol, int32_t max_steps,
                              int32_t check_every, int32_t* steps_done, double* dmu_per_step,
                              dgpe_obs* obs) {
    if (!plan) return fail(DGPE_EINVAL, "plan is NULL");
    if (plan_live(*plan) != DGPE_OK) return DGPE_ESTATE;
    dgpe_status st = check_ptr(psi, "psi");
    if (st != DGPE_OK) return st;
    if (!steps_done || !dmu_per_step || !obs)
        return fail(DGPE_EINVAL, "steps_done, dmu_per_step and obs must be non-NULL");
    if (!(tol > 0) || !std::isfinite(tol)) return fail(DGPE_EINVAL, "tol must be finite and > 0");
    if (max_steps < 0 || check_every < 1)
        return fail(DGPE_EINVAL, "max_steps must be >= 0 and check_every >= 1");
    Plan& p = *plan;
    if (!p.imag) return fail(DGPE_ESTATE, "the ground state needs an imaginary-time plan");
    auto obs_of = [&](dgpe_obs* o) {
        return p.f32 ? observables_impl<float>(p, psi, 1.0, o) : observables_impl<double>(p, psi, 1.0, o);
    };
    dgpe_obs o{};
    if ((st = obs_of(&o)) != DGPE_OK) return st;
    double mu = o.mu, rate = INFINITY;
    int done = 0;
    auto steps = [&](int k) {
        return p.f32 ? run_steps<float>(p, psi, k, nullptr) : run_steps<double>(p, psi, k, nullptr);
    };
    // The check_every steps between two checks are the same launches every
    // time (same buffers and parameters): captured once as a HIP graph and
    // replayed, they reach the GPU without one host launch per kernel.  If
    // the capture fails the steps run as plain launches.
    ChunkGraph chunk(p);
    while (done < max_steps) {
        const int k = std::min(check_every, max_steps - done);
        if (k == check_every) st = chunk.run([&] { return steps(k); });
        else st = steps(k);
        if (st != DGPE_OK) return st;
        done += k;
        if ((st = obs_of(&o)) != DGPE_OK) return st;
        rate = std::fabs(o.mu - mu) / k;
        mu = o.mu;
        if (rate < tol) break;
    }
    *steps_done = done;
    *dmu_per_step = rate;
    *obs = o;
    return DGPE_OK;
}

dgpe_status dgpe_density(dgpe_plan plan, const void* psi, void* out) {
    if (!plan) return fail(DGPE_EINVAL, "plan is NULL");
    if (plan_live(*plan) != DGPE_OK) return DGPE_ESTATE;
    dgpe_status st = check_ptr(psi, "psi");
    if (st != DGPE_OK) return st;
    if ((st = check_ptr(out, "out")) != DGPE_OK) return st;
    DGPE_HIP(plan->f32 ? launch_density<float>(*plan, psi, out) : launch_density<double>(*plan, psi, out));
    return DGPE_OK;
}

dgpe_status dgpe_write_density(dgpe_plan plan, const void* psi, const char* path) {
    if (!plan || !path) return fail(DGPE_EINVAL, "plan and path must be non-NULL");
    if (plan_live(*plan) != DGPE_OK) return DGPE_ESTATE;
    dgpe_status st = check_ptr(psi, "psi");
    if (st != DGPE_OK) return st;
    Plan& p = *plan;
    const size_t rsz = p.f32 ? 4 : 8;
    // the density of the whole grid in the Phi buffer, then x-planes to the
    // host through a bounded buffer, widened to FP64 and appended in order
    DGPE_HIP(p.f32 ? launch_density<float>(p, psi, p.phi) : launch_density<double>(p, psi, p.phi));
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(DGPE_EINVAL, std::string("cannot open ") + path + " for writing");
    const size_t plane = (size_t)p.n[1] * p.n[2];
    const size_t chunk_planes = std::max<size_t>(1, ((size_t)8 << 20) / (plane * rsz));
    std::vector<unsigned char> raw(chunk_planes * plane * rsz);
    std::vector<double> wide(chunk_planes * plane);
    for (size_t x0 = 0; x0 < (size_t)p.n[0]; x0 += chunk_planes) {
        const size_t np = std::min(chunk_planes, (size_t)p.n[0] - x0);
        const size_t cnt = np * plane;
        hipError_t e = hipMemcpyAsync(raw.data(), (const char*)p.phi + x0 * plane * rsz, cnt * rsz,
                                      hipMemcpyDeviceToHost, p.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
        if (e != hipSuccess) {
            std::fclose(f);
            return fail(DGPE_EHIP, std::string("density download: ") + hipGetErrorString(e));
        }
        for (size_t i = 0; i < cnt; ++i) {
            if (p.f32) {
                float v;
                std::memcpy(&v, raw.data() + i * 4, 4);
                wide[i] = v;
            } else {
                std::memcpy(&wide[i], raw.data() + i * 8, 8);
            }
        }
        if (std::fwrite(wide.data(), sizeof(double), cnt, f) != cnt) {
            std::fclose(f);
            return fail(DGPE_EINVAL, std::string("short write to ") + path);
        }
    }
    if (std::fclose(f) != 0) return fail(DGPE_EINVAL, std::string("cannot close ") + path);
    return DGPE_OK;
}

dgpe_status dgpe_potential(dgpe_plan plan, const void* psi, void* phi) {
    if (!plan) return fail(DGPE_EINVAL, "plan is NULL");
    if (plan_live(*plan) != DGPE_OK) return DGPE_ESTATE;
    dgpe_status st = check_ptr(psi, "psi");
    if (st != DGPE_OK) return st;
    if ((st = check_ptr(phi, "phi")) != DGPE_OK) return st;
    Plan& p = *plan;
    if (p.f32) {
        if ((st = convolve_density<float>(p, psi, nullptr)) != DGPE_OK) return st;
        DGPE_HIP(launch_c2r_phi<float>(p, phi));
    } else {
        if ((st = convolve_density<double>(p, psi, nullptr)) != DGPE_OK) return st;
        DGPE_HIP(launch_c2r_phi<double>(p, phi));
    }
    return DGPE_OK;
}

dgpe_status dgpe_energy_mu_rms(dgpe_plan plan, const void* psi, double amp, dgpe_obs* out) {
    if (!plan || !out) return fail(DGPE_EINVAL, "plan and out must be non-NULL");
    if (plan_live(*plan) != DGPE_OK) return DGPE_ESTATE;
    dgpe_status st = check_ptr(psi, "psi");
    if (st != DGPE_OK) return st;
    if (!std::isfinite(amp)) return fail(DGPE_EINVAL, "amp must be finite");
    return plan->f32 ? observables_impl<float>(*plan, psi, amp, out)
                     : observables_impl<double>(*plan, psi, amp, out);
}

size_t dgpe_adjoint_workspace_bytes(dgpe_plan plan, int32_t nsteps, int32_t ckpt_every) {
    if (!plan || nsteps < 1 || ckpt_every < 1) return 0;
    return adj_layout(*plan, nsteps, std::min(ckpt_every, nsteps)).end;
}

dgpe_status dgpe_step_adjoint(dgpe_plan plan, const void* psi0, int32_t nsteps, const double* amp,
                              int32_t ckpt_every, int32_t objective, const void* target,
                              void* adj_ws, size_t adj_ws_bytes, void* psi_final, double* J,
                              double* dJ_damp, double dJ_dtrap[3], void* dJ_dpsi0) {
    if (!plan) return fail(DGPE_EINVAL, "plan is NULL");
    if (plan_live(*plan) != DGPE_OK) return DGPE_ESTATE;
    Plan& p = *plan;
    if (p.imag) return fail(DGPE_ESTATE, "the adjoint needs a real-time plan");
    if (p.scheme != 0) return fail(DGPE_ESTATE, "the adjoint is that of the first-order step");
    if (p.q2d) return fail(DGPE_ESTATE, "the adjoint is that of the three-dimensional step");
    if (nsteps < 1 || ckpt_every < 1) return fail(DGPE_EINVAL, "nsteps and ckpt_every must be >= 1");
    if (!amp || !J || !dJ_damp || !dJ_dtrap) return fail(DGPE_EINVAL, "amp, J, dJ_damp, dJ_dtrap required");
    for (int i = 0; i <= nsteps; ++i)
        if (!std::isfinite(amp[i])) return fail(DGPE_EINVAL, "amp must be finite");
    if (objective != DGPE_OBJ_ENERGY && objective != DGPE_OBJ_OVERLAP)
        return fail(DGPE_EINVAL, "unknown objective");
    dgpe_status st = check_ptr(psi0, "psi0");
    if (st != DGPE_OK) return st;
    if (objective == DGPE_OBJ_OVERLAP && (st = check_ptr(target, "target")) != DGPE_OK) return st;
    if (psi_final && (st = check_ptr(psi_final, "psi_final")) != DGPE_OK) return st;
    if (dJ_dpsi0 && (st = check_ptr(dJ_dpsi0, "dJ_dpsi0")) != DGPE_OK) return st;
    const int K = std::min(ckpt_every, nsteps);
    if ((st = check_ptr(adj_ws, "adj_ws")) != DGPE_OK) return fail(DGPE_EWORKSPACE, dgpe_last_error());
    if (adj_ws_bytes < adj_layout(p, nsteps, K).end)
        return fail(DGPE_EWORKSPACE, "adjoint workspace too small");
    return p.f32 ? adjoint_impl<float>(p, psi0, nsteps, amp, K, objective, target, (char*)adj_ws,
                                       psi_final, J, dJ_damp, dJ_dtrap, dJ_dpsi0)
                 : adjoint_impl<double>(p, psi0, nsteps, amp, K, objective, target, (char*)adj_ws,
                                        psi_final, J, dJ_damp, dJ_dtrap, dJ_dpsi0);
}

dgpe_status dgpe_pass_bytes(dgpe_plan plan, double bytes[DGPE_NPASS]) {
    if (!plan || !bytes) return fail(DGPE_EINVAL, "plan and bytes must be non-NULL");
    pass_bytes(*plan, bytes);
    return DGPE_OK;
}

dgpe_status dgpe_step_profiled(dgpe_plan plan, void* psi, int32_t nsteps, const double* amp,
                               double ms[DGPE_NPASS], double* total_ms) {
    if (!plan || !ms) return fail(DGPE_EINVAL, "plan and ms must be non-NULL");
    if (plan_live(*plan) != DGPE_OK) return DGPE_ESTATE;
    dgpe_status st = check_ptr(psi, "psi");
    if (st != DGPE_OK) return st;
    if (nsteps < 0) return fail(DGPE_EINVAL, "nsteps must be >= 0");
    if (amp)
        for (int i = 0; i < nsteps; ++i)
            if (!std::isfinite(amp[i])) return fail(DGPE_EINVAL, "amp must be finite");
    Plan& p = *plan;
    PassTimer tm;  // owns every event it records, including the call's own pair
    tm.on = true;
    tm.stream = p.stream;
    DGPE_HIP(tm.begin(-1));  // the whole call
    const size_t whole = tm.ev.size() - 2;
    st = p.f32 ? run_steps<float>(p, psi, nsteps, amp, &tm) : run_steps<double>(p, psi, nsteps, amp, &tm);
    if (st != DGPE_OK) return st;
    DGPE_HIP(hipEventRecord(tm.ev[whole + 1], p.stream));
    DGPE_HIP(hipStreamSynchronize(p.stream));
    double sum[DGPE_NPASS] = {0};
    int cnt[DGPE_NPASS] = {0};
    for (size_t i = 0; i < tm.kind.size(); ++i) {
        if (tm.kind[i] < 0) continue;
        float m = 0.f;
        DGPE_HIP(hipEventElapsedTime(&m, tm.ev[2 * i], tm.ev[2 * i + 1]));
        sum[tm.kind[i]] += m;
        cnt[tm.kind[i]] += 1;
    }
    for (int k = 0; k < DGPE_NPASS; ++k) ms[k] = cnt[k] ? sum[k] / cnt[k] : 0.0;
    if (total_ms) {
        float m = 0.f;
        DGPE_HIP(hipEventElapsedTime(&m, tm.ev[whole], tm.ev[whole + 1]));
        *total_ms = m;
    }
    return DGPE_OK;
}

void dgpe_plan_destroy(dgpe_plan plan) { delete plan; }

}  // extern "C"
