// Fast spectral passes: the two-factor register FFT (fft_reg.h) for the
// lengths L = R1 R2 listed in fast_split().  Each pass reads and writes HBM
// once with coalesced accesses and exchanges data through LDS once per
// transform (the generic Stockham kernels in k_spectral.hip cover every
// other length).  Same results as the generic passes up to rounding order.
#include "fft_reg.h"

namespace dgpe {

namespace {

// elements of one block's tile: 4096 complex in FP32, 2048 in FP64
template <typename T>
constexpr int tile_budget() { return sizeof(T) == 4 ? 4096 : 2048; }

template <typename T, int R1, int L>
constexpr int rows_per_block() {
    int nb = 32;
    while (nb > 1 && (nb * L > tile_budget<T>() || nb * R1 > 256)) nb >>= 1;
    return nb;
}

// Columns per block of the x pass: as rows_per_block for lines shorter than
// 384 points; longer lines take up to 64 KB of LDS and 512 threads, so that
// each row of the block's tile is a run of at least 128 bytes (8 columns,
// 64-byte runs, held the 512-point pass to half the HBM bandwidth; 32
// columns, 128 KB, one block per CU, were slower still: 185 against 135 us
// at 512 x 512 x 256).
template <typename T, int R1, int L>
constexpr int xmul_cols() {
    if (L < 384) return rows_per_block<T, R1, L>();
    int nb = 32;
    while (nb > 1 && (nb * L * 2 * (int)sizeof(T) > 64 * 1024 || nb * R1 > 512)) nb >>= 1;
    return nb;
}

// ---------------------------------------------------------------------------
// P2 / P4: FFT along contiguous rows of length L = R1 R2 (the y axis of S).
// Lanes: t fastest (t < R1 threads per row), NB rows per block.
// With npart (imaginary time), block 0 also turns the previous x sweep's norm
// partials into sigma = 1 / (sum dV) after its rows, for the fused z pass of
// this step: the reduction then needs no launch of its own.
// ---------------------------------------------------------------------------
template <typename T, int R1, int R2, bool INV>
__global__ void __launch_bounds__((rows_per_block<T, R1, R1 * R2>() * R1))
    k_rows2(cx<T>* __restrict__ spec, int nrows, const cx<T>* __restrict__ tw,
            const double* __restrict__ npart, int nnpart, double dV, double* __restrict__ sigma_out) {
    constexpr int L = R1 * R2;
    constexpr int NB = rows_per_block<T, R1, L>();
    constexpr int SB = R2 * (R1 + 1);
    __shared__ cx<T> xb[NB * SB];
    __shared__ cx<T> stw[L];
    const int tid = threadIdx.x;
    const int t = tid % R1, b = tid / R1;
    const int row = blockIdx.x * NB + b;
    const bool ok = row < nrows;
    // twiddles, then the rows (rows past the end read the last row, unused):
    // every load in flight before the first wait
    TabRegs<cx<T>, L, NB * R1> rtw;
    tab_issue(rtw, tw, tid);
    cx<T>* base = spec + (size_t)min(row, nrows - 1) * L;
    cx<T> v[R2];
#pragma unroll
    for (int n = 0; n < R2; ++n) v[n] = base[t + R1 * n];
    tab_stage(rtw, stw, tid, [](int i) { return i; });
    __syncthreads();
    if (ok) {
        rdft<T, R2, INV>(v);
        twiddle_phase<T, R2, INV>(v, t, stw);
#pragma unroll
        for (int k = 0; k < R2; ++k) xb[b * SB + k * (R1 + 1) + t] = v[k];
    }
    __syncthreads();
    if (ok && t < R2) {
        cx<T> w[R1];
#pragma unroll
        for (int n = 0; n < R1; ++n) w[n] = xb[b * SB + t * (R1 + 1) + n];
        rdft<T, R1, INV>(w);
#pragma unroll
        for (int k = 0; k < R1; ++k) base[t + R2 * k] = w[k];
    }
    if (npart && blockIdx.x == 0) {  // block-uniform
        __shared__ double sred[(rows_per_block<T, R1, L>() * R1 + 63) / 64];
        const double sum = block_sum_partials(npart, nnpart, sred);
        if (tid == 0) sigma_out[0] = 1.0 / (sum * dV);
    }
}

// ---------------------------------------------------------------------------
// P3: FFT along x (stride Ny) of NB adjacent columns at one kz, multiply by
// U_R/Nt (table [kz][|kx|][|ky|]: each entry read by the blocks of ky and
// Ny - ky, which run together on one XCD), inverse FFT along x.
// Lanes: b fastest (NB columns), t < R1 threads per column.
// ---------------------------------------------------------------------------
template <typename T, int R1, int R2>
__global__ void __launch_bounds__((xmul_cols<T, R1, R1 * R2>() * R1))
    k_xmul2(cx<T>* __restrict__ spec, int Ny, const cx<T>* __restrict__ tw,
            const T* __restrict__ ukern) {
    constexpr int L = R1 * R2;  // Nx
    constexpr int NB = xmul_cols<T, R1, L>();
    constexpr int NT = NB * R1;
    __shared__ cx<T> xb[NB * L];
    __shared__ cx<T> stw[L];
    const int tid = threadIdx.x;
    const int b = tid % NB, t = tid / NB;
    const int ngy = Ny / NB;
    const int bid = xcd_swizzle(blockIdx.x, gridDim.x);
    const int kz = bid / ngy;
    const int y0 = (bid - kz * ngy) * NB;
    // twiddles, the spectrum columns and the kernel values, all in flight
    // before the first wait
    TabRegs<cx<T>, L, NT> rtw;
    tab_issue(rtw, tw, tid);
    cx<T>* base = spec + (size_t)kz * L * Ny + y0 + b;
    cx<T> v[R2];
#pragma unroll
    for (int n = 0; n < R2; ++n) v[n] = base[(size_t)(t + R1 * n) * Ny];
    // after the forward FFT thread t < R2 holds X[kx = t + R2 k]; the kernel is
    // even in kx and ky: table [kz][|kx|][|ky|] (threads t >= R2 read t =
    // R2 - 1's)
    const int hy = Ny / 2 + 1;
    const T* ucol = ukern + (size_t)kz * (L / 2 + 1) * hy + min(y0 + b, Ny - y0 - b);
    T uk[R1];
#pragma unroll
    for (int k = 0; k < R1; ++k) {
        const int kx0 = min(t, R2 - 1) + R2 * k;
        uk[k] = ucol[(size_t)min(kx0, L - kx0) * hy];
    }
    tab_stage(rtw, stw, tid, [](int i) { return i; });
    __syncthreads();
    rdft<T, R2, false>(v);
    twiddle_phase<T, R2, false>(v, t, stw);
#pragma unroll
    for (int k = 0; k < R2; ++k) xb[(k * R1 + t) * NB + b] = v[k];
    __syncthreads();
    cx<T> w[R1];
    if (t < R2) {
#pragma unroll
        for (int n = 0; n < R1; ++n) w[n] = xb[(t * R1 + n) * NB + b];
        rdft<T, R1, false>(w);
#pragma unroll
        for (int k = 0; k < R1; ++k) w[k] = uk[k] * w[k];
        // inverse: the layout of w is the phase-A layout of the (R2, R1) split
        rdft<T, R1, true>(w);
        twiddle_phase<T, R1, true>(w, t, stw);
    }
    __syncthreads();
    if (t < R2) {
#pragma unroll
        for (int j = 0; j < R1; ++j) xb[(j * R2 + t) * NB + b] = w[j];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < R2; ++u) v[u] = xb[(t * R2 + u) * NB + b];
    rdft<T, R2, true>(v);
#pragma unroll
    for (int l = 0; l < R2; ++l) base[(size_t)(t + R1 * l) * Ny] = v[l];
}

// P3 for long lines with R1 = 2 R2 (the 512-point split 32 x 16): as k_xmul2,
// but the size-R1 DFTs of phase B are split over the lane pair (t, t ^ 1):
// lane h = t & 1 of group g = t >> 1 (the phase-B index k2) transforms the
// R1/2 values with n1 = h + 2m, and one radix-2 step across the pair (wave
// shuffles: the pair is NB lanes apart in one wave) joins them,
//   X[k] = E[k] + W_R1^k O[k],  X[k + R1/2] = E[k] - W_R1^k O[k]
// (E from the even n1, O from the odd ones).  The inverse undoes it in the
// opposite order: E'[k] = X[k] + X[k + R1/2], O'[k] = (X[k] - X[k + R1/2])
// W_R1^-k, then inverse DFTs of size R1/2.  Every thread then works in both
// phases with R1/2 = R2 values, which keeps 16-column tiles (128-byte runs)
// at four waves per SIMD.
template <typename T, int R1, int R2>
__global__ void __launch_bounds__((xmul_cols<T, R1, R1 * R2>() * R1))
    k_xmul2s(cx<T>* __restrict__ spec, int Ny, const cx<T>* __restrict__ tw,
             const T* __restrict__ ukern) {
    static_assert(R1 == 2 * R2, "the pair split needs R1 = 2 R2");
    constexpr int L = R1 * R2;  // Nx
    constexpr int NB = xmul_cols<T, R1, L>();
    static_assert(NB <= 32, "lane pairs must share a wave");
    constexpr int NT = NB * R1;
    constexpr int H = R1 / 2;
    __shared__ cx<T> xb[NB * L];
    __shared__ cx<T> stw[L];
    const int tid = threadIdx.x;
    const int b = tid % NB, t = tid / NB;
    const int g = t >> 1, h = t & 1;
    const int ngy = Ny / NB;
    const int bid = xcd_swizzle(blockIdx.x, gridDim.x);
    const int kz = bid / ngy;
    const int y0 = (bid - kz * ngy) * NB;
    TabRegs<cx<T>, L, NT> rtw;
    tab_issue(rtw, tw, tid);
    cx<T>* base = spec + (size_t)kz * L * Ny + y0 + b;
    cx<T> v[R2];
#pragma unroll
    for (int n = 0; n < R2; ++n) v[n] = base[(size_t)(t + R1 * n) * Ny];
    // this lane's outputs of phase B are X[kx = g + R2 (k + H h)], k < H
    const int hy = Ny / 2 + 1;
    const T* ucol = ukern + (size_t)kz * (L / 2 + 1) * hy + min(y0 + b, Ny - y0 - b);
    T uk[H];
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const int kx = g + R2 * (k + H * h);
        uk[k] = ucol[(size_t)min(kx, L - kx) * hy];
    }
    tab_stage(rtw, stw, tid, [](int i) { return i; });
    __syncthreads();
    // phase A: DFT over n2 of x[t + R1 n2], twiddle W_L^{t k2}
    rdft<T, R2, false>(v);
    twiddle_phase<T, R2, false>(v, t, stw);
#pragma unroll
    for (int k = 0; k < R2; ++k) xb[(k * R1 + t) * NB + b] = v[k];
    __syncthreads();
    // phase B, half h of group g: DFT of size H over n1 = h + 2m
    cx<T> w[H];
#pragma unroll
    for (int m = 0; m < H; ++m) w[m] = xb[(g * R1 + h + 2 * m) * NB + b];
    rdft<T, H, false>(w);
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const cx<T> q = {__shfl_xor(w[k].x, NB), __shfl_xor(w[k].y, NB)};
        const cx<T> e = h ? q : w[k];
        const cx<T> o = cmul(h ? w[k] : q, ctw<T, R1, false>(k));
        const cx<T> x = h ? e - o : e + o;
        // multiply by U_R / Nt
        w[k] = uk[k] * x;
    }
    // inverse of the pair step, then inverse DFTs of size H
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const cx<T> q = {__shfl_xor(w[k].x, NB), __shfl_xor(w[k].y, NB)};
        w[k] = h ? cmul(q - w[k], ctw<T, R1, true>(k)) : w[k] + q;
    }
    rdft<T, H, true>(w);
    __syncthreads();  // every lane has read its phase-A values
#pragma unroll
    for (int m = 0; m < H; ++m) {
        const int n1 = h + 2 * m;
        xb[(g * R1 + n1) * NB + b] = cmulc(w[m], stw[n1 * g]);
    }
    __syncthreads();
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) v[k2] = xb[(k2 * R1 + t) * NB + b];
    rdft<T, R2, true>(v);
#pragma unroll
    for (int l = 0; l < R2; ++l) base[(size_t)(t + R1 * l) * Ny] = v[l];
}

// packed real-to-complex post-processing (see k_spectral.hip)
template <typename T>
__device__ __forceinline__ cx<T> r2c_post2(cx<T> zk, cx<T> zm, cx<T> w) {
    const T h = T(0.5);
    const cx<T> E = {h * (zk.x + zm.x), h * (zk.y - zm.y)};
    const cx<T> O = {h * (zk.y + zm.y), -h * (zk.x - zm.x)};
    return E + cmul(w, O);
}

// ---------------------------------------------------------------------------
// P1: density |psi|^2 sigma of NB z-lines packed as z_j = n_{2j} + i n_{2j+1},
// FFT of length M = Nz/2 = R1 R2, post-processing into the half spectrum,
// kz-major store.  Lanes: t fastest.
// ---------------------------------------------------------------------------
// Physics of the pointwise steps (trap half-widths, spacings, trap_a^2 / 2)
struct Phys2 {
    double dt, g, gd, amp;
    int imag;
    int hx, hy, hz;
    double dx, dy, dz, cx, cy, cz;
};

// Constants of the fused z pass's nonlinear exponent, folded on the host:
// th = kx ix^2 + ky iy^2 + kz iz^2 + kg sigma |psi|^2 + kd Phi with (ix, iy, iz)
// the grid offsets from the trap centre, i.e. dt (a V + g sigma |psi|^2 +
// g_d Phi); all times log2(e) for the FP32 imaginary-time factor (taken as exp2)
struct NlConst {
    double kx, ky, kz, kg, kd;
};

// ADJ: the transformed real field is the adjoint source
// s = Im(conj(mu) e^{-i theta} psi_n), theta = dt (a V0 + g |psi_n|^2 + g_d Phi_n)
// (psi holds mu), with the FP64 block sums of s V0, s x^2, s y^2, s z^2 in
// partials[4 * block + q].
template <typename T, int R1, int R2, bool ADJ>
__global__ void __launch_bounds__((rows_per_block<T, R1, R1 * R2>() * R1))
    k_r2c2(const cx<T>* __restrict__ psi, cx<T>* __restrict__ spec, int Nx, int Ny,
           const cx<T>* __restrict__ twz, const cx<T>* __restrict__ twr2c,
           const double* __restrict__ sigma, const cx<T>* __restrict__ psin,
           const T* __restrict__ phin, Phys2 ph, double* __restrict__ partials) {
    constexpr int M = R1 * R2;
    constexpr int NB = rows_per_block<T, R1, M>();
    constexpr int NT = NB * R1;
    // >= M + 1; odd, so that the post-processing reads (line fastest) spread
    // over the banks
    constexpr int SB = R2 * (R1 + 1) + 1;
    __shared__ cx<T> xb[NB * SB];
    __shared__ cx<T> stw[M];
    __shared__ cx<T> sr2c[M + 1];
    const int tid = threadIdx.x;
    const int t = tid % R1, b = tid / R1;
    const int ngy = Ny / NB;
    const int bid = xcd_swizzle(blockIdx.x, gridDim.x);
    const int x = bid / ngy;
    const int y0 = (bid - x * ngy) * NB;
    const size_t line0 = (size_t)x * Ny + y0;
    // twiddles, then the state: every load in flight before the first wait
    TabRegs<cx<T>, M, NT> rtw;
    TabRegs<cx<T>, M + 1, NT> rr2;
    tab_issue(rtw, twz, tid);
    tab_issue(rr2, twr2c, tid);
    const cx<T>* base = psi + (line0 + b) * (2 * M);
    cx<T> pa[R2], pc[R2];
    cx<T> qa[ADJ ? R2 : 1], qc[ADJ ? R2 : 1];
    T fa[ADJ ? R2 : 1], fc[ADJ ? R2 : 1];
#pragma unroll
    for (int n = 0; n < R2; ++n) {
        const int j = t + R1 * n;
        pa[n] = base[2 * j];
        pc[n] = base[2 * j + 1];
        if constexpr (ADJ) {
            const size_t o = (line0 + b) * (2 * M) + 2 * j;
            qa[n] = psin[o];
            qc[n] = psin[o + 1];
            fa[n] = phin[o];
            fc[n] = phin[o + 1];
        }
    }
    tab_stage(rtw, stw, tid, [](int i) { return i; });
    tab_stage(rr2, sr2c, tid, [](int i) { return i; });
    cx<T> v[R2];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (!ADJ) {
        const T sig = sigma ? T(sigma[0]) : T(1);
#pragma unroll
        for (int n = 0; n < R2; ++n) v[n] = cx<T>{abs2(pa[n]) * sig, abs2(pc[n]) * sig};
    } else {
        const T dt = T(ph.dt), gg = T(ph.g), gdd = T(ph.gd), amp = T(ph.amp);
        const T xx = T(x - ph.hx) * T(ph.dx), yy = T(y0 + b - ph.hy) * T(ph.dy);
        const T vxy = T(ph.cx) * xx * xx + T(ph.cy) * yy * yy;
        const double x2 = double(x - ph.hx) * ph.dx * (double(x - ph.hx) * ph.dx);
        const double y2 = double(y0 + b - ph.hy) * ph.dy * (double(y0 + b - ph.hy) * ph.dy);
        auto source = [&](cx<T> m, cx<T> pn, T phi, int iz) {
            const T z = T(iz - ph.hz) * T(ph.dz);
            const T v0 = vxy + T(ph.cz) * z * z;
            const T th = dt * (amp * v0 + gg * abs2(pn) + gdd * phi);
            T sn, cs;
            sin_cos(th, &sn, &cs);
            const cx<T> pp = {pn.x * cs + pn.y * sn, pn.y * cs - pn.x * sn};
            const T sv = m.x * pp.y - m.y * pp.x;  // Im(conj(m) pp)
            const double zd = double(iz - ph.hz) * ph.dz;
            acc[0] += double(sv) * double(v0);
            acc[1] += double(sv) * x2;
            acc[2] += double(sv) * y2;
            acc[3] += double(sv) * zd * zd;
            return sv;
        };
#pragma unroll
        for (int n = 0; n < R2; ++n) {
            const int j = t + R1 * n;
            v[n] = cx<T>{source(pa[n], qa[n], fa[n], 2 * j), source(pc[n], qc[n], fc[n], 2 * j + 1)};
        }
    }
    __syncthreads();
    rdft<T, R2, false>(v);
    twiddle_phase<T, R2, false>(v, t, stw);
#pragma unroll
    for (int k = 0; k < R2; ++k) xb[b * SB + k * (R1 + 1) + t] = v[k];
    __syncthreads();
    cx<T> w[R1];
    if (t < R2) {
#pragma unroll
        for (int n = 0; n < R1; ++n) w[n] = xb[b * SB + t * (R1 + 1) + n];
        rdft<T, R1, false>(w);
    }
    __syncthreads();
    if (t < R2) {
#pragma unroll
        for (int k = 0; k < R1; ++k) xb[b * SB + t + R2 * k] = w[k];  // Z in natural order
    }
    __syncthreads();
    const size_t plane = (size_t)Nx * Ny;
    // two adjacent lines per thread and row: 16-byte stores in FP32
    constexpr int P = sizeof(T) == 4 ? 2 : 1;
    constexpr int NPB = NB / P;
    static_assert(NB % P == 0, "pairs of lines");
    for (int g = tid; g < (M + 1) * NPB; g += NT) {
        const int k = g / NPB, bl = (g - k * NPB) * P;
        cx<T> o[P];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const cx<T> zk = xb[(bl + q) * SB + (k == M ? 0 : k)];
            const cx<T> zm = xb[(bl + q) * SB + (k == 0 ? 0 : M - k)];
            o[q] = r2c_post2(zk, zm, sr2c[k]);
        }
        if constexpr (P == 2) store_unit<T>(spec + (size_t)k * plane + line0 + bl, o);
        else spec[(size_t)k * plane + line0 + bl] = o[0];
    }
    if constexpr (ADJ) {
        __shared__ double red[NT / 64];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double sum = block_sum(acc[q], red);
            if (tid == 0) partials[(size_t)blockIdx.x * 4 + q] = sum;
        }
    }
}

// Spectrum values of the z inverse transform for NB lines, in registers: the
// (M+1) x NB block of X_k (k <= M) read in N rounds of NT threads, every load
// issued before any is waited for; in FP32 each thread reads two adjacent lines
// (16-byte loads).  Out-of-range slots of the last round read the block's last
// unit (in bounds) and stage it again (see tab_stage).
template <typename T, int M, int NB, int NT>
struct SpecRegs {
    static constexpr int P = sizeof(T) == 4 ? 2 : 1;  // lines per load
    static constexpr int total = (M + 1) * (NB / P);  // loads per block
    static constexpr int N = (total + NT - 1) / NT;
    static_assert(NB % P == 0, "pairs of lines");
    cx<T> v[N][P];
};

template <typename T, int M, int NB, int NT>
__device__ __forceinline__ void c2r_issue_loads(SpecRegs<T, M, NB, NT>& r,
                                                const cx<T>* __restrict__ spec, size_t plane,
                                                size_t line0, int tid) {
    using R = SpecRegs<T, M, NB, NT>;
#pragma unroll
    for (int u = 0; u < R::N; ++u) {
        const int g = min(tid + u * NT, R::total - 1);
        const int k = g / (NB / R::P), bl = (g - k * (NB / R::P)) * R::P;
        const cx<T>* src = spec + (size_t)k * plane + line0 + bl;
        if constexpr (R::P == 2) load_unit<T>(src, r.v[u]);
        else r.v[u][0] = src[0];
    }
}

template <typename T, int M, int NB, int NT>
__device__ __forceinline__ void c2r_stage(const SpecRegs<T, M, NB, NT>& r, cx<T>* xin, int tid) {
    using R = SpecRegs<T, M, NB, NT>;
    constexpr int SI = M + 1;
#pragma unroll
    for (int u = 0; u < R::N; ++u) {
        const int g = min(tid + u * NT, R::total - 1);
        const int k = g / (NB / R::P), bl = (g - k * (NB / R::P)) * R::P;
#pragma unroll
        for (int q = 0; q < R::P; ++q) xin[(bl + q) * SI + k] = r.v[u][q];
    }
}

// Front half of the z inverse transform for NB lines, from X_k (k <= M) staged
// in xin (c2r_stage, then a barrier): form Z_j, two-factor inverse FFT.  On
// return thread (b, t < R2) holds z_m = (Phi_{2m}, Phi_{2m+1}) for
// m = t + R2 k in w[k] (already / Nt).  xin needs NB * (M + 1) entries, xb
// NB * R2 * (R1 + 1); they may alias.
template <typename T, int R1, int R2, int NB>
__device__ __forceinline__ void c2r_front2(cx<T> (&w)[R1], cx<T>* xin, cx<T>* xb, const cx<T>* stw,
                                           const cx<T>* sr2c, int tid) {
    constexpr int M = R1 * R2;
    constexpr int SB = R2 * (R1 + 1);
    constexpr int SI = M + 1;
    const int t = tid % R1, b = tid / R1;
    const bool act = tid < NB * R1;
    cx<T> v[R2];
    if (act) {
#pragma unroll
        for (int n = 0; n < R2; ++n) {
            const int j = t + R1 * n;
            if (j == 0) {
                const T x0 = xin[b * SI].x, xm = xin[b * SI + M].x;
                v[n] = cx<T>{x0 + xm, x0 - xm};
            } else {
                const cx<T> xa = xin[b * SI + j], xc = xin[b * SI + M - j];
                const cx<T> s1 = xa + conj(xc);
                const cx<T> d1 = cmulc(xa - conj(xc), sr2c[j]);
                v[n] = cx<T>{s1.x - d1.y, s1.y + d1.x};
            }
        }
        rdft<T, R2, true>(v);
        twiddle_phase<T, R2, true>(v, t, stw);
    }
    __syncthreads();  // xin reads complete before xb (which may alias) is written
    if (act) {
#pragma unroll
        for (int k = 0; k < R2; ++k) xb[b * SB + k * (R1 + 1) + t] = v[k];
    }
    __syncthreads();
    if (act && t < R2) {
#pragma unroll
        for (int n = 0; n < R1; ++n) w[n] = xb[b * SB + t * (R1 + 1) + n];
        rdft<T, R1, true>(w);
    }
}


template <int R1, int R2, int NB>
constexpr int c2r_region() {  // complex entries of the xin / xb region
    constexpr int M = R1 * R2;
    return NB * (M + 1) > NB * R2 * (R1 + 1) ? NB * (M + 1) : NB * R2 * (R1 + 1);
}

// Phi to a real [Nx][Ny][Nz] buffer.
template <typename T, int R1, int R2>
__global__ void __launch_bounds__((rows_per_block<T, R1, R1 * R2>() * R1))
    k_c2r_phi2(T* __restrict__ phi, const cx<T>* __restrict__ spec, int Nx, int Ny,
               const cx<T>* __restrict__ twz, const cx<T>* __restrict__ twr2c) {
    constexpr int M = R1 * R2;
    constexpr int NB = rows_per_block<T, R1, M>();
    constexpr int NT = NB * R1;
    __shared__ cx<T> reg[c2r_region<R1, R2, NB>()];
    __shared__ cx<T> stw[M];
    __shared__ cx<T> sr2c[M + 1];
    const int tid = threadIdx.x;
    const int ngy = Ny / NB;
    const int bid = xcd_swizzle(blockIdx.x, gridDim.x);
    const int x = bid / ngy;
    const int y0 = (bid - x * ngy) * NB;
    const size_t line0 = (size_t)x * Ny + y0;
    TabRegs<cx<T>, M, NT> rtw;
    TabRegs<cx<T>, M + 1, NT> rr2;
    SpecRegs<T, M, NB, NT> rs;
    tab_issue(rtw, twz, tid);
    tab_issue(rr2, twr2c, tid);
    c2r_issue_loads(rs, spec, (size_t)Nx * Ny, line0, tid);
    tab_stage(rtw, stw, tid, [](int i) { return i; });
    tab_stage(rr2, sr2c, tid, [](int i) { return i; });
    c2r_stage(rs, reg, tid);
    __syncthreads();
    cx<T> w[R1];
    c2r_front2<T, R1, R2, NB>(w, reg, reg, stw, sr2c, tid);
    const int t = tid % R1, b = tid / R1;
    if (t < R2) {
        cx<T>* out = reinterpret_cast<cx<T>*>(phi + (line0 + b) * (2 * M));
#pragma unroll
        for (int k = 0; k < R1; ++k) out[t + R2 * k] = w[k];
    }
}

// Adjoint of the nonlinear step fused with the C2R of Phi_s = Phi[s] (the
// convolved adjoint source, in the spectrum buffer): with
// theta = dt (a V0 + g |psi_n|^2 + g_d Phi_n), s = Im(conj(mu) e^{-i theta} psi_n)
// and w = dt (g s + g_d Phi_s),  lam <- e^{+i theta} mu + 2 w psi_n  (lam holds
// mu on entry).  Phi_s stays in LDS; the pointwise update runs over the
// block's NB lines in coalesced 16-byte units.
//
// ZF: the update is followed by the conjugate z sweep that opens the next
// reverse step (the sweeps commute, so it may come first there): each wave
// then holds LPW whole lines in the fused z pass's layout, transposes its
// updated values through its own Phi_s rows to the segment layout and solves
// as the fused z pass does (conjugate tables cntab, kappa64): the arithmetic
// of this kernel followed by the standalone z sweep.
template <typename T, int R1, int R2>
constexpr bool adjupd_zf_ok() {  // whole 16-point segments on whole waves
    constexpr int M = R1 * R2, Nz = 2 * M, nseg = Nz / 16;
    constexpr int NB = rows_per_block<T, R1, M>();
    return Nz % 16 == 0 && nseg <= 16 && (nseg & (nseg - 1)) == 0 &&
           (NB * R1 / 64) * (64 / nseg) == NB && 2 * R2 == 16;
}

template <typename T, int R1, int R2, bool ZF>
__global__ void __launch_bounds__((rows_per_block<T, R1, R1 * R2>() * R1))
    k_c2r_adjupd2(cx<T>* __restrict__ lam, const cx<T>* __restrict__ psin,
                  const T* __restrict__ phin, const cx<T>* __restrict__ spec, int Nx, int Ny,
                  const cx<T>* __restrict__ twz, const cx<T>* __restrict__ twr2c, Phys2 ph,
                  const cx<double>* __restrict__ cntab, cx<double> kappa64) {
    constexpr int M = R1 * R2;
    constexpr int Nz = 2 * M;
    constexpr int NB = rows_per_block<T, R1, M>();
    constexpr int NT = NB * R1;
    constexpr int PS = M + M / 8 + 1;
    constexpr int U = 16 / (int)sizeof(cx<T>);
    constexpr int NU = NB * Nz / (NT * U);
    static_assert(NU * NT * U == NB * Nz, "whole units");
    static_assert(!ZF || adjupd_zf_ok<T, R1, R2>(), "z sweep on whole waves of whole lines");
    constexpr int REG = c2r_region<R1, R2, NB>() > NB * PS ? c2r_region<R1, R2, NB>() : NB * PS;
    // ZF geometry: the fused z pass's (16-point segments, LPW lines per wave)
    using A = cn_acc_t<T, false>;
    constexpr int SZ = 16, nseg = Nz / SZ;
    constexpr int LPW = ZF ? 64 / nseg : 1;
    constexpr int SL = Nz + nseg * U;
    constexpr int fit = (LPW * PS) / SL;
    constexpr int KR = fit >= LPW ? LPW : fit >= 8 ? 8 : fit >= 4 ? 4 : fit >= 2 ? 2 : 1;
    constexpr int TS = ZF ? Nz + Nz / SZ : 1;
    __shared__ __align__(16) cx<T> reg[REG];
    __shared__ cx<T> stw[M];
    __shared__ cx<T> sr2c[M + 1];
    __shared__ cx<A> ta[TS];
    __shared__ cx<A> tp[TS];
    __shared__ cx<A> tq[TS];
    __shared__ cx<A> spe[ZF ? nseg : 1];
    __shared__ cx<A> sqb[ZF ? nseg : 1];
    const int tid = threadIdx.x;
    const int ngy = Ny / NB;
    const int bid = xcd_swizzle(blockIdx.x, gridDim.x);
    const int x = bid / ngy;
    const int y0 = (bid - x * ngy) * NB;
    const size_t line0 = (size_t)x * Ny + y0;
    TabRegs<cx<T>, M, NT> rtw;
    TabRegs<cx<T>, M + 1, NT> rr2;
    SpecRegs<T, M, NB, NT> rs;
    TabRegs<cx<double>, ZF ? Nz : 1, NT> rta, rtp, rtq;
    TabRegs<cx<double>, ZF ? nseg : 1, NT> rpe, rqb;
    tab_issue(rtw, twz, tid);
    tab_issue(rr2, twr2c, tid);
    if constexpr (ZF) {
        tab_issue(rta, cntab + TAB_ALPHA * Nz, tid);
        tab_issue(rtp, cntab + TAB_P * Nz, tid);
        tab_issue(rtq, cntab + TAB_Q * Nz, tid);
        tab_issue(rpe, cntab + TAB_PEND * Nz, tid);
        tab_issue(rqb, cntab + TAB_QBEG * Nz, tid);
    }
    c2r_issue_loads(rs, spec, (size_t)Nx * Ny, line0, tid);
    tab_stage(rtw, stw, tid, [](int i) { return i; });
    tab_stage(rr2, sr2c, tid, [](int i) { return i; });
    if constexpr (ZF) {
        const auto ident = [](int i) { return i; };
        const auto padded = [](int i) { return i + i / SZ; };
        tab_stage(rta, ta, tid, padded);
        tab_stage(rtp, tp, tid, padded);
        tab_stage(rtq, tq, tid, padded);
        tab_stage(rpe, spe, tid, ident);
        tab_stage(rqb, sqb, tid, ident);
    }
    c2r_stage(rs, reg, tid);
    __syncthreads();
    cx<T> w[R1];
    c2r_front2<T, R1, R2, NB>(w, reg, reg, stw, sr2c, tid);
    __syncthreads();  // reg is rewritten with the Phi_s pairs
    {
        const int t = tid % R1, b = tid / R1;
        if (t < R2) {
#pragma unroll
            for (int k = 0; k < R1; ++k) {
                const int m = t + R2 * k;
                reg[b * PS + m + (m >> 3)] = w[k];
            }
        }
    }
    __syncthreads();
    const size_t base = line0 * Nz;
    const T dt = T(ph.dt), gg = T(ph.g), gdd = T(ph.gd), amp = T(ph.amp);
    const T xx = T(x - ph.hx) * T(ph.dx);
    const T vx = T(ph.cx) * xx * xx;
    // value j of this thread: element (line b, z e) of the block's lines.
    // ZF: the wave's LPW lines, unit j of the lane at (j * 64 + lane) U of
    // them; otherwise unit i of the block at (i NT + tid) U.
    const int lane = tid & 63, wv = tid >> 6;
    const auto elem = [&](int j) { return ZF ? wv * LPW * Nz + (j * 64 + lane) * U : (j * NT + tid) * U; };
    cx<T> mu[NU * U], pn[NU * U];
    T fn[NU * U];
#pragma unroll
    for (int i = 0; i < NU; ++i) {
        const int e = elem(i);
        load_unit<T>(lam + base + e, mu + i * U);
        load_unit<T>(psin + base + e, pn + i * U);
#pragma unroll
        for (int u = 0; u < U; ++u) fn[i * U + u] = phin[base + e + u];
    }
    cx<T> o[NU * U];
#pragma unroll
    for (int i = 0; i < NU; ++i) {
        const int e = elem(i);
        const int b = e / Nz;
        const T yy = T(y0 + b - ph.hy) * T(ph.dy);
        const T vxy = vx + T(ph.cy) * yy * yy;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int iz = e % Nz + u;
            const int mm = iz >> 1;
            const cx<T> fs = reg[b * PS + mm + (mm >> 3)];
            const T phis = (iz & 1) ? fs.y : fs.x;
            const T z = T(iz - ph.hz) * T(ph.dz);
            const T v0 = vxy + T(ph.cz) * z * z;
            const cx<T> p = pn[i * U + u], m = mu[i * U + u];
            const T th = dt * (amp * v0 + gg * abs2(p) + gdd * fn[i * U + u]);
            T sn, cs;
            sin_cos(th, &sn, &cs);
            const cx<T> pp = {p.x * cs + p.y * sn, p.y * cs - p.x * sn};
            const T sv = m.x * pp.y - m.y * pp.x;
            const T wv2 = dt * (gg * sv + gdd * phis);
            o[i * U + u] = cx<T>{m.x * cs - m.y * sn + T(2) * wv2 * p.x,
                                 m.y * cs + m.x * sn + T(2) * wv2 * p.y};
        }
        if constexpr (!ZF) store_unit<T>(lam + base + e, o + i * U);
    }
    if constexpr (ZF) {
        static_assert(NU * U == SZ, "a lane's units are one segment's worth of values");
        using WL = WaveLines<T, Nz, SZ, KR>;
        // this wave's Phi_s rows are read: they stage the transposes
        cx<T>* stg = reg + wv * LPW * PS;
        const int seg = lane % nseg;
        cx<A> v[SZ];
        WL::to_segments(stg, o, v, lane);
        const cx<A> kappa = {A(kappa64.x), A(kappa64.y)};
        const int tb = seg * (SZ + 1);
        cn_segment_solve_wave<T, SZ, nseg, false>(v, kappa, ta + tb, tp + tb, tq + tb, spe, sqb, seg);
        WL::store_from_segments(stg, v, lam + base + wv * LPW * Nz, lane);
    }
}

// The symmetric step's half nonlinear step after the sweeps, fused with the
// C2R of Phi (its density's convolution, in the spectrum buffer):
// psi <- psi e^{-theta} (imaginary time) or psi e^{-i theta} (real time),
// theta = dt (a V + g |psi|^2 + g_d Phi); Phi stays in LDS, the state moves in
// coalesced 16-byte units over the block's NB lines; in imaginary time the
// block's FP64 sum of |psi|^2 of the result goes to partials[blockIdx.x].
template <typename T, int R1, int R2, bool IMAG>
__global__ void __launch_bounds__((rows_per_block<T, R1, R1 * R2>() * R1))
    k_c2r_nl2(cx<T>* __restrict__ psi, const cx<T>* __restrict__ spec, int Nx, int Ny,
              const cx<T>* __restrict__ twz, const cx<T>* __restrict__ twr2c, Phys2 ph,
              double* __restrict__ partials) {
    constexpr int M = R1 * R2;
    constexpr int Nz = 2 * M;
    constexpr int NB = rows_per_block<T, R1, M>();
    constexpr int NT = NB * R1;
    constexpr int PS = M + M / 8 + 1;
    constexpr int U = 16 / (int)sizeof(cx<T>);
    constexpr int NU = NB * Nz / (NT * U);
    static_assert(NU * NT * U == NB * Nz, "whole units");
    constexpr int REG = c2r_region<R1, R2, NB>() > NB * PS ? c2r_region<R1, R2, NB>() : NB * PS;
    __shared__ cx<T> reg[REG];
    __shared__ cx<T> stw[M];
    __shared__ cx<T> sr2c[M + 1];
    __shared__ double red[NT / 64];
    const int tid = threadIdx.x;
    const int ngy = Ny / NB;
    const int bid = xcd_swizzle(blockIdx.x, gridDim.x);
    const int x = bid / ngy;
    const int y0 = (bid - x * ngy) * NB;
    const size_t line0 = (size_t)x * Ny + y0;
    TabRegs<cx<T>, M, NT> rtw;
    TabRegs<cx<T>, M + 1, NT> rr2;
    SpecRegs<T, M, NB, NT> rs;
    tab_issue(rtw, twz, tid);
    tab_issue(rr2, twr2c, tid);
    c2r_issue_loads(rs, spec, (size_t)Nx * Ny, line0, tid);
    // the state, issued last: in flight through the inverse transform
    const size_t base = line0 * Nz;
    cx<T> u[NU * U];
#pragma unroll
    for (int i = 0; i < NU; ++i) load_unit<T>(psi + base + (i * NT + tid) * U, u + i * U);
    tab_stage(rtw, stw, tid, [](int i) { return i; });
    tab_stage(rr2, sr2c, tid, [](int i) { return i; });
    c2r_stage(rs, reg, tid);
    __syncthreads();
    cx<T> w[R1];
    c2r_front2<T, R1, R2, NB>(w, reg, reg, stw, sr2c, tid);
    __syncthreads();  // reg is rewritten with the Phi pairs
    {
        const int t = tid % R1, b = tid / R1;
        if (t < R2) {
#pragma unroll
            for (int k = 0; k < R1; ++k) {
                const int m = t + R2 * k;
                reg[b * PS + m + (m >> 3)] = w[k];
            }
        }
    }
    __syncthreads();
    const T dt = T(ph.dt), gg = T(ph.g), gdd = T(ph.gd), amp = T(ph.amp);
    const T xx = T(x - ph.hx) * T(ph.dx);
    const T vx = T(ph.cx) * xx * xx;
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < NU; ++i) {
        const int e = (i * NT + tid) * U;
        const int b = e / Nz;
        const T yy = T(y0 + b - ph.hy) * T(ph.dy);
        const T vxy = vx + T(ph.cy) * yy * yy;
        cx<T> o[U];
#pragma unroll
        for (int v = 0; v < U; ++v) {
            const int iz = e % Nz + v;
            const int mm = iz >> 1;
            const cx<T> fs = reg[b * PS + mm + (mm >> 3)];
            const T phi = (iz & 1) ? fs.y : fs.x;
            const T z = T(iz - ph.hz) * T(ph.dz);
            const cx<T> q = u[i * U + v];
            const T th = dt * (amp * (vxy + T(ph.cz) * z * z) + gg * abs2(q) + gdd * phi);
            if constexpr (IMAG) {
                o[v] = exp_of(-th) * q;
                acc += double(o[v].x) * o[v].x + double(o[v].y) * o[v].y;
            } else {
                o[v] = rotate_phase(q, th);
            }
        }
        store_unit<T>(psi + base + e, o);
    }
    if constexpr (IMAG) {
        const double sum = block_sum(acc, red);
        if (tid == 0) partials[blockIdx.x] = sum;
    }
}

// ---------------------------------------------------------------------------
// P5: z inverse transform -> Phi, nonlinear phase, Crank-Nicolson along z.
// LDS: region (xin / xb, then Phi pairs, then the z carries) | Psi tile |
// twiddles | segment carry products.
// ---------------------------------------------------------------------------

// lines per block of the fused z pass: the state tile (Nz (NB+1) complex) must
// fit next to the spectral region in 64 KB of LDS
template <typename T, int R1, int M>
constexpr int step_nb() {
    int nb = rows_per_block<T, R1, M>();
    while (nb > 1 && (size_t)(2 * M) * (nb + 1) * 2 * sizeof(T) > 40 * 1024) nb >>= 1;
    return nb;
}

template <typename T, int R1, int R2, int SZ>
constexpr int step2_nb() {
    return rows_per_block<T, R1, R1 * R2>();
}

template <typename T, int R1, int R2, int SZ>
constexpr int step2_threads() {
    constexpr int M = R1 * R2;
    constexpr int NB = step2_nb<T, R1, R2, SZ>();
    constexpr int nseg = (2 * M + SZ - 1) / SZ;
    constexpr int a = NB * R1, c = NB * nseg;
    constexpr int m = a > c ? a : c;
    return (m + 63) / 64 * 64;
}

// Staging geometry of the fused z pass.  A wave owns LPW = 64 / nseg whole
// lines; its state moves between HBM and registers in 16-byte units with
// consecutive lanes on consecutive addresses, and is transposed to and from
// the segment layout of the tridiagonal solve through the LDS rows that held
// the wave's Phi (free once the nonlinear step has read them), KR lines at a
// time.  A staged line is Nz values with one unit of padding after each
// segment, so that the segment-wise 16-byte accesses spread over the banks.
template <typename T, int R1, int R2, int SZ>
struct Step2Geom {
    static constexpr int M = R1 * R2;
    static constexpr int Nz = 2 * M;
    static constexpr int nseg = Nz / SZ;
    static constexpr int LPW = 64 / nseg;
    static constexpr int U = 16 / (int)sizeof(cx<T>);
    static constexpr int NU = SZ / U;  // units per lane
    // Phi pairs at m + (m >> PSH): one pad entry per 8 (FP32) or 16 (FP64, 16-byte
    // entries) spreads the reads over the banks; the smaller FP64 pad keeps the
    // block within 53 KB of LDS, three blocks per CU
    static constexpr int PSH = sizeof(T) == 8 ? 4 : 3;
    static constexpr int PS = M + (M >> PSH) + 1;
    static constexpr int SL = Nz + nseg * U;
    static constexpr int fit = (LPW * PS) / SL;
    static constexpr int KR = fit >= LPW ? LPW : fit >= 8 ? 8 : fit >= 4 ? 4 : fit >= 2 ? 2 : 1;
    static constexpr int JR = KR * Nz / (64 * U);  // unit loads per lane and round
};

// Fused P5 with the state kept in registers: each wave loads its lines
// (coalesced 16-byte units) at kernel start, so the loads overlap the spectrum
// load and the inverse FFT; the nonlinear phase is applied in that layout with
// Phi from LDS; the values are then transposed through LDS to the segment
// layout (lane = segment, segment fastest) for the z tridiagonal solve
// (neighbours and carries by wave shuffles), and back for coalesced stores.
// LDS: region (xin / xb, then Phi pairs, then the staging) | alpha, P, Q tables
// | twiddles.
//
// YF: the block's NB lines are NB / 16 whole segments of the y axis (16 lines
// each), and the y Crank-Nicolson solve is started here: after the z solve the
// lines are transposed through LDS (half of z at a time) and every (segment,
// z) column is solved with zero carries and without its two outside
// neighbours (u at the lines just before and after the segment).  By
// linearity the exact solution is that local one plus E_i c_d + Q_i c_x, where
// c_d is the true forward value entering the segment plus the left neighbour,
// c_x the true solution after the segment plus the right neighbour.  The
// block writes the local solution to psi_out and, per column, three arrays
// [Nx][Ny/16][Nz] to ycar: d at the last line plus u there, x at the first
// line plus u there, and u at the first line; the carry pass turns these into
// c_d and c_x, which the x sweep adds while it loads.
//
// Occupancy: FP32 imaginary time at five waves per SIMD; the FP64 fused-y
// variant at 256-point lines at three (168 registers, a few spilled: 147 ->
// 142 us at 256^3 against two waves at its natural 180).
template <typename T, int R1, int R2, int SZ, bool RC, bool PHI, bool YF>
__global__ void __launch_bounds__((step2_threads<T, R1, R2, SZ>()))
__attribute__((amdgpu_waves_per_eu(RC && sizeof(T) == 4 ? 5 : (YF && R1 * R2 == 128 ? 3 : 1), 8)))
    k_c2r_step2(const cx<T>* psi_in, cx<T>* psi_out, T* __restrict__ phi_out,
                const cx<T>* __restrict__ spec, int Nx, int Ny,
                const cx<T>* __restrict__ twz, const cx<T>* __restrict__ twr2c,
                const cx<double>* __restrict__ cntab, cx<double> kappa64,
                const double* __restrict__ sigma, Phys2 ph, NlConst nl,
                const cx<double>* __restrict__ ytab, cx<double> kappay64,
                cx<T>* __restrict__ ycar, int phi_sigma) {
    using A = cn_acc_t<T, RC>;
    using G = Step2Geom<T, R1, R2, SZ>;
    constexpr int M = G::M, Nz = G::Nz, nseg = G::nseg, LPW = G::LPW, U = G::U, NU = G::NU;
    constexpr int PS = G::PS, SL = G::SL, KR = G::KR, JR = G::JR, PSH = G::PSH;
    constexpr int NB = step2_nb<T, R1, R2, SZ>();
    constexpr int NT = step2_threads<T, R1, R2, SZ>();
    static_assert(Nz % SZ == 0 && SZ % U == 0, "full segments of whole units");
    static_assert((nseg & (nseg - 1)) == 0 && 64 % nseg == 0, "a line's segments share a wave");
    static_assert(NB % LPW == 0 && NB * nseg <= NT, "whole waves of lines");
    static_assert(LPW % KR == 0 && (KR * Nz) % (64 * U) == 0 && KR * SL <= LPW * PS,
                  "staging rounds of whole unit loads inside the wave's Phi rows");
    static_assert((LPW * PS) % U == 0, "16-byte aligned staging");
    // Phi pairs at m + (m >> PSH) and table entries at e + e/SZ (bank spread)
    constexpr int TS = Nz + Nz / SZ;
    constexpr int REG = c2r_region<R1, R2, NB>() > NB * PS ? c2r_region<R1, R2, NB>() : NB * PS;
    __shared__ __align__(16) cx<T> reg[REG];
    __shared__ cx<A> ta[TS];
    __shared__ cx<A> tp[TS];
    __shared__ cx<A> tq[TS];
    __shared__ cx<A> spe[nseg];
    __shared__ cx<A> sqb[nseg];
    __shared__ cx<T> stw[M];
    __shared__ cx<T> sr2c[M + 1];
    __shared__ cx<A> sya[YF ? NB : 1];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const bool act = wv * LPW < NB;  // wave-uniform
    const int ngy = Ny / NB;
    const int bid = xcd_swizzle(blockIdx.x, gridDim.x);
    const int x = bid / ngy;
    const int y0 = (bid - x * ngy) * NB;
    const size_t line0 = (size_t)x * Ny + y0;
    // Every global load of the block is issued before the first wait: tables
    // and the spectrum block first, the state last, so that staging the former
    // in LDS leaves the state loads in flight through the inverse FFT.
    TabRegs<cx<T>, M, NT> rtw;
    TabRegs<cx<T>, M + 1, NT> rr2;
    TabRegs<cx<double>, Nz, NT> rta, rtp, rtq;
    TabRegs<cx<double>, nseg, NT> rpe, rqb;
    SpecRegs<T, M, NB, NT> rsp;
    tab_issue(rtw, twz, tid);
    tab_issue(rr2, twr2c, tid);
    tab_issue(rta, cntab + TAB_ALPHA * Nz, tid);
    tab_issue(rtp, cntab + TAB_P * Nz, tid);
    tab_issue(rtq, cntab + TAB_Q * Nz, tid);
    tab_issue(rpe, cntab + TAB_PEND * Nz, tid);
    tab_issue(rqb, cntab + TAB_QBEG * Nz, tid);
    TabRegs<cx<double>, YF ? NB : 1, NT> rya;
    if constexpr (YF) tab_issue(rya, ytab + TAB_ALPHA * Ny + y0, tid);
    c2r_issue_loads(rsp, spec, (size_t)Nx * Ny, line0, tid);
    // the wave's LPW lines are LPW * Nz consecutive values; unit j of this lane
    // holds values (j * 64 + lane) * U + u (waves without lines load the last
    // wave's, unused, to keep the load sequence uniform)
    const size_t wl = (line0 + (size_t)min(wv * LPW, NB - LPW)) * Nz;  // the wave's first value
    cx<T> a[SZ];
#pragma unroll
    for (int j = 0; j < NU; ++j) load_unit<T>(psi_in + wl + (j * 64 + lane) * U, a + j * U);
    const auto ident = [](int i) { return i; };
    const auto padded = [](int i) { return i + i / SZ; };
    tab_stage(rtw, stw, tid, ident);
    tab_stage(rr2, sr2c, tid, ident);
    tab_stage(rta, ta, tid, padded);
    tab_stage(rtp, tp, tid, padded);
    tab_stage(rtq, tq, tid, padded);
    tab_stage(rpe, spe, tid, ident);
    tab_stage(rqb, sqb, tid, ident);
    if constexpr (YF) tab_stage(rya, sya, tid, ident);
    c2r_stage(rsp, reg, tid);
    __syncthreads();
    cx<T> w[R1];
    c2r_front2<T, R1, R2, NB>(w, reg, reg, stw, sr2c, tid);
    __syncthreads();  // reg is rewritten with the Phi pairs
    {
        const int t = tid % R1, b = tid / R1;
        if (tid < NB * R1 && t < R2) {
#pragma unroll
            for (int k = 0; k < R1; ++k) {
                const int m = t + R2 * k;
                reg[b * PS + m + (m >> PSH)] = w[k];
            }
        }
    }
    __syncthreads();
    if (!YF && !act) return;  // no barrier follows (YF: the y phase has barriers)
    const int seg = lane % nseg;
    cx<A> v[SZ];
    if (act) {
    // nonlinear step in the load layout (pre-step density, lazily normalised).
    // The exponent is a line term (x, y) plus a z term, shared by the points
    // of a line and of a z index, plus the density and Phi terms.  Imaginary
    // time, FP32: the factor sqrt(sigma) enters the exponent; its rounding only
    // rescales the stored state, which the next step's norm absorbs.  Real
    // time takes no sigma (the phase keeps the norm).
    constexpr bool kB2 = RC && sizeof(T) == 4;
    const double sg = sigma ? sigma[0] : 1.0;
    const T kn = T(nl.kg * sg), kp = T(phi_sigma ? nl.kd * sg : nl.kd);
    const T ky = T(nl.ky), kz = T(nl.kz);
    const int ix = x - ph.hx;
    T cx0 = T(nl.kx * double(ix * ix));
    if constexpr (kB2) cx0 -= T(0.5) * __builtin_amdgcn_logf(T(sg));
    [[maybe_unused]] const T rs = RC && !kB2 ? T(sqrt(sg)) : T(1);
    const int iy0 = y0 + wv * LPW - ph.hy;
    const cx<T>* prow = reg + wv * LPW * PS;
    // with 64 U | Nz the units j of all lanes lie on one line and the z offset
    // of a unit is a constant plus lane U
    constexpr bool kLine = Nz % (64 * U) == 0;
#pragma unroll
    for (int j = 0; j < NU; ++j) {
        const int c0 = (j * 64 + lane) * U;
        const int lw = kLine ? (j * 64 * U) / Nz : c0 / Nz;
        const int e0 = kLine ? (j * 64 * U) % Nz + lane * U : c0 % Nz;
        const int iy = iy0 + lw;
        const T cl = ky * T(iy * iy) + cx0;
        const int m = e0 >> 1;
        const cx<T> fv = prow[lw * PS + m + (m >> PSH)];
        if constexpr (PHI) {  // Phi of the pre-step density, for the adjoint
            const T phs = phi_sigma ? T(sg) : T(1);
            if constexpr (U == 2) *reinterpret_cast<cx<T>*>(phi_out + wl + c0) = phs * fv;
            else phi_out[wl + c0] = phs * ((e0 & 1) ? fv.y : fv.x);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u;
            const T phi = (e & 1) ? fv.y : fv.x;
            const int iz = e - ph.hz;
            const T sz = T(iz);
            cx<T>& q = a[j * U + u];
            const T th = kp * phi + (kn * abs2(q) + (cl + kz * sz * sz));
            if constexpr (kB2) {  // imaginary time, FP32: 2^-th
                q = __builtin_amdgcn_exp2f(-th) * q;
            } else if constexpr (RC) {
                q = (rs * exp_of(-th)) * q;
            } else {
                q = rotate_phase(q, th);
            }
        }
    }
    // to the segment layout, KR lines per round, through this wave's Phi rows
    cx<T>* stg = reg + wv * LPW * PS;
    WaveLines<T, Nz, SZ, KR>::to_segments(stg, a, v, lane);
    // Crank-Nicolson along z: the nseg segments of a line are nseg consecutive
    // lanes of one wave (carries by shuffles)
    const cx<A> kappa = {A(kappa64.x), A(kappa64.y)};
    const int tb = seg * (SZ + 1);
    cn_segment_solve_wave<T, SZ, nseg, RC>(v, kappa, ta + tb, tp + tb, tq + tb, spe, sqb, seg);
    // back to the load layout and out
    if constexpr (!YF) WaveLines<T, Nz, SZ, KR>::store_from_segments(stg, v, psi_out + wl, lane);
    }  // act
    if constexpr (YF) {
        // local y solve of 16-line segments, half of z per round: lines padded
        // by one 16-byte unit per 16 values
        constexpr int HZ = Nz / 2, LS = HZ + U * (HZ / 16), NSY = NB / 16;
        static_assert(SZ == 16 && NB % 16 == 0 && NB * LS <= REG && HZ * NSY <= NT,
                      "y segments of 16 lines, one half of z per round in the region");
        const cx<A> zero = {A(0), A(0)};
        const cx<A> kappay = {A(kappay64.x), A(kappay64.y)};
        const int nky = Ny / 16;
        const size_t cst = (size_t)Nx * nky * Nz;  // one carry array
        const int col = tid % HZ, ys = tid / HZ;
        const int sl = lane / nseg;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            __syncthreads();  // staging reads (and the previous round's) done
            const int z0 = seg * SZ - h * HZ;
            if (act && z0 >= 0 && z0 < HZ) {
                cx<T>* dst = reg + (wv * LPW + sl) * LS + z0 + U * (z0 / 16);
#pragma unroll
                for (int j = 0; j < SZ / U; ++j) {
                    cx<T> t2[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) t2[u] = to_store<T>(v[j * U + u]);
                    store_unit<T>(dst + j * U, t2);
                }
            }
            __syncthreads();
            if (tid < HZ * NSY) {
                cx<A> w2[16];
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    w2[j] = widen<A>(reg[(ys * 16 + j) * LS + col + U * (col / 16)]);
                const cx<A>* al = sya + ys * 16;
                const cx<A> ufirst = w2[0], ulast = w2[15];
                cx<A> d = zero, prev = zero;
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const cx<A> cur = w2[j];
                    const cx<A> nxt = j < 15 ? w2[j < 15 ? j + 1 : j] : zero;
                    d = kmul<RC>(al[j], kfma<RC>(kappay, cur, (d + prev) + nxt));
                    prev = cur;
                    w2[j] = d;
                }
                const cx<A> dlast = d;
                cx<A> xv = zero;
#pragma unroll
                for (int j = 15; j >= 0; --j) {
                    xv = kfma<RC>(al[j], xv, w2[j]);
                    w2[j] = xv;
                }
                const int z = h * HZ + col;
                cx<T>* out = psi_out + (line0 + ys * 16) * Nz + z;
#pragma unroll
                for (int j = 0; j < 16; ++j) out[(size_t)j * Nz] = to_store<T>(w2[j]);
                const size_t ci = ((size_t)x * nky + (y0 >> 4) + ys) * Nz + z;
                ycar[ci] = to_store<T>(dlast + ulast);
                ycar[cst + ci] = to_store<T>(w2[0] + ufirst);
                ycar[2 * cst + ci] = to_store<T>(ufirst);
            }
        }
    }
}

}  // namespace

// ---- dispatch --------------------------------------------------------------

#define DGPE_SPLITS(X) \
    X(4, 4) X(8, 4) X(8, 6) X(8, 8) X(12, 8) X(16, 8) X(16, 12) X(16, 16) X(24, 16) X(32, 16)

template <typename T>
int fast_rows_per_block(int L) {
    switch (L) {
#define DGPE_CASE(A, B) \
    case A * B: return rows_per_block<T, A, A * B>();
        DGPE_SPLITS(DGPE_CASE)
#undef DGPE_CASE
        default: return 0;
    }
}

template <typename T>
int fast_rows_threads(int L) {
    switch (L) {
#define DGPE_CASE(A, B) \
    case A * B: return rows_per_block<T, A, A * B>() * A;
        DGPE_SPLITS(DGPE_CASE)
#undef DGPE_CASE
        default: return 0;
    }
}

template <typename T>
bool fast_rows_sigma_ok(const Plan& p) {
    const int nt = fast_rows_threads<T>(p.n[1]);
    return nt > 0 && nt % 64 == 0;
}

template <typename T>
bool fast_rows(const Plan& p, bool inverse, const double* npart, int nnpart, double* sigma_out) {
    const int L = p.n[1];
    const Split2 s = fast_split(L);
    if (!s.r1) return false;
    if (npart && (inverse || !fast_rows_sigma_ok<T>(p))) return false;
    const int nb = fast_rows_per_block<T>(L);
    const int nrows = (p.n[2] / 2 + 1) * p.n[0];
    const int blocks = (nrows + nb - 1) / nb;
    const double dV = p.d[0] * p.d[1] * p.d[2];
    switch (L) {
#define DGPE_CASE(A, B)                                                                              \
    case A * B:                                                                                      \
        if (inverse)                                                                                 \
            hipLaunchKernelGGL((k_rows2<T, A, B, true>), dim3(blocks), dim3(nb * A), 0, p.stream,   \
                               (cx<T>*)p.spec, nrows, (const cx<T>*)p.tw[1], nullptr, 0, dV,        \
                               nullptr);                                                             \
        else                                                                                         \
            hipLaunchKernelGGL((k_rows2<T, A, B, false>), dim3(blocks), dim3(nb * A), 0, p.stream,  \
                               (cx<T>*)p.spec, nrows, (const cx<T>*)p.tw[1], npart, nnpart, dV,     \
                               sigma_out);                                                           \
        return true;
        DGPE_SPLITS(DGPE_CASE)
#undef DGPE_CASE
        default: return false;
    }
}

template <typename T>
int fast_xmul_cols(int L) {
    switch (L) {
#define DGPE_CASE(A, B) \
    case A * B: return xmul_cols<T, A, A * B>();
        DGPE_SPLITS(DGPE_CASE)
#undef DGPE_CASE
        default: return 0;
    }
}

template <typename T>
bool fast_xmul(const Plan& p) {
    const int L = p.n[0];
    const Split2 s = fast_split(L);
    if (!s.r1) return false;
    const int nb = fast_xmul_cols<T>(L);
    if (p.n[1] % nb) return false;
    const int blocks = (p.n[2] / 2 + 1) * (p.n[1] / nb);
    if (L == 512) {  // R1 = 2 R2: phase B split over lane pairs
        hipLaunchKernelGGL((k_xmul2s<T, 32, 16>), dim3(blocks), dim3(nb * 32), 0, p.stream,
                           (cx<T>*)p.spec, p.n[1], (const cx<T>*)p.tw[0], (const T*)p.ukern);
        return true;
    }
    switch (L) {
#define DGPE_CASE(A, B)                                                                              \
    case A * B:                                                                                      \
        hipLaunchKernelGGL((k_xmul2<T, A, B>), dim3(blocks), dim3(nb * A), 0, p.stream,             \
                           (cx<T>*)p.spec, p.n[1], (const cx<T>*)p.tw[0], (const T*)p.ukern);        \
        return true;
        DGPE_SPLITS(DGPE_CASE)
#undef DGPE_CASE
        default: return false;
    }
}

template <typename T>
bool fast_r2c(const Plan& p, const void* psi, const double* sigma) {
    const int M = p.n[2] / 2;
    const Split2 s = fast_split(M);
    if (!s.r1) return false;
    const int nb = fast_rows_per_block<T>(M);
    if (p.n[1] % nb) return false;
    const int blocks = p.n[0] * (p.n[1] / nb);
    switch (M) {
#define DGPE_CASE(A, B)                                                                              \
    case A * B:                                                                                      \
        hipLaunchKernelGGL((k_r2c2<T, A, B, false>), dim3(blocks), dim3(nb * A), 0, p.stream,       \
                           (const cx<T>*)psi, (cx<T>*)p.spec, p.n[0], p.n[1], (const cx<T>*)p.tw[2], \
                           (const cx<T>*)p.twr2c, sigma, (const cx<T>*)nullptr, (const T*)nullptr,  \
                           Phys2{}, (double*)nullptr);                                               \
        return true;
        DGPE_SPLITS(DGPE_CASE)
#undef DGPE_CASE
        default: return false;
    }
}

template <typename T>
bool fast_r2c_adj(const Plan& p, const void* mu, const void* psin, const void* phin, double amp,
                  double* partials, int* nblocks) {
    const int M = p.n[2] / 2;
    const Split2 s = fast_split(M);
    if (!s.r1) return false;
    const int nb = fast_rows_per_block<T>(M);
    if (p.n[1] % nb) return false;
    const int blocks = p.n[0] * (p.n[1] / nb);
    if ((size_t)blocks * 4 > p.red_count) return false;
    *nblocks = blocks;
    Phys2 ph{p.dt, p.g, p.gd, amp, 0, p.n[0] / 2, p.n[1] / 2, p.n[2] / 2,
             p.d[0], p.d[1], p.d[2], 0.5 * p.trap[0] * p.trap[0], 0.5 * p.trap[1] * p.trap[1],
             0.5 * p.trap[2] * p.trap[2]};
    switch (M) {
#define DGPE_CASE(A, B)                                                                              \
    case A * B:                                                                                      \
        hipLaunchKernelGGL((k_r2c2<T, A, B, true>), dim3(blocks), dim3(nb * A), 0, p.stream,        \
                           (const cx<T>*)mu, (cx<T>*)p.spec, p.n[0], p.n[1], (const cx<T>*)p.tw[2],  \
                           (const cx<T>*)p.twr2c, (const double*)nullptr, (const cx<T>*)psin,       \
                           (const T*)phin, ph, partials);                                            \
        return true;
        DGPE_SPLITS(DGPE_CASE)
#undef DGPE_CASE
        default: return false;
    }
}

template <typename T>
bool fast_c2r_adjupd(const Plan& p, void* lam, const void* psin, const void* phin, double amp,
                     bool zsweep, bool* zdone) {
    *zdone = false;
    const int M = p.n[2] / 2;
    const Split2 s = fast_split(M);
    if (!s.r1) return false;
    const int nb = fast_rows_per_block<T>(M);
    if (p.n[1] % nb) return false;
    const int blocks = p.n[0] * (p.n[1] / nb);
    Phys2 ph{p.dt, p.g, p.gd, amp, 0, p.n[0] / 2, p.n[1] / 2, p.n[2] / 2,
             p.d[0], p.d[1], p.d[2], 0.5 * p.trap[0] * p.trap[0], 0.5 * p.trap[1] * p.trap[1],
             0.5 * p.trap[2] * p.trap[2]};
    // the conjugate z sweep of the next reverse step, where the z tables hold
    // 16-point segments and the split has the fused form
    const bool zf = zsweep && !p.imag && p.lc.seg[2] == 16;
    const cx<double>* ztab = (const cx<double>*)p.cntab[2][1];
    const cx_coef kz = cn_kappa(p, 2, true);
    const cx<double> kappa = {kz.re, kz.im};
    switch (M) {
#define DGPE_LAUNCH(A, B, ZFV)                                                                       \
    hipLaunchKernelGGL((k_c2r_adjupd2<T, A, B, ZFV>), dim3(blocks), dim3(nb * A), 0, p.stream,       \
                       (cx<T>*)lam, (const cx<T>*)psin, (const T*)phin, (const cx<T>*)p.spec,        \
                       p.n[0], p.n[1], (const cx<T>*)p.tw[2], (const cx<T>*)p.twr2c, ph, ztab, kappa)
#define DGPE_CASE(A, B)                                                                              \
    case A * B:                                                                                      \
        if constexpr (adjupd_zf_ok<T, A, B>()) {                                                     \
            if (zf) {                                                                                \
                DGPE_LAUNCH(A, B, true);                                                             \
                *zdone = true;                                                                       \
                return true;                                                                         \
            }                                                                                        \
        }                                                                                            \
        DGPE_LAUNCH(A, B, false);                                                                    \
        return true;
        DGPE_SPLITS(DGPE_CASE)
#undef DGPE_CASE
#undef DGPE_LAUNCH
        default: return false;
    }
}

template <typename T>
bool fast_c2r_phi(const Plan& p, void* phi) {
    const int M = p.n[2] / 2;
    const Split2 s = fast_split(M);
    if (!s.r1) return false;
    const int nb = fast_rows_per_block<T>(M);
    if (p.n[1] % nb) return false;
    const int blocks = p.n[0] * (p.n[1] / nb);
    switch (M) {
#define DGPE_CASE(A, B)                                                                              \
    case A * B:                                                                                      \
        hipLaunchKernelGGL((k_c2r_phi2<T, A, B>), dim3(blocks), dim3(nb * A), 0, p.stream, (T*)phi, \
                           (const cx<T>*)p.spec, p.n[0], p.n[1], (const cx<T>*)p.tw[2],             \
                           (const cx<T>*)p.twr2c);                                                   \
        return true;
        DGPE_SPLITS(DGPE_CASE)
#undef DGPE_CASE
        default: return false;
    }
}

template <typename T>
bool fast_c2r_nl(const Plan& p, void* psi, double dt, double amp, double* partials, int* nblocks) {
    const int M = p.n[2] / 2;
    const Split2 s = fast_split(M);
    if (!s.r1) return false;
    const int nb = fast_rows_per_block<T>(M);
    if (p.n[1] % nb) return false;
    const int blocks = p.n[0] * (p.n[1] / nb);
    if ((size_t)blocks > p.red_count) return false;
    *nblocks = blocks;
    Phys2 ph{dt, p.g, p.gd, amp, p.imag ? 1 : 0, p.n[0] / 2, p.n[1] / 2, p.n[2] / 2,
             p.d[0], p.d[1], p.d[2], 0.5 * p.trap[0] * p.trap[0], 0.5 * p.trap[1] * p.trap[1],
             0.5 * p.trap[2] * p.trap[2]};
    switch (M) {
#define DGPE_CASE(A, B)                                                                              \
    case A * B:                                                                                      \
        if (p.imag)                                                                                  \
            hipLaunchKernelGGL((k_c2r_nl2<T, A, B, true>), dim3(blocks), dim3(nb * A), 0, p.stream, \
                               (cx<T>*)psi, (const cx<T>*)p.spec, p.n[0], p.n[1],                   \
                               (const cx<T>*)p.tw[2], (const cx<T>*)p.twr2c, ph, partials);         \
        else                                                                                         \
            hipLaunchKernelGGL((k_c2r_nl2<T, A, B, false>), dim3(blocks), dim3(nb * A), 0,           \
                               p.stream, (cx<T>*)psi, (const cx<T>*)p.spec, p.n[0], p.n[1],         \
                               (const cx<T>*)p.tw[2], (const cx<T>*)p.twr2c, ph, partials);         \
        return true;
        DGPE_SPLITS(DGPE_CASE)
#undef DGPE_CASE
        default: return false;
    }
}

// fused P5 for Nz/2 in {32, 64, 128} with 16-point z segments
#define DGPE_STEP_SPLITS(X) X(8, 4) X(8, 8) X(16, 8)

template <typename T>
int fast_c2r_step_lines(const Plan& p) {
    const int M = p.n[2] / 2;
    if (p.lc.seg[2] != 16 || p.n[2] % 16) return 0;
    int nb = 0;
    switch (M) {
#define DGPE_CASE(A, B) \
    case A * B: nb = step2_nb<T, A, B, 16>(); break;
        DGPE_STEP_SPLITS(DGPE_CASE)
#undef DGPE_CASE
        default: return 0;
    }
    return p.n[1] % nb ? 0 : nb;
}

template <typename T>
bool fast_c2r_step_yfused_ok(const Plan& p) {
    const int nb = fast_c2r_step_lines<T>(p);
    return nb > 0 && nb % 16 == 0 && p.imag && p.lc.seg[1] == 16 && p.n[1] % 16 == 0;
}

template <typename T>
bool fast_c2r_step(const Plan& p, const void* psi_in, void* psi_out, const double* sigma,
                   double amp, void* phi_out, void* ycar, bool phi_sigma) {
    const int M = p.n[2] / 2;
    const int nb = fast_c2r_step_lines<T>(p);
    if (!nb) return false;
    if (ycar && (phi_out || !fast_c2r_step_yfused_ok<T>(p))) return false;
    const cx_coef k = cn_kappa(p, 2, false);
    const cx<double> kappa = {k.re, k.im};
    const cx_coef ky = cn_kappa(p, 1, false);
    const cx<double> kappay = {ky.re, ky.im};
    Phys2 ph{p.dt_nl, p.g, p.gd, amp, p.imag ? 1 : 0, p.n[0] / 2, p.n[1] / 2, p.n[2] / 2,
             p.d[0], p.d[1], p.d[2], 0.5 * p.trap[0] * p.trap[0], 0.5 * p.trap[1] * p.trap[1],
             0.5 * p.trap[2] * p.trap[2]};
    // the compiled pass applies sigma only in imaginary time
    if (sigma && !p.imag) return false;
    const double b2 = (p.imag && sizeof(T) == 4) ? 1.4426950408889634 : 1.0;  // log2(e)
    const double ka = b2 * p.dt_nl * amp;
    const NlConst nl{ka * ph.cx * p.d[0] * p.d[0], ka * ph.cy * p.d[1] * p.d[1],
                     ka * ph.cz * p.d[2] * p.d[2], b2 * p.dt_nl * p.g, b2 * p.dt_nl * p.gd};
    const cx<double>* tab = (const cx<double>*)p.cntab[2][0];
    const cx<double>* ytab = (const cx<double>*)p.cntab[1][0];
    const int blocks = p.n[0] * (p.n[1] / nb);
    switch (M) {
#define DGPE_LAUNCH(A, B, RCV, PHIV, YFV)                                                           \
    hipLaunchKernelGGL((k_c2r_step2<T, A, B, 16, RCV, PHIV, YFV>), dim3(blocks),                   \
                       dim3(step2_threads<T, A, B, 16>()), 0, p.stream, (const cx<T>*)psi_in,       \
                       (cx<T>*)psi_out, (T*)phi_out,                                                \
                       (const cx<T>*)p.spec, p.n[0], p.n[1], (const cx<T>*)p.tw[2],                \
                       (const cx<T>*)p.twr2c, tab, kappa, sigma, ph, nl, ytab, kappay, (cx<T>*)ycar, \
                       phi_sigma ? 1 : 0)
#define DGPE_CASE(A, B)                                         \
    case A * B:                                                 \
        if (p.imag) {                                           \
            if (ycar) DGPE_LAUNCH(A, B, true, false, true);     \
            else if (phi_out) DGPE_LAUNCH(A, B, true, true, false); \
            else DGPE_LAUNCH(A, B, true, false, false);         \
        } else {                                                \
            if (phi_out) DGPE_LAUNCH(A, B, false, true, false); \
            else DGPE_LAUNCH(A, B, false, false, false);        \
        }                                                       \
        return true;
        DGPE_STEP_SPLITS(DGPE_CASE)
#undef DGPE_CASE
#undef DGPE_LAUNCH
        default: return false;
    }
}

#define DGPE_INST(T)                                                 \
    template bool fast_rows<T>(const Plan&, bool, const double*, int, double*); \
    template bool fast_xmul<T>(const Plan&);                         \
    template bool fast_r2c<T>(const Plan&, const void*, const double*); \
    template bool fast_r2c_adj<T>(const Plan&, const void*, const void*, const void*, double, \
                                  double*, int*);                   \
    template bool fast_c2r_phi<T>(const Plan&, void*);               \
    template bool fast_c2r_nl<T>(const Plan&, void*, double, double, double*, int*); \
    template bool fast_c2r_adjupd<T>(const Plan&, void*, const void*, const void*, double, bool, \
                                     bool*);                                                      \
    template bool fast_c2r_step<T>(const Plan&, const void*, void*, const double*, double, void*, \
                                   void*, bool);                                                  \
    template bool fast_rows_sigma_ok<T>(const Plan&);                                             \
    template bool fast_c2r_step_yfused_ok<T>(const Plan&);
DGPE_INST(float)
DGPE_INST(double)
#undef DGPE_INST

}  // namespace dgpe
