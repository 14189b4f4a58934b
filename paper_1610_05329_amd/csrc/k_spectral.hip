// Spectral passes of the split step on gfx950: the dipolar potential
// Phi = IDFT[U_R DFT[n]] by the convolution theorem (paper, program summary,
// "Solution method"), with the real-to-complex transform of the real density
// and its Hermitian half spectrum ("Summary of revisions", DBEC-GP-OMP), and a
// row-column multi-dimensional FFT (DBEC-GP-MPI-CUDA package, row-column
// algorithm) done as one LDS-resident 1D pass per axis.
//
// Half spectrum layout in HBM: S[kz][x][y], kz = 0..Nz/2 slowest.  With this
// layout every pass reads and writes whole contiguous rows or row segments:
//   P1 r2c_density : z-lines of psi -> S (kz-major write, B-wide segments)
//   P2 rows (fwd)  : FFT along y of contiguous rows S[kz][x][:]
//   P3 xmul        : FFT along x (stride Ny) . U_R/Nt . inverse FFT along x
//   P4 rows (inv)  : inverse FFT along y
//   P5 c2r_step    : S -> Phi along z, nonlinear phase, z Crank-Nicolson
#include "dgpe_device.h"

namespace dgpe {

namespace {

constexpr int kEmax = 16;  // max elements per thread in an LDS FFT
constexpr int kLU = 4;     // global loads in flight per thread in tile loads

// FFT passes: occupancy hint (none: forcing 4 waves per SIMD spills)
#define DGPE_FFT_OCC

template <typename T>
struct V2 {};
template <>
struct V2<float> {
    using pair = float4;  // two complex64
};
template <>
struct V2<double> {
    using pair = double4;  // two complex128 (32 B)
};

template <typename T>
__device__ __forceinline__ void load_pair(const cx<T>* p, cx<T>& a, cx<T>& b) {
    a = p[0];
    b = p[1];
}

// Trap shape V0 = (nu^2 x^2 + lam^2 y^2 + gam^2 z^2)/2 at integer indices.
struct TrapGeo {
    int hx, hy, hz;     // N/2
    double dx, dy, dz;  // spacings
    double cx, cy, cz;  // trap_a^2 / 2
};

template <typename T>
__device__ __forceinline__ T trap_v0(const TrapGeo& g, int ix, int iy, int iz) {
    const T x = T(ix - g.hx) * T(g.dx);
    const T y = T(iy - g.hy) * T(g.dy);
    const T z = T(iz - g.hz) * T(g.dz);
    return T(g.cx) * x * x + T(g.cy) * y * y + T(g.cz) * z * z;
}

TrapGeo make_geo(const Plan& p) {
    TrapGeo g;
    g.hx = p.n[0] / 2;
    g.hy = p.n[1] / 2;
    g.hz = p.n[2] / 2;
    g.dx = p.d[0];
    g.dy = p.d[1];
    g.dz = p.d[2];
    g.cx = 0.5 * p.trap[0] * p.trap[0];
    g.cy = 0.5 * p.trap[1] * p.trap[1];
    g.cz = 0.5 * p.trap[2] * p.trap[2];
    return g;
}

struct Phys {
    double dt, g, gd, amp;
    int imag;
};

// ---------------------------------------------------------------------------
// Post-processing of the packed half-length FFT into the real-to-complex
// spectrum: with z_j = n_{2j} + i n_{2j+1} and Z = FFT_M(z), M = N/2,
//   X_k = E_k + W_N^k O_k,  E_k = (Z_k + conj Z_{M-k})/2,
//   O_k = (Z_k - conj Z_{M-k})/(2i),  k = 0..M  (Z_M = Z_0).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ cx<T> r2c_post(cx<T> zk, cx<T> zm, cx<T> w) {
    const T h = T(0.5);
    const cx<T> E = {h * (zk.x + zm.x), h * (zk.y - zm.y)};
    const cx<T> O = {h * (zk.y + zm.y), -h * (zk.x - zm.x)};
    return E + cmul(w, O);
}

// Source of the real field transformed by the z pass.
enum { SRC_DENSITY = 0, SRC_ADJ_S = 1 };

// P1 (and its adjoint twin): real field along z-lines -> half spectrum.
// Block: B = 2^logB consecutive lines (x, y0..y0+B-1), M = Nz/2.
template <typename T, int SRC>
__global__ void __launch_bounds__(256) DGPE_FFT_OCC k_r2c_z(const cx<T>* __restrict__ psi,
                                              const cx<T>* __restrict__ psin,
                                              const T* __restrict__ phin, cx<T>* __restrict__ spec,
                                              int Nx, int Ny, int Nz, int logB, int ES, FftDesc fz,
                                              const cx<T>* __restrict__ twz,
                                              const cx<T>* __restrict__ twr2c,
                                              const double* __restrict__ sigma, TrapGeo geo,
                                              Phys ph, double* __restrict__ partials) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const int M = Nz >> 1;
    cx<T>* stw = buf + M * ES;
    cx<T>* sr2c = stw + M;
    const int B = 1 << logB;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int ngy = Ny >> logB;
    const int x = blockIdx.x / ngy;
    const int y0 = (blockIdx.x - x * ngy) << logB;
    for (int i = tid; i < M; i += nthr) stw[i] = twz[i];
    for (int i = tid; i <= M; i += nthr) sr2c[i] = twr2c[i];
    const size_t line0 = (size_t)x * Ny + y0;
    const int total = B * M;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (SRC == SRC_DENSITY) {
        const T sig = sigma ? T(sigma[0]) : T(1);
        const cx<T>* base = psi + line0 * Nz;
        for (int g0 = tid; g0 < total; g0 += kLU * nthr) {
            cx<T> a[kLU], b[kLU];
#pragma unroll
            for (int u = 0; u < kLU; ++u) {
                const int g = g0 + u * nthr;
                if (g < total) load_pair(base + 2 * g, a[u], b[u]);
            }
#pragma unroll
            for (int u = 0; u < kLU; ++u) {
                const int g = g0 + u * nthr;
                if (g < total) {
                    const int bl = g / M, j = g - bl * M;
                    buf[j * ES + bl] = cx<T>{abs2(a[u]) * sig, abs2(b[u]) * sig};
                }
            }
        }
    } else {
        // adjoint source s = Im(conj(mu) exp(-i theta) psi_n),
        // theta = dt (a V0 + g |psi_n|^2 + gd Phi_n); psi holds mu here.
        const cx<T>* bm = psi + line0 * Nz;
        const cx<T>* bp = psin + line0 * Nz;
        const T* bf = phin + line0 * Nz;
        const T dt = T(ph.dt), gg = T(ph.g), gdd = T(ph.gd), amp = T(ph.amp);
        for (int g = tid; g < total; g += nthr) {
            const int bl = g / M, j = g - bl * M;
            T sv[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int idx = 2 * g + h;
                const int iz = 2 * j + h;
                const cx<T> m = bm[idx], pn = bp[idx];
                const T v0 = trap_v0<T>(geo, x, y0 + bl, iz);
                const T th = dt * (amp * v0 + gg * abs2(pn) + gdd * bf[idx]);
                T sn, cs;
                sin_cos(th, &sn, &cs);
                const cx<T> pp = {pn.x * cs + pn.y * sn, pn.y * cs - pn.x * sn};
                const T s = m.x * pp.y - m.y * pp.x;  // Im(conj(m) pp)
                sv[h] = s;
                const double xx = double(x - geo.hx) * geo.dx;
                const double yy = double(y0 + bl - geo.hy) * geo.dy;
                const double zz = double(iz - geo.hz) * geo.dz;
                acc[0] += double(s) * double(v0);
                acc[1] += double(s) * xx * xx;
                acc[2] += double(s) * yy * yy;
                acc[3] += double(s) * zz * zz;
            }
            buf[j * ES + bl] = cx<T>{sv[0], sv[1]};
        }
    }
    __syncthreads();
    lds_fft<T, false, kEmax>(buf, ES, fz, logB, stw, tid, nthr);
    const size_t plane = (size_t)Nx * Ny;
    const int nout = (M + 1) << logB;
    for (int g = tid; g < nout; g += nthr) {
        const int k = g >> logB, bl = g & (B - 1);
        const cx<T> zk = buf[(k == M ? 0 : k) * ES + bl];
        const cx<T> zm = buf[(k == 0 ? 0 : M - k) * ES + bl];
        spec[(size_t)k * plane + line0 + bl] = r2c_post(zk, zm, sr2c[k]);
    }
    if (SRC == SRC_ADJ_S) {
        __shared__ double red[16];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double s = block_sum(acc[q], red);
            if (tid == 0) partials[(size_t)blockIdx.x * 4 + q] = s;
            __syncthreads();
        }
    }
}

// P2 / P4: FFT along contiguous rows of length L (the y axis of S).
template <typename T, bool INV>
__global__ void __launch_bounds__(256) DGPE_FFT_OCC k_rows(cx<T>* __restrict__ spec, int nrows, int L,
                                             FastDiv divL, int logB, int ES, FftDesc f,
                                             const cx<T>* __restrict__ tw) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    cx<T>* stw = buf + L * ES;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int B = 1 << logB;
    for (int i = tid; i < L; i += nthr) stw[i] = tw[i];
    const int r0 = blockIdx.x << logB;
    const int rows = min(B, nrows - r0);
    const int total = rows * L;
    cx<T>* base = spec + (size_t)r0 * L;
    for (int g0 = tid; g0 < total; g0 += kLU * nthr) {
        cx<T> a[kLU];
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const int g = g0 + u * nthr;
            if (g < total) a[u] = base[g];
        }
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const int g = g0 + u * nthr;
            if (g < total) {
                const int b = fdiv(g, divL), e = g - b * L;
                buf[e * ES + b] = a[u];
            }
        }
    }
    __syncthreads();
    lds_fft<T, INV, kEmax>(buf, ES, f, logB, stw, tid, nthr);
    for (int g = tid; g < total; g += nthr) {
        const int b = fdiv(g, divL), e = g - b * L;
        base[g] = buf[e * ES + b];
    }
}

// P3: FFT along x (stride Ny) of B = 2^logB adjacent columns at one kz, multiply
// by U_R(k)/Nt (real, even in kx and ky: table indexed by |kx|, |ky|), inverse
// FFT along x.
template <typename T>
__global__ void __launch_bounds__(256) DGPE_FFT_OCC k_xmul(cx<T>* __restrict__ spec, int Nx, int Ny, int logB,
                                             int ES, FftDesc fx, const cx<T>* __restrict__ tw,
                                             const T* __restrict__ ukern) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    cx<T>* stw = buf + Nx * ES;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int B = 1 << logB;
    for (int i = tid; i < Nx; i += nthr) stw[i] = tw[i];
    const int ngy = Ny >> logB;
    const int kz = blockIdx.x / ngy;
    const int y0 = (blockIdx.x - kz * ngy) << logB;
    cx<T>* base = spec + (size_t)kz * Nx * Ny + y0;
    const int total = Nx << logB;
    for (int g0 = tid; g0 < total; g0 += kLU * nthr) {
        cx<T> a[kLU];
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const int g = g0 + u * nthr;
            if (g < total) a[u] = base[(size_t)(g >> logB) * Ny + (g & (B - 1))];
        }
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const int g = g0 + u * nthr;
            if (g < total) buf[(g >> logB) * ES + (g & (B - 1))] = a[u];
        }
    }
    __syncthreads();
    lds_fft<T, false, kEmax>(buf, ES, fx, logB, stw, tid, nthr);
    const int hy = Ny / 2 + 1;
    const T* ucol = ukern + (size_t)kz * (Nx / 2 + 1) * hy;
    for (int g = tid; g < total; g += nthr) {
        const int e = g >> logB, b = g & (B - 1);
        const int kx = min(e, Nx - e), ky = min(y0 + b, Ny - y0 - b);
        const T u = ucol[(size_t)kx * hy + ky];
        cx<T>& c = buf[e * ES + b];
        c = u * c;
    }
    __syncthreads();
    lds_fft<T, true, kEmax>(buf, ES, fx, logB, stw, tid, nthr);
    for (int g = tid; g < total; g += nthr)
        base[(size_t)(g >> logB) * Ny + (g & (B - 1))] = buf[(g >> logB) * ES + (g & (B - 1))];
}

// Common front half of P5: load the half spectrum of B z-lines, pre-process
// for the packed inverse, inverse FFT of length M.  On return buf[j*ES + b]
// holds (Phi_{2j}, Phi_{2j+1}) of line b (already divided by Nt).
//   Z_k = (X_k + conj X_{M-k}) + i (X_k - conj X_{M-k}) conj(W_N^k),  k < M,
// with the imaginary parts of X_0 and X_M (zero for an exact Hermitian
// spectrum) dropped.
template <typename T>
__device__ __forceinline__ void c2r_front(cx<T>* buf, cx<T>* stw, cx<T>* sr2c,
                                          const cx<T>* __restrict__ spec,
                                          const cx<T>* __restrict__ twz,
                                          const cx<T>* __restrict__ twr2c, int Nx, int Ny, int M,
                                          int logB, int ES, const FftDesc& fz, size_t line0) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int B = 1 << logB;
    for (int i = tid; i < M; i += nthr) stw[i] = twz[i];
    for (int i = tid; i <= M; i += nthr) sr2c[i] = twr2c[i];
    const size_t plane = (size_t)Nx * Ny;
    const int total = (M + 1) << logB;
    for (int g0 = tid; g0 < total; g0 += kLU * nthr) {
        cx<T> a[kLU];
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const int g = g0 + u * nthr;
            if (g < total) a[u] = spec[(size_t)(g >> logB) * plane + line0 + (g & (B - 1))];
        }
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const int g = g0 + u * nthr;
            if (g < total) buf[(g >> logB) * ES + (g & (B - 1))] = a[u];
        }
    }
    __syncthreads();
    const int npairs = (M / 2 + 1) << logB;
    for (int g = tid; g < npairs; g += nthr) {
        const int k = g >> logB, b = g & (B - 1);
        if (k == 0) {
            const T x0 = buf[b].x, xm = buf[M * ES + b].x;
            buf[b] = cx<T>{x0 + xm, x0 - xm};
        } else {
            const int km = M - k;
            const cx<T> xa = buf[k * ES + b], xb = buf[km * ES + b];
            // Z_k
            const cx<T> s1 = xa + conj(xb);
            const cx<T> d1 = cmulc(xa - conj(xb), sr2c[k]);
            buf[k * ES + b] = cx<T>{s1.x - d1.y, s1.y + d1.x};
            if (km != k) {
                const cx<T> s2 = xb + conj(xa);
                const cx<T> d2 = cmulc(xb - conj(xa), sr2c[km]);
                buf[km * ES + b] = cx<T>{s2.x - d2.y, s2.y + d2.x};
            }
        }
    }
    __syncthreads();
    lds_fft<T, true, kEmax>(buf, ES, fz, logB, stw, tid, nthr);
}

// P5: z inverse transform -> Phi, nonlinear phase, Crank-Nicolson along z.
// LDS: F (M+1 rows) | Psi (Nz rows) | twiddles | segment carry products.
template <typename T, int SZ, bool RC, bool GUARD>
__global__ void __launch_bounds__(256) k_c2r_step(const cx<T>* psi_in, cx<T>* psi_out,
                                                 T* __restrict__ phi_out,
                                                 const cx<T>* __restrict__ spec, int Nx, int Ny,
                                                 int Nz, int logB, int ES, FftDesc fz,
                                                 const cx<T>* __restrict__ twz,
                                                 const cx<T>* __restrict__ twr2c,
                                                 const cx<double>* __restrict__ cntab,
                                                 cx<double> kappa64,
                                                 const double* __restrict__ sigma, TrapGeo geo,
                                                 Phys ph, int fcap) {
    using A = cn_acc_t<T, RC>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int M = Nz >> 1;
    const int nseg = (Nz + SZ - 1) / SZ;
    // F: the spectrum tile, later the carries; fcap >= max((M+1) ES, carries)
    cx<T>* F = reinterpret_cast<cx<T>*>(smem_raw);
    cx<T>* P = F + fcap;
    cx<T>* stw = P + Nz * ES;
    cx<T>* sr2c = stw + M;
    const size_t off = ((size_t)(fcap + Nz * ES + M + M + 1) * sizeof(cx<T>) + 15) & ~size_t(15);
    cx<A>* spe = reinterpret_cast<cx<A>*>(smem_raw + off);
    cx<A>* sqb = spe + nseg;
    const int B = 1 << logB;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int ngy = Ny >> logB;
    const int x = blockIdx.x / ngy;
    const int y0 = (blockIdx.x - x * ngy) << logB;
    const size_t line0 = (size_t)x * Ny + y0;
    for (int i = tid; i < nseg; i += nthr) {
        spe[i] = widen<A>(cntab[TAB_PEND * Nz + i]);
        sqb[i] = widen<A>(cntab[TAB_QBEG * Nz + i]);
    }
    c2r_front<T>(F, stw, sr2c, spec, twz, twr2c, Nx, Ny, M, logB, ES, fz, line0);

    // nonlinear step on the B lines (pre-step density, lazily normalised)
    const double sg = sigma ? sigma[0] : 1.0;
    const T sig = T(sg), rs = T(sqrt(sg));
    const T dt = T(ph.dt), gg = T(ph.g), gdd = T(ph.gd), amp = T(ph.amp);
    const cx<T>* base_in = psi_in + line0 * Nz;
    cx<T>* base = psi_out + line0 * Nz;
    const int total = B * Nz;
    for (int g0 = tid; g0 < total; g0 += kLU * nthr) {
        cx<T> a[kLU];
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const int g = g0 + u * nthr;
            if (g < total) a[u] = base_in[g];
        }
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const int g = g0 + u * nthr;
            if (g < total) {
                const int b = g / Nz, e = g - b * Nz;
                const cx<T> fv = F[(e >> 1) * ES + b];
                const T phi = (e & 1) ? fv.y : fv.x;
                if (phi_out) phi_out[line0 * Nz + g] = phi;  // for the adjoint
                const T n = abs2(a[u]) * sig;
                const T th = dt * (amp * trap_v0<T>(geo, x, y0 + b, e) + gg * n + gdd * phi);
                cx<T> r;
                if (ph.imag) {
                    const T f = rs * exp_of(-th);
                    r = f * a[u];
                } else {
                    r = rs * rotate_phase(a[u], th);
                }
                P[e * ES + b] = r;
            }
        }
    }
    __syncthreads();

    // Crank-Nicolson along z: thread -> (line b, segment s)
    cx<A>* dl = reinterpret_cast<cx<A>*>(F);  // F is dead now; carries reuse it
    cx<A>* xf = dl + nseg * B;
    const cx<A> kappa = {A(kappa64.x), A(kappa64.y)};
    const int bl = tid & (B - 1);
    const int seg = tid >> logB;
    const int e0 = seg * SZ;
    const int cnt = (seg < nseg) ? min(SZ, Nz - e0) : 0;
    cx<A> v[SZ];
    cx<A> left = {A(0), A(0)}, right = {A(0), A(0)};
    if (cnt > 0) {
#pragma unroll
        for (int i = 0; i < SZ; ++i)
            if (!GUARD || i < cnt) v[i] = widen<A>(P[(e0 + i) * ES + bl]);
        if (e0 > 0) left = widen<A>(P[(e0 - 1) * ES + bl]);
        if (e0 + cnt < Nz) right = widen<A>(P[(e0 + cnt) * ES + bl]);
    }
    cn_segment_solve<T, SZ, RC, GUARD>(v, cnt, left, right, kappa, cntab + TAB_ALPHA * Nz,
                                       cntab + TAB_P * Nz, cntab + TAB_Q * Nz, spe, sqb, e0, seg,
                                       nseg, dl, xf, bl, B);
    // cn_segment_solve ended with a barrier after every neighbour read
    if (cnt > 0) {
#pragma unroll
        for (int i = 0; i < SZ; ++i)
            if (!GUARD || i < cnt) P[(e0 + i) * ES + bl] = to_store<T>(v[i]);
    }
    __syncthreads();
    for (int g = tid; g < total; g += nthr) {
        const int b = g / Nz, e = g - b * Nz;
        base[g] = P[e * ES + b];
    }
}

// Phi to a real [Nx][Ny][Nz] buffer (dgpe_potential, observables, adjoint).
template <typename T>
__global__ void __launch_bounds__(256) k_c2r_phi(T* __restrict__ phi, const cx<T>* __restrict__ spec,
                                                int Nx, int Ny, int Nz, int logB, int ES, FftDesc fz,
                                                const cx<T>* __restrict__ twz,
                                                const cx<T>* __restrict__ twr2c) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int M = Nz >> 1;
    cx<T>* F = reinterpret_cast<cx<T>*>(smem_raw);
    cx<T>* stw = F + (M + 1) * ES;
    cx<T>* sr2c = stw + M;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int ngy = Ny >> logB;
    const int x = blockIdx.x / ngy;
    const int y0 = (blockIdx.x - x * ngy) << logB;
    const size_t line0 = (size_t)x * Ny + y0;
    c2r_front<T>(F, stw, sr2c, spec, twz, twr2c, Nx, Ny, M, logB, ES, fz, line0);
    T* base = phi + line0 * Nz;
    const int total = (1 << logB) * Nz;
    for (int g = tid; g < total; g += nthr) {
        const int b = g / Nz, e = g - b * Nz;
        const cx<T> fv = F[(e >> 1) * ES + b];
        base[g] = (e & 1) ? fv.y : fv.x;
    }
}

// U_R(k)/Nt on the table [kz][|kx|][ky] (plan time), FP64 math.
// Quasi-2D kernel / Nt on the table [kz][|kx|] (the grid's y axis is the
// tight one, of one point): the 3D kernel of dipoles along the tight axis
// (perp) or along z averaged over the tight trap's ground state of width l,
//   perp:     (4 pi/3)/(sqrt(2 pi) l) (2 - 3 F(u))
//   in plane: (4 pi/3)/(sqrt(2 pi) l) (-1 + 3 (kz^2/q^2) F(u)),
// u = q l / sqrt 2, F(u) = sqrt(pi) u exp(u^2) erfc(u) (erfcx: no overflow).
template <typename T>
__global__ void k_ukern_q2d(T* __restrict__ out, int Nx, int Nz, double dkx, double dkz, double ell,
                            bool perp, double inv_nt) {
    const int hx = Nx / 2 + 1, hz = Nz / 2 + 1;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= hx * hz) return;
    const int kx = i % hx, kz = i / hx;
    const double qx = kx * dkx, qz = kz * dkz;
    const double q2 = qx * qx + qz * qz;
    const double u = sqrt(q2) * ell * M_SQRT1_2;
    const double F = 1.7724538509055160273 * u * erfcx(u);  // sqrt(pi) u erfcx(u)
    const double pre = (4.0 * M_PI / 3.0) / (2.5066282746310005024 * ell);  // / (sqrt(2 pi) l)
    const double v = perp ? pre * (2.0 - 3.0 * F) : pre * (-1.0 + (q2 > 0.0 ? 3.0 * qz * qz / q2 * F : 0.0));
    out[i] = T(v * inv_nt);
}

template <typename T>
__global__ void k_ukern(T* __restrict__ out, int Nx, int Ny, int Nz, double dkx, double dky,
                        double dkz, double R, double inv_nt) {
    const int hx = Nx / 2 + 1, hy = Ny / 2 + 1, hz = Nz / 2 + 1;
    const size_t total = (size_t)hx * hy * hz;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const int ky = int(i % hy);
        const int kx = int((i / hy) % hx);
        const int kz = int(i / ((size_t)hx * hy));
        const double qx = kx * dkx, qy = ky * dky, qz = kz * dkz;
        const double k2 = qx * qx + qy * qy + qz * qz;
        double u = 0.0;
        if (k2 > 0.0) {
            const double k = sqrt(k2);
            const double t = k * R;
            double f;
            if (t < 0.1) {
                const double t2 = t * t;
                f = t2 * (1.0 / 10.0 - t2 * (1.0 / 280.0 - t2 * (1.0 / 15120.0)));
            } else {
                double s, c;
                sincos(t, &s, &c);
                f = 1.0 + 3.0 * c / (t * t) - 3.0 * s / (t * t * t);
            }
            u = (4.0 * M_PI / 3.0) * (3.0 * qz * qz / k2 - 1.0) * f * inv_nt;
        }
        out[i] = T(u);
    }
}

// stride of a line element in an LDS tile of 2^logB lines, element-major:
// one pad per element spreads the lines over the banks; a single line needs
// none (consecutive threads take consecutive elements)
inline int tile_es(int logB) { return logB == 0 ? 1 : (1 << logB) + 1; }

inline size_t sm_r2c(const Plan& p, int es, size_t csz) {
    const int M = p.n[2] / 2;
    return (size_t)(M * es + M + M + 1) * csz;
}
// capacity (in complex values of the storage type) of the spectrum tile that
// later holds the z carries (arithmetic type, at most 16 bytes each)
inline int c2r_fcap(const Plan& p, int es, size_t csz) {
    const int M = p.n[2] / 2;
    const int nseg = (p.n[2] + p.lc.seg[2] - 1) / p.lc.seg[2];
    const size_t carries = ((size_t)2 * nseg * ((size_t)1 << p.lc.logB_z) * 16 + csz - 1) / csz;
    return (int)std::max<size_t>((size_t)(M + 1) * es, carries);
}
inline size_t sm_c2r_step(const Plan& p, int es, size_t csz) {
    const int M = p.n[2] / 2;
    const int nseg = (p.n[2] + p.lc.seg[2] - 1) / p.lc.seg[2];
    const size_t off = ((size_t)(c2r_fcap(p, es, csz) + p.n[2] * es + M + M + 1) * csz + 15) & ~size_t(15);
    return off + (size_t)2 * nseg * 16;
}
inline size_t sm_c2r_phi(const Plan& p, int es, size_t csz) {
    const int M = p.n[2] / 2;
    return (size_t)((M + 1) * es + M + M + 1) * csz;
}

}  // namespace

int r2c_blocks(const Plan& p) { return p.n[0] * (p.n[1] >> p.lc.logB_z); }

template <typename T>
hipError_t launch_r2c_density(const Plan& p, const void* psi, const double* sigma) {
    if (p.fast && fast_r2c<T>(p, psi, sigma)) return hipGetLastError();
    const int es = tile_es(p.lc.logB_z);
    const size_t sm = sm_r2c(p, es, sizeof(cx<T>));
    Phys ph{};
    hipLaunchKernelGGL((k_r2c_z<T, SRC_DENSITY>), dim3(r2c_blocks(p)), dim3(p.lc.threads), sm,
                       p.stream, (const cx<T>*)psi, (const cx<T>*)nullptr, (const T*)nullptr,
                       (cx<T>*)p.spec, p.n[0], p.n[1], p.n[2], p.lc.logB_z, es, p.fz,
                       (const cx<T>*)p.tw[2], (const cx<T>*)p.twr2c, sigma, make_geo(p), ph,
                       (double*)nullptr);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_r2c_adjoint_s(const Plan& p, const void* mu, const void* psin, const void* phin,
                                double amp, double* partials, int* nblocks) {
    if (p.fast && fast_r2c_adj<T>(p, mu, psin, phin, amp, partials, nblocks)) return hipGetLastError();
    *nblocks = r2c_blocks(p);
    const int es = tile_es(p.lc.logB_z);
    const size_t sm = sm_r2c(p, es, sizeof(cx<T>));
    Phys ph{p.dt, p.g, p.gd, amp, 0};
    hipLaunchKernelGGL((k_r2c_z<T, SRC_ADJ_S>), dim3(r2c_blocks(p)), dim3(p.lc.threads), sm,
                       p.stream, (const cx<T>*)mu, (const cx<T>*)psin, (const T*)phin,
                       (cx<T>*)p.spec, p.n[0], p.n[1], p.n[2], p.lc.logB_z, es, p.fz,
                       (const cx<T>*)p.tw[2], (const cx<T>*)p.twr2c, (const double*)nullptr,
                       make_geo(p), ph, partials);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rows(const Plan& p, bool inverse, const double* npart, int nnpart,
                       double* sigma_out) {
    if (p.fast && fast_rows<T>(p, inverse, npart, nnpart, sigma_out)) return hipGetLastError();
    if (npart) return hipErrorInvalidValue;  // only the compiled pass reduces the norm
    const int L = p.n[1];
    const int es = tile_es(p.lc.logB_y);
    const int nrows = (p.n[2] / 2 + 1) * p.n[0];
    const int blocks = (nrows + (1 << p.lc.logB_y) - 1) >> p.lc.logB_y;
    const size_t sm = (size_t)(L * es + L) * sizeof(cx<T>);
    FastDiv dv{(uint32_t)L, (uint32_t)((0x100000000ull + L - 1) / L)};
    if (inverse)
        hipLaunchKernelGGL((k_rows<T, true>), dim3(blocks), dim3(p.lc.threads), sm, p.stream,
                           (cx<T>*)p.spec, nrows, L, dv, p.lc.logB_y, es, p.fy,
                           (const cx<T>*)p.tw[1]);
    else
        hipLaunchKernelGGL((k_rows<T, false>), dim3(blocks), dim3(p.lc.threads), sm, p.stream,
                           (cx<T>*)p.spec, nrows, L, dv, p.lc.logB_y, es, p.fy,
                           (const cx<T>*)p.tw[1]);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_xmul(const Plan& p) {
    if (p.fast && fast_xmul<T>(p)) return hipGetLastError();
    const int es = tile_es(p.lc.logB_x);
    const int blocks = (p.n[2] / 2 + 1) * (p.n[1] >> p.lc.logB_x);
    const size_t sm = (size_t)(p.n[0] * es + p.n[0]) * sizeof(cx<T>);
    hipLaunchKernelGGL((k_xmul<T>), dim3(blocks), dim3(p.lc.threads), sm, p.stream, (cx<T>*)p.spec,
                       p.n[0], p.n[1], p.lc.logB_x, es, p.fx, (const cx<T>*)p.tw[0],
                       (const T*)p.ukern);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_c2r_step(const Plan& p, const void* psi_in, void* psi_out, const double* sigma,
                           double amp, void* phi_out, void* ycar, bool phi_sigma) {
    if (p.fast && fast_c2r_step<T>(p, psi_in, psi_out, sigma, amp, phi_out, ycar, phi_sigma))
        return hipGetLastError();
    // only the compiled fused pass starts the y solve or scales Phi by sigma
    if (ycar || phi_sigma) return hipErrorInvalidValue;
    const int es = tile_es(p.lc.logB_z);
    const size_t sm = sm_c2r_step(p, es, sizeof(cx<T>));
    const cx_coef k = cn_kappa(p, 2, false);
    const cx<double> kappa = {k.re, k.im};
    Phys ph{p.dt_nl, p.g, p.gd, amp, p.imag ? 1 : 0};
    const cx<double>* tab = (const cx<double>*)p.cntab[2][0];
    const int S = p.lc.seg[2];
    const bool guard = (p.n[2] % S) != 0;
#define DGPE_C2R_STEP(SZV, RCV, GV)                                                                \
    hipLaunchKernelGGL((k_c2r_step<T, SZV, RCV, GV>), dim3(r2c_blocks(p)), dim3(p.lc.threads), sm, \
                       p.stream, (const cx<T>*)psi_in, (cx<T>*)psi_out, (T*)phi_out,                \
                       (const cx<T>*)p.spec, p.n[0], p.n[1], p.n[2],                                \
                       p.lc.logB_z, es, p.fz, (const cx<T>*)p.tw[2], (const cx<T>*)p.twr2c, tab,    \
                       kappa, sigma, make_geo(p), ph, c2r_fcap(p, es, sizeof(cx<T>)))
#define DGPE_C2R_S(SZV)                              \
    if (p.imag) {                                    \
        if (guard) DGPE_C2R_STEP(SZV, true, true);   \
        else DGPE_C2R_STEP(SZV, true, false);        \
    } else {                                         \
        if (guard) DGPE_C2R_STEP(SZV, false, true);  \
        else DGPE_C2R_STEP(SZV, false, false);       \
    }
    if (S == 16) { DGPE_C2R_S(16) }
    else if (S == 32) { DGPE_C2R_S(32) }
    else return hipErrorInvalidValue;
#undef DGPE_C2R_S
#undef DGPE_C2R_STEP
    return hipGetLastError();
}

template <typename T>
hipError_t launch_c2r_phi(const Plan& p, void* phi_out) {
    if (p.fast && fast_c2r_phi<T>(p, phi_out)) return hipGetLastError();
    const int es = tile_es(p.lc.logB_z);
    const size_t sm = sm_c2r_phi(p, es, sizeof(cx<T>));
    hipLaunchKernelGGL((k_c2r_phi<T>), dim3(r2c_blocks(p)), dim3(p.lc.threads), sm, p.stream,
                       (T*)phi_out, (const cx<T>*)p.spec, p.n[0], p.n[1], p.n[2], p.lc.logB_z, es,
                       p.fz, (const cx<T>*)p.tw[2], (const cx<T>*)p.twr2c);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ukern(const Plan& p) {
    const double two_pi = 2.0 * M_PI;
    if (p.q2d) {
        const int total = (p.n[0] / 2 + 1) * (p.n[2] / 2 + 1);
        const double nt = (double)p.n[0] * p.n[2];
        hipLaunchKernelGGL((k_ukern_q2d<T>), dim3((total + 255) / 256), dim3(256), 0, p.stream,
                           (T*)p.ukern, p.n[0], p.n[2], two_pi / (p.n[0] * p.d[0]),
                           two_pi / (p.n[2] * p.d[2]), 1.0 / std::sqrt(p.trap[1]), p.q2d == 1,
                           1.0 / nt);
        return hipGetLastError();
    }
    const double nt = (double)p.n[0] * p.n[1] * p.n[2];
    const size_t total = (size_t)(p.n[0] / 2 + 1) * (p.n[1] / 2 + 1) * (p.n[2] / 2 + 1);
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 65535);
    hipLaunchKernelGGL((k_ukern<T>), dim3(blocks), dim3(256), 0, p.stream, (T*)p.ukern, p.n[0],
                       p.n[1], p.n[2], two_pi / (p.n[0] * p.d[0]), two_pi / (p.n[1] * p.d[1]),
                       two_pi / (p.n[2] * p.d[2]), p.R, 1.0 / nt);
    return hipGetLastError();
}

#define DGPE_INST(T)                                                                               \
    template hipError_t launch_r2c_density<T>(const Plan&, const void*, const double*);            \
    template hipError_t launch_r2c_adjoint_s<T>(const Plan&, const void*, const void*, const void*, \
                                                double, double*, int*);                            \
    template hipError_t launch_rows<T>(const Plan&, bool, const double*, int, double*);           \
    template hipError_t launch_xmul<T>(const Plan&);                                               \
    template hipError_t launch_c2r_step<T>(const Plan&, const void*, void*, const double*, double, \
                                           void*, void*, bool); \
    template hipError_t launch_c2r_phi<T>(const Plan&, void*);                                     \
    template hipError_t launch_ukern<T>(const Plan&);
DGPE_INST(float)
DGPE_INST(double)
#undef DGPE_INST

}  // namespace dgpe
