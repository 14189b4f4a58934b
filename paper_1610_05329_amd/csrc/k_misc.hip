// Pointwise and reduction kernels: imaginary-time renormalisation, the
// observables (norm, chemical potential, energy parts, rms sizes), the
// deterministic FP64 reductions and the pointwise parts of the adjoint step.
#include "dgpe_device.h"

namespace dgpe {

namespace {

constexpr int kRedThreads = 256;
constexpr int kObsWidth = 10;

struct Geo {
    int nx, ny, nz;
    int hx, hy, hz;
    double dx, dy, dz;
    double cx, cy, cz;  // trap_a^2 / 2
};

Geo geo_of(const Plan& p) {
    Geo g;
    g.nx = p.n[0];
    g.ny = p.n[1];
    g.nz = p.n[2];
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

__device__ __forceinline__ void coords(const Geo& g, size_t idx, int& ix, int& iy, int& iz) {
    iz = int(idx % g.nz);
    const size_t r = idx / g.nz;
    iy = int(r % g.ny);
    ix = int(r / g.ny);
}

// psi <- sqrt(sigma) psi (the pending imaginary-time normalisation)
template <typename T>
__global__ void k_scale(cx<T>* __restrict__ psi, size_t n, const double* __restrict__ sigma) {
    const T s = T(sqrt(sigma[0]));
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        psi[i] = s * psi[i];
}

// Per-block partial sums of the observables, FP64:
//   [0] sum n  [1..3] sum |psi_{i+1} - psi_i|^2 along x, y, z (ghost zeros)
//   [4] sum V0 n  [5] sum n^2  [6] sum Phi n  [7..9] sum x^2 n, y^2 n, z^2 n
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
    k_observables(const cx<T>* __restrict__ psi, const T* __restrict__ phi, Geo g,
                  double* __restrict__ partials) {
    __shared__ double red[kRedThreads / 64];
    double acc[kObsWidth];
#pragma unroll
    for (int q = 0; q < kObsWidth; ++q) acc[q] = 0.0;
    const size_t nt = (size_t)g.nx * g.ny * g.nz;
    const size_t sy = g.nz, sx = (size_t)g.ny * g.nz;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nt;
         i += (size_t)gridDim.x * blockDim.x) {
        int ix, iy, iz;
        coords(g, i, ix, iy, iz);
        const cx<T> pt = psi[i];
        const double pr = pt.x, pi = pt.y;
        const double n = pr * pr + pi * pi;
        double dr, di;
        const cx<T> zz = (iz + 1 < g.nz) ? psi[i + 1] : cx<T>{T(0), T(0)};
        dr = double(zz.x) - pr;
        di = double(zz.y) - pi;
        acc[3] += dr * dr + di * di + (iz == 0 ? n : 0.0);
        const cx<T> yy = (iy + 1 < g.ny) ? psi[i + sy] : cx<T>{T(0), T(0)};
        dr = double(yy.x) - pr;
        di = double(yy.y) - pi;
        acc[2] += dr * dr + di * di + (iy == 0 ? n : 0.0);
        const cx<T> xx = (ix + 1 < g.nx) ? psi[i + sx] : cx<T>{T(0), T(0)};
        dr = double(xx.x) - pr;
        di = double(xx.y) - pi;
        acc[1] += dr * dr + di * di + (ix == 0 ? n : 0.0);
        const double x = (ix - g.hx) * g.dx, y = (iy - g.hy) * g.dy, z = (iz - g.hz) * g.dz;
        const double x2 = x * x, y2 = y * y, z2 = z * z;
        acc[0] += n;
        acc[4] += (g.cx * x2 + g.cy * y2 + g.cz * z2) * n;
        acc[5] += n * n;
        acc[6] += double(phi[i]) * n;
        acc[7] += x2 * n;
        acc[8] += y2 * n;
        acc[9] += z2 * n;
    }
#pragma unroll
    for (int q = 0; q < kObsWidth; ++q) {
        const double s = block_sum(acc[q], red);
        if (threadIdx.x == 0) partials[(size_t)blockIdx.x * kObsWidth + q] = s;
    }
}

// out[w] = sum_b partials[b][w]: each thread a strided Neumaier sum, then a
// fixed tree; identical inputs give bitwise identical outputs.  Block j reduces
// the j-th set of partials (at partials + j * set_stride) into out + j * width.
__global__ void __launch_bounds__(kRedThreads)
    k_reduce(const double* __restrict__ partials, int nblocks, int width, double* __restrict__ out,
             double* __restrict__ sigma_out, double dV, size_t set_stride) {
    __shared__ double ss[kRedThreads];
    partials += blockIdx.x * set_stride;
    if (out) out += (size_t)blockIdx.x * width;
    if (blockIdx.x > 0) sigma_out = nullptr;
    constexpr int kBatch = 8;  // loads in flight per thread before the adds
    for (int w = 0; w < width; ++w) {
        double s = 0.0, c = 0.0;
        for (int b0 = threadIdx.x; b0 < nblocks; b0 += kBatch * kRedThreads) {
            double vb[kBatch];
#pragma unroll
            for (int j = 0; j < kBatch; ++j) {
                const int b = b0 + j * kRedThreads;
                vb[j] = b < nblocks ? partials[(size_t)b * width + w] : 0.0;
            }
#pragma unroll
            for (int j = 0; j < kBatch; ++j) {
                if (b0 + j * kRedThreads >= nblocks) break;
                const double v = vb[j];
                const double t = s + v;
                c += (fabs(s) >= fabs(v)) ? (s - t) + v : (v - t) + s;
                s = t;
            }
        }
        ss[threadIdx.x] = s + c;
        __syncthreads();
        for (int h = kRedThreads / 2; h > 0; h >>= 1) {
            if (threadIdx.x < h) ss[threadIdx.x] += ss[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (out) out[w] = ss[0];
            if (w == 0 && sigma_out) sigma_out[0] = 1.0 / (ss[0] * dV);
        }
        __syncthreads();
    }
}

// Adjoint of the nonlinear step: with theta = dt (a V0 + g|psi_n|^2 + gd Phi_n),
// psi' = exp(-i theta) psi_n, s = Im(conj(mu) psi'), w = dt (g s + gd Phi_s):
//   lam <- exp(+i theta) mu + 2 w psi_n      (lam holds mu on entry)
template <typename T>
__global__ void k_adj_update(cx<T>* __restrict__ lam, const cx<T>* __restrict__ psin,
                             const T* __restrict__ phin, const T* __restrict__ phis, Geo g,
                             double dt, double gg, double gdd, double amp) {
    const size_t nt = (size_t)g.nx * g.ny * g.nz;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nt;
         i += (size_t)gridDim.x * blockDim.x) {
        int ix, iy, iz;
        coords(g, i, ix, iy, iz);
        const T x = T(ix - g.hx) * T(g.dx), y = T(iy - g.hy) * T(g.dy), z = T(iz - g.hz) * T(g.dz);
        const T v0 = T(g.cx) * x * x + T(g.cy) * y * y + T(g.cz) * z * z;
        const cx<T> pn = psin[i], m = lam[i];
        const T th = T(dt) * (T(amp) * v0 + T(gg) * abs2(pn) + T(gdd) * phin[i]);
        T sn, cs;
        sin_cos(th, &sn, &cs);
        const cx<T> pp = {pn.x * cs + pn.y * sn, pn.y * cs - pn.x * sn};
        const T s = m.x * pp.y - m.y * pp.x;
        const T w = T(dt) * (T(gg) * s + T(gdd) * phis[i]);
        lam[i] = cx<T>{m.x * cs - m.y * sn + T(2) * w * pn.x, m.y * cs + m.x * sn + T(2) * w * pn.y};
    }
}

// Energy seed lam_N = 2 dV (-1/2 Lap_D + a V0 + g n + gd Phi) psi_N and the
// partial sums of V0 n, x^2 n, y^2 n, z^2 n for the direct trap derivatives.
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
    k_adj_seed(cx<T>* __restrict__ lam, const cx<T>* __restrict__ psi, const T* __restrict__ phi,
               Geo g, double gg, double gdd, double amp, double* __restrict__ partials) {
    __shared__ double red[kRedThreads / 64];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const size_t nt = (size_t)g.nx * g.ny * g.nz;
    const size_t sy = g.nz, sx = (size_t)g.ny * g.nz;
    const double dV = g.dx * g.dy * g.dz;
    const double ix2 = 1.0 / (g.dx * g.dx), iy2 = 1.0 / (g.dy * g.dy), iz2 = 1.0 / (g.dz * g.dz);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nt;
         i += (size_t)gridDim.x * blockDim.x) {
        int ix, iy, iz;
        coords(g, i, ix, iy, iz);
        const cx<T> zero = {T(0), T(0)};
        const cx<T> c = psi[i];
        const cx<T> zm = iz > 0 ? psi[i - 1] : zero, zp = iz + 1 < g.nz ? psi[i + 1] : zero;
        const cx<T> ym = iy > 0 ? psi[i - sy] : zero, yp = iy + 1 < g.ny ? psi[i + sy] : zero;
        const cx<T> xm = ix > 0 ? psi[i - sx] : zero, xp = ix + 1 < g.nx ? psi[i + sx] : zero;
        const double lr = (double(xm.x) + xp.x - 2.0 * c.x) * ix2 + (double(ym.x) + yp.x - 2.0 * c.x) * iy2 +
                          (double(zm.x) + zp.x - 2.0 * c.x) * iz2;
        const double li = (double(xm.y) + xp.y - 2.0 * c.y) * ix2 + (double(ym.y) + yp.y - 2.0 * c.y) * iy2 +
                          (double(zm.y) + zp.y - 2.0 * c.y) * iz2;
        const double x = (ix - g.hx) * g.dx, y = (iy - g.hy) * g.dy, z = (iz - g.hz) * g.dz;
        const double v0 = g.cx * x * x + g.cy * y * y + g.cz * z * z;
        const double n = double(c.x) * c.x + double(c.y) * c.y;
        const double pot = amp * v0 + gg * n + gdd * double(phi[i]);
        lam[i] = cx<T>{T(2.0 * dV * (-0.5 * lr + pot * c.x)), T(2.0 * dV * (-0.5 * li + pot * c.y))};
        acc[0] += v0 * n;
        acc[1] += x * x * n;
        acc[2] += y * y * n;
        acc[3] += z * z * n;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double s = block_sum(acc[q], red);
        if (threadIdx.x == 0) partials[(size_t)blockIdx.x * 4 + q] = s;
    }
}

// The nonlinear step on its own (the half steps of the symmetric scheme):
// theta = dt (a V0 + g |psi|^2 + gd Phi) from the state's own density;
// psi <- psi exp(-theta) with per-block FP64 sums of |psi'|^2 (imaginary time)
// or psi <- psi exp(-i theta) (real time).  Phi is the potential of |psi|^2.
template <typename T, bool IMAG>
__global__ void __launch_bounds__(kRedThreads)
    k_nonlinear(cx<T>* __restrict__ psi, const T* __restrict__ phi, Geo g, double dt, double gg,
                double gdd, double amp, double* __restrict__ partials) {
    __shared__ double red[kRedThreads / 64];
    double acc = 0.0;
    const size_t nt = (size_t)g.nx * g.ny * g.nz;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nt;
         i += (size_t)gridDim.x * blockDim.x) {
        int ix, iy, iz;
        coords(g, i, ix, iy, iz);
        const T x = T(ix - g.hx) * T(g.dx), y = T(iy - g.hy) * T(g.dy), z = T(iz - g.hz) * T(g.dz);
        const T v0 = T(g.cx) * x * x + T(g.cy) * y * y + T(g.cz) * z * z;
        const cx<T> u = psi[i];
        const T th = T(dt) * (T(amp) * v0 + T(gg) * abs2(u) + T(gdd) * phi[i]);
        cx<T> w;
        if (IMAG) {
            const T e = exp(-th);
            w = cx<T>{u.x * e, u.y * e};
            acc += double(w.x) * w.x + double(w.y) * w.y;
        } else {
            w = rotate_phase(u, th);
        }
        psi[i] = w;
    }
    if (IMAG) {
        const double s = block_sum(acc, red);
        if (threadIdx.x == 0) partials[blockIdx.x] = s;
    }
}

// n = |psi|^2 with FP64 products, rounded once to the plan precision
template <typename T>
__global__ void k_density(const cx<T>* __restrict__ psi, T* __restrict__ out, size_t nt) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nt;
         i += (size_t)gridDim.x * blockDim.x) {
        const cx<T> u = psi[i];
        out[i] = T(double(u.x) * double(u.x) + double(u.y) * double(u.y));
    }
}

// partial sums of conj(target) psi (re, im)
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
    k_overlap(const cx<T>* __restrict__ tgt, const cx<T>* __restrict__ psi, size_t nt,
              double* __restrict__ partials) {
    __shared__ double red[kRedThreads / 64];
    double re = 0.0, im = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nt;
         i += (size_t)gridDim.x * blockDim.x) {
        const cx<T> t = tgt[i], p = psi[i];
        re += double(t.x) * p.x + double(t.y) * p.y;
        im += double(t.x) * p.y - double(t.y) * p.x;
    }
    const double a = block_sum(re, red);
    if (threadIdx.x == 0) partials[(size_t)blockIdx.x * 2] = a;
    const double b = block_sum(im, red);
    if (threadIdx.x == 0) partials[(size_t)blockIdx.x * 2 + 1] = b;
}

// lam = coef * target, coef = 2 dV c (complex, host value)
template <typename T>
__global__ void k_overlap_seed(cx<T>* __restrict__ lam, const cx<T>* __restrict__ tgt, size_t nt,
                               double cr, double ci) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nt;
         i += (size_t)gridDim.x * blockDim.x) {
        const cx<T> t = tgt[i];
        lam[i] = cx<T>{T(cr * t.x - ci * t.y), T(cr * t.y + ci * t.x)};
    }
}

inline int grid_for(size_t n, int threads, int cap) {
    size_t b = (n + threads - 1) / threads;
    return (int)std::max<size_t>(1, std::min<size_t>(b, cap));
}

}  // namespace

int observables_blocks(const Plan& p) {
    const size_t nt = (size_t)p.n[0] * p.n[1] * p.n[2];
    return grid_for(nt, kRedThreads, 2048);
}

template <typename T>
hipError_t launch_scale(const Plan& p, void* psi, const double* sigma) {
    const size_t nt = (size_t)p.n[0] * p.n[1] * p.n[2];
    hipLaunchKernelGGL((k_scale<T>), dim3(grid_for(nt, 256, 16384)), dim3(256), 0, p.stream,
                       (cx<T>*)psi, nt, sigma);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_observables(const Plan& p, const void* psi, const void* phi, double amp,
                              double* partials, int* nblocks) {
    (void)amp;
    const int nb = observables_blocks(p);
    *nblocks = nb;
    hipLaunchKernelGGL((k_observables<T>), dim3(nb), dim3(kRedThreads), 0, p.stream,
                       (const cx<T>*)psi, (const T*)phi, geo_of(p), partials);
    return hipGetLastError();
}

hipError_t launch_reduce(const Plan& p, const double* partials, int nblocks, int width, double* out,
                         double* sigma_out, int nsets, size_t set_stride) {
    hipLaunchKernelGGL(k_reduce, dim3(nsets), dim3(kRedThreads), 0, p.stream, partials, nblocks,
                       width, out, sigma_out, p.d[0] * p.d[1] * p.d[2], set_stride);
    return hipGetLastError();
}

hipError_t launch_norm_finalize(const Plan& p, const double* partials, int nblocks, double* sigma) {
    return launch_reduce(p, partials, nblocks, 1, nullptr, sigma);
}

template <typename T>
hipError_t launch_adj_update(const Plan& p, void* lam, const void* psin, const void* phin,
                             const void* phis, double amp) {
    const size_t nt = (size_t)p.n[0] * p.n[1] * p.n[2];
    hipLaunchKernelGGL((k_adj_update<T>), dim3(grid_for(nt, 256, 16384)), dim3(256), 0, p.stream,
                       (cx<T>*)lam, (const cx<T>*)psin, (const T*)phin, (const T*)phis, geo_of(p),
                       p.dt, p.g, p.gd, amp);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_seed(const Plan& p, void* lam, const void* psi, const void* phi, double amp,
                           double* partials, int* nblocks) {
    const int nb = observables_blocks(p);
    *nblocks = nb;
    hipLaunchKernelGGL((k_adj_seed<T>), dim3(nb), dim3(kRedThreads), 0, p.stream, (cx<T>*)lam,
                       (const cx<T>*)psi, (const T*)phi, geo_of(p), p.g, p.gd, amp, partials);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_overlap(const Plan& p, const void* target, const void* psi, double* partials,
                          int* nblocks) {
    const size_t nt = (size_t)p.n[0] * p.n[1] * p.n[2];
    const int nb = observables_blocks(p);
    *nblocks = nb;
    hipLaunchKernelGGL((k_overlap<T>), dim3(nb), dim3(kRedThreads), 0, p.stream,
                       (const cx<T>*)target, (const cx<T>*)psi, nt, partials);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_overlap_seed(const Plan& p, void* lam, const void* target, const double* coef) {
    const size_t nt = (size_t)p.n[0] * p.n[1] * p.n[2];
    hipLaunchKernelGGL((k_overlap_seed<T>), dim3(grid_for(nt, 256, 16384)), dim3(256), 0, p.stream,
                       (cx<T>*)lam, (const cx<T>*)target, nt, coef[0], coef[1]);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_nonlinear(const Plan& p, void* psi, const void* phi, double dt, double amp,
                            double* partials, int* nblocks) {
    const int nb = observables_blocks(p);
    if (nblocks) *nblocks = nb;
    if (p.imag)
        hipLaunchKernelGGL((k_nonlinear<T, true>), dim3(nb), dim3(kRedThreads), 0, p.stream,
                           (cx<T>*)psi, (const T*)phi, geo_of(p), dt, p.g, p.gd, amp, partials);
    else
        hipLaunchKernelGGL((k_nonlinear<T, false>), dim3(nb), dim3(kRedThreads), 0, p.stream,
                           (cx<T>*)psi, (const T*)phi, geo_of(p), dt, p.g, p.gd, amp, partials);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_density(const Plan& p, const void* psi, void* out) {
    const size_t nt = (size_t)p.n[0] * p.n[1] * p.n[2];
    hipLaunchKernelGGL((k_density<T>), dim3(grid_for(nt, 256, 16384)), dim3(256), 0, p.stream,
                       (const cx<T>*)psi, (T*)out, nt);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(const Plan& p, void* dst, const void* src) {
    const size_t nt = (size_t)p.n[0] * p.n[1] * p.n[2];
    return hipMemcpyAsync(dst, src, nt * sizeof(cx<T>), hipMemcpyDeviceToDevice, p.stream);
}

#define DGPE_INST(T)                                                                              \
    template hipError_t launch_scale<T>(const Plan&, void*, const double*);                       \
    template hipError_t launch_observables<T>(const Plan&, const void*, const void*, double,      \
                                              double*, int*);                                     \
    template hipError_t launch_adj_update<T>(const Plan&, void*, const void*, const void*,        \
                                             const void*, double);                                \
    template hipError_t launch_adj_seed<T>(const Plan&, void*, const void*, const void*, double,  \
                                           double*, int*);                                        \
    template hipError_t launch_overlap<T>(const Plan&, const void*, const void*, double*, int*);  \
    template hipError_t launch_overlap_seed<T>(const Plan&, void*, const void*, const double*);   \
    template hipError_t launch_nonlinear<T>(const Plan&, void*, const void*, double, double,       \
                                            double*, int*);                                       \
    template hipError_t launch_density<T>(const Plan&, const void*, void*);                       \
    template hipError_t launch_copy<T>(const Plan&, void*, const void*);
DGPE_INST(float)
DGPE_INST(double)
#undef DGPE_INST

}  // namespace dgpe
