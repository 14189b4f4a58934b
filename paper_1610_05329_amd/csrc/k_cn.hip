// Crank-Nicolson kinetic sweeps (paper, program summary, "Solution method":
// split-step Crank-Nicolson) as batched tridiagonal solves on gfx950.
//
// Strided axes (y: stride Nz, x: stride Ny*Nz): lanes take adjacent columns
// (adjacent z, or adjacent (y, z)), so every load and store of a wave is one
// contiguous run; the waves of a block take consecutive segments of the same
// lines and exchange only carries through LDS (exact segmented Thomas).
// The z axis (contiguous lines) is solved inside the fused spectral pass; the
// standalone z kernel here serves the adjoint.
#include "dgpe_device.h"

namespace dgpe {

namespace {

constexpr int kMaxThreads = 1024;

template <typename T, int S>
__global__ void __launch_bounds__(kMaxThreads)
    k_cn_strided(cx<T>* __restrict__ f, int L, int C, int logZB, int nseg,
                 const cx<T>* __restrict__ tab, cx<T> A, double* __restrict__ norm_partials) {
    __shared__ cx<T> s_first[kMaxThreads];
    __shared__ cx<T> s_last[kMaxThreads];
    __shared__ cx<T> s_dl[kMaxThreads];
    __shared__ double s_red[kMaxThreads / 64];
    const int tid = threadIdx.x;
    const int ZB = 1 << logZB;
    const int ncb = C >> logZB;
    const int o = blockIdx.x / ncb;
    const int c0 = (blockIdx.x - o * ncb) << logZB;
    const int cl = tid & (ZB - 1);
    const int seg = tid >> logZB;
    const int e0 = seg * S;
    const int cnt = (seg < nseg) ? min(S, L - e0) : 0;
    cx<T>* base = f + (size_t)o * L * C + c0 + cl;
    cx<T> v[S];
    cx<T> lastv = {T(0), T(0)};
#pragma unroll
    for (int i = 0; i < S; ++i)
        if (i < cnt) v[i] = base[(size_t)(e0 + i) * C];
#pragma unroll
    for (int i = 0; i < S; ++i)
        if (i == cnt - 1) lastv = v[i];
    if (cnt > 0) {
        s_first[seg * ZB + cl] = v[0];
        s_last[seg * ZB + cl] = lastv;
    }
    __syncthreads();
    cx<T> left = {T(0), T(0)}, right = {T(0), T(0)};
    if (cnt > 0) {
        if (seg > 0) left = s_last[(seg - 1) * ZB + cl];
        if (seg + 1 < nseg) right = s_first[(seg + 1) * ZB + cl];
    }
    // s_first is only rewritten (as the backward carries) after the solver's
    // first barrier, by which time every neighbour read above has completed.
    cn_segment_solve<T, S>(v, cnt, left, right, A, tab, L, e0, seg, nseg, s_dl, s_first, cl, ZB);
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < S; ++i) {
        if (i < cnt) {
            base[(size_t)(e0 + i) * C] = v[i];
            acc += double(abs2(v[i]));
        }
    }
    if (norm_partials) {
        const double s = block_sum(acc, s_red);
        if (tid == 0) norm_partials[blockIdx.x] = s;
    }
}

// Standalone z sweep of B = 2^logB contiguous lines, staged through LDS.
template <typename T, int SZ>
__global__ void __launch_bounds__(256) k_cn_z(cx<T>* __restrict__ f, int Nz, int logB, int ES,
                                             const cx<T>* __restrict__ tab, cx<T> A) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* P = reinterpret_cast<cx<T>*>(smem_raw);
    const int B = 1 << logB;
    const int nseg = (Nz + SZ - 1) / SZ;
    cx<T>* dl = P + Nz * ES;
    cx<T>* xf = dl + nseg * B;
    const int tid = threadIdx.x, nthr = blockDim.x;
    cx<T>* base = f + (size_t)blockIdx.x * B * Nz;
    const int total = B * Nz;
    for (int g = tid; g < total; g += nthr) {
        const int b = g / Nz, e = g - b * Nz;
        P[e * ES + b] = base[g];
    }
    __syncthreads();
    const int bl = tid & (B - 1);
    const int seg = tid >> logB;
    const int e0 = seg * SZ;
    const int cnt = (seg < nseg) ? min(SZ, Nz - e0) : 0;
    cx<T> v[SZ];
    cx<T> left = {T(0), T(0)}, right = {T(0), T(0)};
    if (cnt > 0) {
#pragma unroll
        for (int i = 0; i < SZ; ++i)
            if (i < cnt) v[i] = P[(e0 + i) * ES + bl];
        if (e0 > 0) left = P[(e0 - 1) * ES + bl];
        if (e0 + cnt < Nz) right = P[(e0 + cnt) * ES + bl];
    }
    cn_segment_solve<T, SZ>(v, cnt, left, right, A, tab, Nz, e0, seg, nseg, dl, xf, bl, B);
    if (cnt > 0) {
#pragma unroll
        for (int i = 0; i < SZ; ++i)
            if (i < cnt) P[(e0 + i) * ES + bl] = v[i];
    }
    __syncthreads();
    for (int g = tid; g < total; g += nthr) {
        const int b = g / Nz, e = g - b * Nz;
        base[g] = P[e * ES + b];
    }
}

template <typename T>
cx<T> cn_coef(const Plan& p, int axis, bool conjugate) {
    const double a = p.dt / (4.0 * p.d[axis] * p.d[axis]);
    if (p.imag) return cx<T>{T(a), T(0)};
    return cx<T>{T(0), T(conjugate ? -a : a)};
}

}  // namespace

int cn_strided_blocks(const Plan& p, int axis) {
    const int zb = 1 << p.lc.logZB[axis];
    if (axis == 1) return p.n[0] * (p.n[2] / zb);
    return (p.n[1] * p.n[2]) / zb;
}

template <typename T>
hipError_t launch_cn_strided(const Plan& p, void* f, int axis, bool conjugate,
                             double* norm_partials) {
    const int L = p.n[axis];
    const int C = (axis == 1) ? p.n[2] : p.n[1] * p.n[2];
    const int S = p.lc.seg[axis];
    const int logZB = p.lc.logZB[axis];
    const int nseg = (L + S - 1) / S;
    const int threads = nseg << logZB;
    const cx<T>* tab = (const cx<T>*)p.cntab[axis][conjugate ? 1 : 0];
    const cx<T> A = cn_coef<T>(p, axis, conjugate);
    const int blocks = cn_strided_blocks(p, axis);
#define DGPE_CN(SV)                                                                               \
    hipLaunchKernelGGL((k_cn_strided<T, SV>), dim3(blocks), dim3(threads), 0, p.stream, (cx<T>*)f, \
                       L, C, logZB, nseg, tab, A, norm_partials)
    if (S == 8) DGPE_CN(8);
    else if (S == 16) DGPE_CN(16);
    else if (S == 32) DGPE_CN(32);
    else return hipErrorInvalidValue;
#undef DGPE_CN
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cn_z(const Plan& p, void* f, bool conjugate) {
    const int Nz = p.n[2];
    const int logB = p.lc.logB_z;
    const int B = 1 << logB;
    const int es = B + 1;
    const int S = p.lc.seg[2];
    const int nseg = (Nz + S - 1) / S;
    const size_t sm = (size_t)(Nz * es + 2 * nseg * B) * sizeof(cx<T>);
    const int blocks = (p.n[0] * p.n[1]) >> logB;
    const cx<T>* tab = (const cx<T>*)p.cntab[2][conjugate ? 1 : 0];
    const cx<T> A = cn_coef<T>(p, 2, conjugate);
#define DGPE_CNZ(SV)                                                                             \
    hipLaunchKernelGGL((k_cn_z<T, SV>), dim3(blocks), dim3(p.lc.threads), sm, p.stream, (cx<T>*)f, \
                       Nz, logB, es, tab, A)
    if (S == 8) DGPE_CNZ(8);
    else if (S == 16) DGPE_CNZ(16);
    else if (S == 32) DGPE_CNZ(32);
    else return hipErrorInvalidValue;
#undef DGPE_CNZ
    return hipGetLastError();
}

#define DGPE_INST(T)                                                                  \
    template hipError_t launch_cn_strided<T>(const Plan&, void*, int, bool, double*); \
    template hipError_t launch_cn_z<T>(const Plan&, void*, bool);
DGPE_INST(float)
DGPE_INST(double)
#undef DGPE_INST

}  // namespace dgpe
