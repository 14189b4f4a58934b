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

// Tables are complex FP64 in the workspace (see dgpe_internal.h).
struct CnTab {
    const cx<double>* a;
    const cx<double>* p;
    const cx<double>* q;
    const cx<double>* pend;
    const cx<double>* qbeg;
};

CnTab tab_of(const void* base, int N) {
    const cx<double>* t = (const cx<double>*)base;
    return CnTab{t + TAB_ALPHA * N, t + TAB_P * N, t + TAB_Q * N, t + TAB_PEND * N,
                 t + TAB_QBEG * N};
}

template <typename A>
__device__ __forceinline__ cx<A> narrow_tab(cx<double> v) { return cx<A>{A(v.x), A(v.y)}; }

// LDS: A1[nseg*ZB] | A2[nseg*ZB] (arithmetic type) | alpha | P | Q (each
// nseg*(S+1): segment s at s*(S+1), so that the segments of a wave read
// distinct banks) | pend | qbeg
template <typename T, int S, bool RC, bool GUARD>
__global__ void __launch_bounds__(sizeof(cn_acc_t<T, RC>) == 8 ? kMaxThreads / 2 : kMaxThreads)
    k_cn_strided(cx<T>* __restrict__ f, int L, int C, int logZB, int nseg, CnTab tg,
                 cx<double> kappa64, double* __restrict__ norm_partials) {
    using A = cn_acc_t<T, RC>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double s_red[kMaxThreads / 64];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int ZB = 1 << logZB;
    const int nsl = nseg << logZB;
    cx<A>* A1 = reinterpret_cast<cx<A>*>(smem_raw);
    cx<A>* A2 = A1 + nsl;
    const int TL = nseg * (S + 1);
    cx<A>* ta = A2 + nsl;
    cx<A>* tp = ta + TL;
    cx<A>* tq = tp + TL;
    cx<A>* pe = tq + TL;
    cx<A>* qb = pe + nseg;
    // First round of the table loads (one entry of each table per thread,
    // clamped: the writes below are unconditional so the loads stay ahead of
    // the state loads; see tab_stage), then the state, then staging.
    const int i0 = min(tid, L - 1), s0 = min(tid, nseg - 1);
    const cx<double> a0 = tg.a[i0], p0 = tg.p[i0], q0 = tg.q[i0];
    const cx<double> pe0 = tg.pend[s0], qb0 = tg.qbeg[s0];
    const cx<A> kappa = narrow_tab<A>(kappa64);
    const int ncb = C >> logZB;
    const int bid = xcd_swizzle(blockIdx.x, gridDim.x);
    const int o = bid / ncb;
    const int c0 = (bid - o * ncb) << logZB;
    const int cl = tid & (ZB - 1);
    const int seg = tid >> logZB;
    const int e0 = seg * S;
    const int cnt = (seg < nseg) ? min(S, L - e0) : 0;
    cx<T>* base = f + (size_t)o * L * C + c0 + cl;
    cx<A> v[S];
#pragma unroll
    for (int i = 0; i < S; ++i)
        if (!GUARD || i < cnt) v[i] = widen<A>(base[(size_t)(e0 + i) * C]);
    ta[i0 + i0 / S] = narrow_tab<A>(a0);
    tp[i0 + i0 / S] = narrow_tab<A>(p0);
    tq[i0 + i0 / S] = narrow_tab<A>(q0);
    pe[s0] = narrow_tab<A>(pe0);
    qb[s0] = narrow_tab<A>(qb0);
    for (int i = tid + nthr; i < L; i += nthr) {  // lines longer than the block
        const int ip = i + i / S;
        ta[ip] = narrow_tab<A>(tg.a[i]);
        tp[ip] = narrow_tab<A>(tg.p[i]);
        tq[ip] = narrow_tab<A>(tg.q[i]);
    }
    for (int i = tid + nthr; i < nseg; i += nthr) {
        pe[i] = narrow_tab<A>(tg.pend[i]);
        qb[i] = narrow_tab<A>(tg.qbeg[i]);
    }
    cx<A> lastv = v[S - 1];
    if (GUARD) {
#pragma unroll
        for (int i = 0; i < S; ++i)
            if (i == cnt - 1) lastv = v[i];
    }
    if (cnt > 0) {
        A1[seg * ZB + cl] = v[0];
        A2[seg * ZB + cl] = lastv;
    }
    __syncthreads();
    cx<A> left = {A(0), A(0)}, right = {A(0), A(0)};
    if (cnt > 0) {
        if (seg > 0) left = A2[(seg - 1) * ZB + cl];
        if (seg + 1 < nseg) right = A1[(seg + 1) * ZB + cl];
    }
    __syncthreads();  // neighbour reads done: A2 becomes the forward carries, A1 the backward ones
    cn_segment_solve<T, S, RC, GUARD>(v, cnt, left, right, kappa, ta, tp, tq, pe, qb, seg * (S + 1), seg,
                                      nseg, A2, A1, cl, ZB);
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < S; ++i) {
        if (!GUARD || i < cnt) {
            const cx<T> o = to_store<T>(v[i]);
            base[(size_t)(e0 + i) * C] = o;
            acc += double(abs2(o));
        }
    }
    if (norm_partials) {
        const double s = block_sum(acc, s_red);
        if (tid == 0) norm_partials[blockIdx.x] = s;
    }
}

// Standalone z sweep of B = 2^logB contiguous lines, staged through LDS.
// LDS: P (Nz rows, storage type) | carries (arithmetic type) | pend | qbeg
template <typename T, int SZ, bool RC, bool GUARD>
__global__ void __launch_bounds__(256) k_cn_z(cx<T>* __restrict__ f, int Nz, int logB, int ES,
                                             CnTab tg, cx<double> kappa64) {
    using A = cn_acc_t<T, RC>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* P = reinterpret_cast<cx<T>*>(smem_raw);
    const int B = 1 << logB;
    const int nseg = (Nz + SZ - 1) / SZ;
    cx<A>* dl = reinterpret_cast<cx<A>*>(smem_raw + (((size_t)Nz * ES * sizeof(cx<T>) + 15) & ~size_t(15)));
    cx<A>* xf = dl + nseg * B;
    cx<A>* pe = xf + nseg * B;
    cx<A>* qb = pe + nseg;
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int i = tid; i < nseg; i += nthr) {
        pe[i] = narrow_tab<A>(tg.pend[i]);
        qb[i] = narrow_tab<A>(tg.qbeg[i]);
    }
    const cx<A> kappa = narrow_tab<A>(kappa64);
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
    cx<A> v[SZ];
    cx<A> left = {A(0), A(0)}, right = {A(0), A(0)};
    if (cnt > 0) {
#pragma unroll
        for (int i = 0; i < SZ; ++i)
            if (!GUARD || i < cnt) v[i] = widen<A>(P[(e0 + i) * ES + bl]);
        if (e0 > 0) left = widen<A>(P[(e0 - 1) * ES + bl]);
        if (e0 + cnt < Nz) right = widen<A>(P[(e0 + cnt) * ES + bl]);
    }
    cn_segment_solve<T, SZ, RC, GUARD>(v, cnt, left, right, kappa, tg.a, tg.p, tg.q, pe, qb, e0,
                                          seg, nseg, dl, xf, bl, B);
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

// Standalone z sweep, fast path (Nz = 64, 128 or 256, 16-point segments):
// each wave owns LPW = 64 / nseg whole lines, loads them with coalesced
// 16-byte units, transposes them through LDS to the segment layout, solves with
// shuffle carries (the fused z pass's solver) and stores them back coalesced.
// Waves are independent after the table staging: no block barrier follows it.
template <typename T, int Nz, bool RC>
__global__ void __launch_bounds__(256) k_cn_z2(cx<T>* __restrict__ f, int nlines,
                                              const cx<double>* __restrict__ cntab,
                                              cx<double> kappa64) {
    using A = cn_acc_t<T, RC>;
    constexpr int SZ = 16;
    constexpr int NT = 256, NW = NT / 64;
    constexpr int nseg = Nz / SZ;
    constexpr int U = 16 / (int)sizeof(cx<T>);
    constexpr int KR = (64 * U) / Nz > 1 ? (64 * U) / Nz : 1;
    using WL = WaveLines<T, Nz, SZ, KR>;
    constexpr int LPW = WL::LPW, NU = WL::NU;
    constexpr int TS = Nz + Nz / SZ;
    __shared__ __align__(16) cx<T> stg[NW * KR * WL::SL];
    __shared__ cx<A> ta[TS];
    __shared__ cx<A> tp[TS];
    __shared__ cx<A> tq[TS];
    __shared__ cx<A> spe[nseg];
    __shared__ cx<A> sqb[nseg];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wl0 = (xcd_swizzle(blockIdx.x, gridDim.x) * NW + wv) * LPW;
    TabRegs<cx<double>, Nz, NT> rta, rtp, rtq;
    TabRegs<cx<double>, nseg, NT> rpe, rqb;
    tab_issue(rta, cntab + TAB_ALPHA * Nz, tid);
    tab_issue(rtp, cntab + TAB_P * Nz, tid);
    tab_issue(rtq, cntab + TAB_Q * Nz, tid);
    tab_issue(rpe, cntab + TAB_PEND * Nz, tid);
    tab_issue(rqb, cntab + TAB_QBEG * Nz, tid);
    // waves past the last line load the last wave's lines (unused)
    cx<T>* wp = f + (size_t)min(wl0, nlines - LPW) * Nz;
    cx<T> a[SZ];
#pragma unroll
    for (int j = 0; j < NU; ++j) load_unit<T>(wp + (j * 64 + lane) * U, a + j * U);
    const auto ident = [](int i) { return i; };
    const auto padded = [](int i) { return i + i / SZ; };
    tab_stage(rta, ta, tid, padded);
    tab_stage(rtp, tp, tid, padded);
    tab_stage(rtq, tq, tid, padded);
    tab_stage(rpe, spe, tid, ident);
    tab_stage(rqb, sqb, tid, ident);
    __syncthreads();
    if (wl0 >= nlines) return;  // no barrier follows
    cx<T>* st = stg + wv * KR * WL::SL;
    const int seg = lane % nseg;
    cx<A> v[SZ];
    WL::to_segments(st, a, v, lane);
    const cx<A> kappa = {A(kappa64.x), A(kappa64.y)};
    const int tb = seg * (SZ + 1);
    cn_segment_solve_wave<T, SZ, nseg, RC>(v, kappa, ta + tb, tp + tb, tq + tb, spe, sqb, seg);
    WL::store_from_segments(st, v, wp, lane);
}

}  // namespace

cx_coef cn_kappa(const Plan& p, int axis, bool conjugate) {
    // kappa = 1/A - 2 with A = dt/(4 d^2) (imaginary time) or +-i dt/(4 d^2)
    const double a = p.dt / (4.0 * p.d[axis] * p.d[axis]);
    if (p.imag) return cx_coef{1.0 / a - 2.0, 0.0};
    return cx_coef{-2.0, conjugate ? 1.0 / a : -1.0 / a};
}

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
    const CnTab tg = tab_of(p.cntab[axis][conjugate ? 1 : 0], L);
    const cx_coef k = cn_kappa(p, axis, conjugate);
    const cx<double> kappa = {k.re, k.im};
    const int blocks = cn_strided_blocks(p, axis);
    const size_t asz = (p.imag ? sizeof(T) : sizeof(double)) * 2;
    const size_t sm = (size_t)(2 * threads + 3 * nseg * (S + 1) + 2 * nseg) * asz;
    const bool guard = (L % S) != 0;
#define DGPE_CN(SV, RCV, GV)                                                                      \
    hipLaunchKernelGGL((k_cn_strided<T, SV, RCV, GV>), dim3(blocks), dim3(threads), sm, p.stream, \
                       (cx<T>*)f, L, C, logZB, nseg, tg, kappa, norm_partials)
#define DGPE_CN_S(SV)                           \
    if (p.imag) {                               \
        if (guard) DGPE_CN(SV, true, true);     \
        else DGPE_CN(SV, true, false);          \
    } else {                                    \
        if (guard) DGPE_CN(SV, false, true);    \
        else DGPE_CN(SV, false, false);         \
    }
    if (S == 16) { DGPE_CN_S(16) }
    else return hipErrorInvalidValue;
#undef DGPE_CN_S
#undef DGPE_CN
    return hipGetLastError();
}

template <typename T>
bool fast_cn_z(const Plan& p, void* f, bool conjugate) {
    const int Nz = p.n[2];
    const int nlines = p.n[0] * p.n[1];
    const int lpw = 64 / (Nz / 16);
    // the z tables hold 16-point segments when lc.seg[2] == 16
    if (!p.fast || p.lc.seg[2] != 16 || (Nz != 64 && Nz != 128 && Nz != 256) || nlines % lpw)
        return false;
    const int blocks = (nlines / lpw + 3) / 4;
    const cx<double>* tab = (const cx<double>*)p.cntab[2][conjugate ? 1 : 0];
    const cx_coef k = cn_kappa(p, 2, conjugate);
    const cx<double> kappa = {k.re, k.im};
#define DGPE_CNZ2(NZ)                                                                           \
    if (p.imag)                                                                                 \
        hipLaunchKernelGGL((k_cn_z2<T, NZ, true>), dim3(blocks), dim3(256), 0, p.stream,        \
                           (cx<T>*)f, nlines, tab, kappa);                                      \
    else                                                                                        \
        hipLaunchKernelGGL((k_cn_z2<T, NZ, false>), dim3(blocks), dim3(256), 0, p.stream,       \
                           (cx<T>*)f, nlines, tab, kappa);
    switch (Nz) {
        case 64: DGPE_CNZ2(64) break;
        case 128: DGPE_CNZ2(128) break;
        default: DGPE_CNZ2(256) break;
    }
#undef DGPE_CNZ2
    return true;
}

template <typename T>
hipError_t launch_cn_z(const Plan& p, void* f, bool conjugate) {
    if (fast_cn_z<T>(p, f, conjugate)) return hipGetLastError();
    const int Nz = p.n[2];
    const int logB = p.lc.logB_z;
    const int B = 1 << logB;
    const int es = B + 1;
    const int S = p.lc.seg[2];
    const int nseg = (Nz + S - 1) / S;
    const size_t sm = (((size_t)Nz * es * sizeof(cx<T>) + 15) & ~size_t(15)) +
                      (size_t)(2 * nseg * B + 2 * nseg) * sizeof(cx<double>);
    const int blocks = (p.n[0] * p.n[1]) >> logB;
    const CnTab tg = tab_of(p.cntab[2][conjugate ? 1 : 0], Nz);
    const cx_coef k = cn_kappa(p, 2, conjugate);
    const cx<double> kappa = {k.re, k.im};
    const bool guard = (Nz % S) != 0;
#define DGPE_CNZ(SV, RCV, GV)                                                                     \
    hipLaunchKernelGGL((k_cn_z<T, SV, RCV, GV>), dim3(blocks), dim3(p.lc.threads), sm, p.stream, \
                       (cx<T>*)f, Nz, logB, es, tg, kappa)
#define DGPE_CNZ_S(SV)                          \
    if (p.imag) {                               \
        if (guard) DGPE_CNZ(SV, true, true);    \
        else DGPE_CNZ(SV, true, false);         \
    } else {                                    \
        if (guard) DGPE_CNZ(SV, false, true);   \
        else DGPE_CNZ(SV, false, false);        \
    }
    if (S == 16) { DGPE_CNZ_S(16) }
    else if (S == 32) { DGPE_CNZ_S(32) }
    else return hipErrorInvalidValue;
#undef DGPE_CNZ_S
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
