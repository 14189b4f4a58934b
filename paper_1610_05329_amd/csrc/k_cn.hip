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
    const cx<double>* g;
    const cx<double>* h;
};

CnTab tab_of(const void* base, int N) {
    const cx<double>* t = (const cx<double>*)base;
    return CnTab{t + TAB_ALPHA * N, t + TAB_P * N, t + TAB_Q * N, t + TAB_PEND * N,
                 t + TAB_QBEG * N, t + TAB_G * N, t + TAB_H * N};
}

template <typename A>
__device__ __forceinline__ cx<A> narrow_tab(cx<double> v) { return cx<A>{A(v.x), A(v.y)}; }

// A table entry; with real coefficients (imaginary time) the imaginary parts
// are zero and only the real part is read.
template <bool RC>
__device__ __forceinline__ cx<double> tab_at(const cx<double>* t, int i) {
    if constexpr (RC) return cx<double>{reinterpret_cast<const double*>(t)[2 * i], 0.0};
    else return t[i];
}

// LDS: A1[nseg*ZB] | A2[nseg*ZB] (arithmetic type) | alpha | P | Q or G (each
// nseg*(S+1): segment s at s*(S+1), so that the segments of a wave read
// distinct banks) | pend | qbeg | H (per segment; used with G)
//
// YC (x axis only): the input is the local solution of the y solve split in
// 16-line segments, and every value is completed first as
// u += E_y c_d(x, y / 16, z) + Q_y c_x(x, y / 16, z), with the pairs
// (c_d, c_x) from the carry pass at ycar, tiled per block
// ([Ny/16][Nz/ZB][Nx][ZB][2]: the blocks of one segment and z range read one
// contiguous tile), and E, Q from the y tables.
//
// GT: the alpha, P and Q (or G) tables are read from global memory where they
// are used (L1/L2 resident, shared by every block), not staged in LDS.
template <typename T, int S, bool RC, bool GUARD, bool YC, bool GT>
__global__ void __launch_bounds__(YC || sizeof(T) == 8 ? kMaxThreads / 2 : kMaxThreads)
__attribute__((amdgpu_waves_per_eu(YC && sizeof(cn_acc_t<T, RC>) == 4 ? 4 : 1, 8)))
    k_cn_strided(cx<T>* __restrict__ f, int L, int C, int logZB, int nseg, CnTab tg,
                 cx<double> kappa64, double* __restrict__ norm_partials,
                 const cx<T>* __restrict__ ycar, const cx<double>* __restrict__ ytab, int Ny,
                 int Nz) {
    using A = cn_acc_t<T, RC>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double s_red[kMaxThreads / 64];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int ZB = 1 << logZB;
    const int nsl = nseg << logZB;
    static_assert(!(GT && YC), "the carry-completing sweep stages its tables");
    cx<A>* A1 = reinterpret_cast<cx<A>*>(smem_raw);
    cx<A>* A2 = A1 + nsl;
    const int TL = GT ? 0 : nseg * (S + 1);
    cx<A>* ta = A2 + nsl;
    cx<A>* tp = ta + TL;
    cx<A>* tq = tp + TL;
    cx<A>* pe = tq + TL;
    cx<A>* qb = pe + nseg;
    cx<A>* hs = qb + nseg;
    // First round of the table loads (one entry of each table per thread,
    // clamped: the writes below are unconditional so the loads stay ahead of
    // the state loads; see tab_stage), then the state, then staging.
    const int i0 = min(tid, L - 1), s0 = min(tid, nseg - 1);
    // solves that store at the arithmetic's precision take the Q table, the
    // ones that store narrower the G and H tables (see cn_segment_solve); the
    // tq area holds either
    constexpr bool kQ = sizeof(T) >= sizeof(A);
    const cx<double> a0 = GT ? cx<double>{0.0, 0.0} : tab_at<RC>(tg.a, i0);
    const cx<double> p0 = GT ? cx<double>{0.0, 0.0} : tab_at<RC>(tg.p, i0);
    const cx<double> q0 = (kQ && !GT) ? tab_at<RC>(tg.q, i0) : cx<double>{0.0, 0.0};
    const cx<double> pe0 = tab_at<RC>(tg.pend, s0), qb0 = tab_at<RC>(tg.qbeg, s0);
    const cx<A> kappa = narrow_tab<A>(kappa64);
    const int ncb = C >> logZB;
    const int bid = xcd_swizzle(blockIdx.x, gridDim.x);
    const int o = YC ? 0 : bid / ncb;
    // YC: z range major, so that each XCD's contiguous range of blocks covers
    // one z range for all y, and the 16 blocks of a segment that read the same
    // carry tile run close together in its L2 (measured 58 -> 55 us at 256^3)
    const int c0 = YC ? (bid % Ny) * Nz + ((bid / Ny) << logZB) : (bid - o * ncb) << logZB;
    const int cl = tid & (ZB - 1);
    const int seg = tid >> logZB;
    const int e0 = seg * S;
    const int cnt = (seg < nseg) ? min(S, L - e0) : 0;
    cx<T>* base = f + (size_t)o * L * C + c0 + cl;
    // YC: the column's y carry factors, then its carries after the state
    const int ycol = YC ? (c0 + cl) / Nz : 0, zcol = YC ? (c0 + cl) - ycol * Nz : 0;
    cx<double> ey64 = {0.0, 0.0}, qy64 = {0.0, 0.0};
    if constexpr (YC) {
        ey64 = tab_at<RC>(ytab, TAB_E * Ny + ycol);
        qy64 = tab_at<RC>(ytab, TAB_Q * Ny + ycol);
    }
    // YC (x axis, state under 4 GiB): buffer accesses, one address register
    // per lane for the state and one for the carry pairs
    constexpr uint32_t csz = sizeof(cx<T>);
    const uint32_t cstep = (uint32_t)C * csz;  // one x step of the state
    const uint32_t foff = ((uint32_t)e0 * (uint32_t)C + (uint32_t)(c0 + cl)) * csz;
    const __amdgpu_buffer_rsrc_t rf = buf_rsrc(f, YC ? (uint32_t)L * cstep : 0u);
    // the line's values are held in the state's precision between the
    // recurrences, which run in A (FP64 in real time): only the factors must
    // not be rounded to FP32, the stored intermediates may
    cx<T> v[S];
#pragma unroll
    for (int i = 0; i < S; ++i)
        if (!GUARD || i < cnt) {
            if constexpr (YC)
                v[i] = buf_load_cx<T>(rf, foff, i * cstep);
            else
                v[i] = base[(size_t)(e0 + i) * C];
        }
    if constexpr (YC) {
        const uint32_t kst = (uint32_t)ZB * 2 * csz;  // one x step of the pairs
        const uint32_t tile = (uint32_t)(ycol >> 4) * (uint32_t)(Nz >> logZB) + (uint32_t)(zcol >> logZB);
        const uint32_t coff = ((tile * (uint32_t)L + (uint32_t)e0) * (uint32_t)ZB + (uint32_t)cl) * 2 * csz;
        const __amdgpu_buffer_rsrc_t rc =
            buf_rsrc(ycar, (uint32_t)(Ny >> 4) * (uint32_t)(Nz >> logZB) * (uint32_t)L * kst);
        cx<T> cc[S][2];
#pragma unroll
        for (int i = 0; i < S; ++i)
            if (!GUARD || i < cnt) {
                if constexpr (sizeof(T) == 4) {  // the pair is one 16-byte access
                    const cx2<T> q = buf_load_cx2<T>(rc, coff, i * kst);
                    cc[i][0] = q.a;
                    cc[i][1] = q.b;
                } else {
                    cc[i][0] = buf_load_cx<T>(rc, coff, i * kst);
                    cc[i][1] = buf_load_cx<T>(rc, coff + csz, i * kst);
                }
            }
        // every load is issued: keep the table staging (which waits for the
        // table loads) below this point
        __builtin_amdgcn_sched_barrier(0);
        const cx<A> ey = narrow_tab<A>(ey64), qy = narrow_tab<A>(qy64);
#pragma unroll
        for (int i = 0; i < S; ++i)
            if (!GUARD || i < cnt)
                v[i] = to_store<T>(kfma<RC>(qy, widen<A>(cc[i][1]),
                                            kfma<RC>(ey, widen<A>(cc[i][0]), widen<A>(v[i]))));
    }
    pe[s0] = narrow_tab<A>(pe0);
    qb[s0] = narrow_tab<A>(qb0);
    if constexpr (!GT) {
        ta[i0 + i0 / S] = narrow_tab<A>(a0);
        tp[i0 + i0 / S] = narrow_tab<A>(p0);
    }
    if constexpr (kQ) {
        if constexpr (!GT) tq[i0 + i0 / S] = narrow_tab<A>(q0);
    } else {
        // G and H are first read after the neighbour exchange below, which
        // waits for the state anyway: loaded after it (registers)
        if constexpr (!GT) tq[i0 + i0 / S] = narrow_tab<A>(tab_at<RC>(tg.g, i0));
        hs[s0] = narrow_tab<A>(tab_at<RC>(tg.h, s0));
    }
    if constexpr (!GT) {
        for (int i = tid + nthr; i < L; i += nthr) {  // lines longer than the block
            const int ip = i + i / S;
            ta[ip] = narrow_tab<A>(tg.a[i]);
            tp[ip] = narrow_tab<A>(tg.p[i]);
            tq[ip] = narrow_tab<A>(kQ ? tg.q[i] : tg.g[i]);
        }
    }
    for (int i = tid + nthr; i < nseg; i += nthr) {
        pe[i] = narrow_tab<A>(tg.pend[i]);
        qb[i] = narrow_tab<A>(tg.qbeg[i]);
        if constexpr (!kQ) hs[i] = narrow_tab<A>(tg.h[i]);
    }
    cx<T> lastv = v[S - 1];
    if (GUARD) {
#pragma unroll
        for (int i = 0; i < S; ++i)
            if (i == cnt - 1) lastv = v[i];
    }
    if (cnt > 0) {
        A1[seg * ZB + cl] = widen<A>(v[0]);
        A2[seg * ZB + cl] = widen<A>(lastv);
    }
    __syncthreads();
    cx<A> left = {A(0), A(0)}, right = {A(0), A(0)};
    if (cnt > 0) {
        if (seg > 0) left = A2[(seg - 1) * ZB + cl];
        if (seg + 1 < nseg) right = A1[(seg + 1) * ZB + cl];
    }
    __syncthreads();  // neighbour reads done: A2 becomes the forward carries, A1 the backward ones
    if constexpr (GT) {
        const cx<double>* gq = kQ ? tg.q : tg.g;
        cn_segment_solve<T, S, RC, GUARD>(v, cnt, left, right, kappa, tg.a, tg.p, gq, pe, qb, e0, seg,
                                          nseg, A2, A1, cl, ZB, gq, hs);
    } else {
        cn_segment_solve<T, S, RC, GUARD>(v, cnt, left, right, kappa, ta, tp, tq, pe, qb, seg * (S + 1),
                                          seg, nseg, A2, A1, cl, ZB, tq, hs);
    }
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < S; ++i) {
        if (!GUARD || i < cnt) {
            const cx<T> o = to_store<T>(v[i]);
            if constexpr (YC)
                buf_store_cx<T>(o, rf, foff, i * cstep);
            else
                base[(size_t)(e0 + i) * C] = o;
            acc += double(abs2(o));
        }
    }
    if (norm_partials) {
        const double s = block_sum(acc, s_red);
        if (tid == 0) norm_partials[blockIdx.x] = s;
    }
}

// Carries of the y solve split in 16-line segments by the fused z pass.  One
// thread per (x, z) column with K = Ny / 16 <= KM segments; arrays q of car
// ([3][Nx][K][Nz]): 0 local d at the segment's last line plus u there (dl +
// ul), 1 local x at its first line plus u there (xf + uf), 2 u at its first
// line (uf).  With the Thomas factors alpha, the segment products PEND, QBEG
// and the carry response E (y tables):
//   forward:  c_d(0) = 0,  c_d(k+1) = (dl + ul)(k) + alpha_last(k) uf(k+1) + PEND(k) c_d(k)
//             (the true d at the segment's last line, plus the next segment's
//             left neighbour)
//   backward: c_x(K-1) = 0,  c_x(k-1) = (xf + uf)(k) + E_first(k) c_d(k) + QBEG(k) c_x(k)
//             (the true x at the segment's first line, plus the previous
//             segment's right neighbour), uf(K) = 0.
// The pairs (c_d(k), c_x(k)) go after the three arrays, tiled for the x
// sweep: [K][Nz/ZB][Nx][ZB][2] with ZB = 2^lzb columns per sweep block.  Every
// load of the column is issued before the first use.
template <typename T, bool RC, int KM>
__global__ void __launch_bounds__(64) k_cn_ycarry(cx<T>* __restrict__ car, int Nx, int Ny, int Nz,
                                                 const cx<double>* __restrict__ ytab, int lzb) {
    using A = cn_acc_t<T, RC>;
    // per segment: alpha at its last line, PEND, E at its first line, QBEG
    __shared__ cx<A> sf[4][KM];
    const int K = Ny >> 4;
    const int tid = threadIdx.x;
    const int g = blockIdx.x * 64 + tid;
    // table loads first (one per thread, clamped), then the column's values
    const int tq = min(tid / KM, 3), tk = min(tid % KM, K - 1);
    const int tix = tq == 0 ? TAB_ALPHA * Ny + 16 * tk + 15
                  : tq == 1 ? TAB_PEND * Ny + tk
                  : tq == 2 ? TAB_E * Ny + 16 * tk
                            : TAB_QBEG * Ny + tk;
    const cx<double> tv = tab_at<RC>(ytab, tix);
    const bool act = g < Nx * Nz;
    const int gg = act ? g : 0;
    const int x = gg / Nz, z = gg - x * Nz;
    const size_t cst = (size_t)Nx * K * Nz;
    cx<T>* c0 = car + (size_t)x * K * Nz + z;
    cx<T> dl[KM], xf[KM], uf[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k)
        if (k < K) {
            const size_t o = (size_t)k * Nz;
            dl[k] = c0[o];
            xf[k] = c0[cst + o];
            uf[k] = c0[2 * cst + o];
        }
    if (tid < 4 * KM) sf[tq][tid % KM] = narrow_tab<A>(tv);
    __syncthreads();
    if (!act) return;
    const cx<A> zero = {A(0), A(0)};
    cx<A> cd[KM];
    cx<A> c = zero;
#pragma unroll
    for (int k = 0; k < KM; ++k)
        if (k < K) {
            cd[k] = c;
            const cx<A> ufn = k + 1 < K ? widen<A>(uf[k + 1 < KM ? k + 1 : k]) : zero;
            c = kfma<RC>(sf[1][k], c, kfma<RC>(sf[0][k], ufn, widen<A>(dl[k])));
        }
    const int zbm = (1 << lzb) - 1;
    const size_t ktile = (size_t)(Nz >> lzb) * Nx << lzb;  // pairs per segment
    cx<T>* pr = car + 3 * cst +
                ((((size_t)(z >> lzb) * Nx + x) << lzb) + (z & zbm)) * 2;
    c = zero;
#pragma unroll
    for (int k = KM - 1; k >= 0; --k)
        if (k < K) {
            const cx<A> cxk = c;
            c = kfma<RC>(sf[3][k], cxk, kfma<RC>(sf[2][k], cd[k], widen<A>(xf[k])));
            cx<T> t2[2] = {to_store<T>(cd[k]), to_store<T>(cxk)};
            if constexpr (sizeof(T) == 4) {
                store_unit<T>(pr + (size_t)k * ktile * 2, t2);
            } else {
                pr[(size_t)k * ktile * 2] = t2[0];
                pr[(size_t)k * ktile * 2 + 1] = t2[1];
            }
        }
}

// The same carries with each column's K segments split between two lanes of
// one wave (lane l: segments [0, H), lane l + 32: [H, K), H = ceil(K/2)), so
// that twice as many waves share the latency of the loads.  Each lane runs its
// part of a chain from a zero carry; the upper half's forward values are then
// completed with prod PEND times the lower half's end value, and the lower
// half's backward values with prod QBEG times the upper half's end value (one
// shuffle each).  Same layouts and tables as k_cn_ycarry; 32 columns per block.
template <typename T, bool RC, int KH>
__global__ void __launch_bounds__(64) k_cn_ycarry2(cx<T>* __restrict__ car, int Nx, int Ny, int Nz,
                                                  const cx<double>* __restrict__ ytab, int lzb) {
    using A = cn_acc_t<T, RC>;
    constexpr int KM = 2 * KH;
    __shared__ cx<A> sf[4][KM];
    const int K = Ny >> 4, H = (K + 1) >> 1;
    const int tid = threadIdx.x, lane = tid & 63;
    const int half = tid >> 5;
    const int g = blockIdx.x * 32 + (tid & 31);
    const int tq = min(tid / KM, 3), tk = min(tid % KM, K - 1);
    const int tix = tq == 0 ? TAB_ALPHA * Ny + 16 * tk + 15
                  : tq == 1 ? TAB_PEND * Ny + tk
                  : tq == 2 ? TAB_E * Ny + 16 * tk
                            : TAB_QBEG * Ny + tk;
    const cx<double> tv = tab_at<RC>(ytab, tix);
    const bool act = g < Nx * Nz;
    const int gg = act ? g : 0;
    const int x = gg / Nz, z = gg - x * Nz;
    const int k0 = half ? H : 0, k1 = half ? K : H;
    const size_t cst = (size_t)Nx * K * Nz;
    cx<T>* c0 = car + (size_t)x * K * Nz + z;
    cx<T> dl[KH], xf[KH], uf[KH];
#pragma unroll
    for (int j = 0; j < KH; ++j)
        if (k0 + j < k1) {
            const size_t o = (size_t)(k0 + j) * Nz;
            dl[j] = c0[o];
            xf[j] = c0[cst + o];
            uf[j] = c0[2 * cst + o];
        }
    const cx<A> zero = {A(0), A(0)}, one = {A(1), A(0)};
    const cx<A> ufend = k1 < K ? widen<A>(c0[2 * cst + (size_t)k1 * Nz]) : zero;
    if (tid < 4 * KM) sf[tq][tid % KM] = narrow_tab<A>(tv);
    __syncthreads();
    // forward, from a zero carry at k0
    cx<A> cd[KH];
    cx<A> c = zero;
#pragma unroll
    for (int j = 0; j < KH; ++j)
        if (k0 + j < k1) {
            const int k = k0 + j;
            cd[j] = c;
            const cx<A> ufn = (k + 1 < k1) ? widen<A>(uf[j + 1 < KH ? j + 1 : j]) : ufend;
            c = kfma<RC>(sf[1][k], c, kfma<RC>(sf[0][k], ufn, widen<A>(dl[j])));
        }
    const cx<A> cin = shfl_up_c(c, 32, 64);  // the lower half's end value, on the upper lanes
    if (half) {
        cx<A> pp = one;
#pragma unroll
        for (int j = 0; j < KH; ++j)
            if (k0 + j < k1) {
                cd[j] = kfma<RC>(pp, cin, cd[j]);
                pp = kmul<RC>(sf[1][k0 + j], pp);
            }
    }
    // backward, from a zero carry at k1 - 1
    cx<A> cx_[KH];
    c = zero;
#pragma unroll
    for (int j = KH - 1; j >= 0; --j)
        if (k0 + j < k1) {
            const int k = k0 + j;
            cx_[j] = c;
            c = kfma<RC>(sf[3][k], c, kfma<RC>(sf[2][k], cd[j], widen<A>(xf[j])));
        }
    const cx<A> xin = shfl_down_c(c, 32, 64);  // the upper half's end value, on the lower lanes
    if (!half) {
        cx<A> qq = one;
#pragma unroll
        for (int j = KH - 1; j >= 0; --j)
            if (k0 + j < k1) {
                cx_[j] = kfma<RC>(qq, xin, cx_[j]);
                qq = kmul<RC>(sf[3][k0 + j], qq);
            }
    }
    if (!act) return;
    const int zbm = (1 << lzb) - 1;
    const size_t ktile = (size_t)(Nz >> lzb) * Nx << lzb;  // pairs per segment
    cx<T>* pr = car + 3 * cst + ((((size_t)(z >> lzb) * Nx + x) << lzb) + (z & zbm)) * 2;
#pragma unroll
    for (int j = 0; j < KH; ++j)
        if (k0 + j < k1) {
            cx<T> t2[2] = {to_store<T>(cd[j]), to_store<T>(cx_[j])};
            cx<T>* dst = pr + (size_t)(k0 + j) * ktile * 2;
            if constexpr (sizeof(T) == 4) {
                store_unit<T>(dst, t2);
            } else {
                dst[0] = t2[0];
                dst[1] = t2[1];
            }
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
    cx<T> v[SZ];
    cx<A> left = {A(0), A(0)}, right = {A(0), A(0)};
    if (cnt > 0) {
#pragma unroll
        for (int i = 0; i < SZ; ++i)
            if (!GUARD || i < cnt) v[i] = P[(e0 + i) * ES + bl];
        if (e0 > 0) left = widen<A>(P[(e0 - 1) * ES + bl]);
        if (e0 + cnt < Nz) right = widen<A>(P[(e0 + cnt) * ES + bl]);
    }
    cn_segment_solve<T, SZ, RC, GUARD>(v, cnt, left, right, kappa, tg.a, tg.p, tg.q, pe, qb, e0,
                                          seg, nseg, dl, xf, bl, B, tg.g, tg.h);
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

int cn_strided_logzb(const Plan& p, int axis, bool ycarry) {
    int logZB = p.lc.logZB[axis];
    if (!ycarry) return logZB;
    // the carry-completing variant holds two more values per point: blocks of
    // at most kMaxThreads / 2 (fewer columns per block when the line needs it)
    const int nseg = (p.n[axis] + p.lc.seg[axis] - 1) / p.lc.seg[axis];
    while (logZB > 0 && (nseg << logZB) > kMaxThreads / 2) --logZB;
    return (nseg << logZB) > kMaxThreads / 2 ? -1 : logZB;
}

int cn_strided_blocks(const Plan& p, int axis, bool ycarry) {
    const int lz = cn_strided_logzb(p, axis, ycarry);
    if (lz < 0) return 0;
    const int zb = 1 << lz;
    if (axis == 1) return p.n[0] * (p.n[2] / zb);
    return (p.n[1] * p.n[2]) / zb;
}

template <typename T>
hipError_t launch_cn_strided(const Plan& p, void* f, int axis, bool conjugate,
                             double* norm_partials, const void* ycar) {
    if (ycar && (axis != 0 || conjugate || !p.imag || p.lc.seg[1] != 16 || p.n[1] % 16))
        return hipErrorInvalidValue;
    const int L = p.n[axis];
    const int C = (axis == 1) ? p.n[2] : p.n[1] * p.n[2];
    const int S = p.lc.seg[axis];
    const int logZB = cn_strided_logzb(p, axis, ycar != nullptr);
    const int nseg = (L + S - 1) / S;
    if (logZB < 0 || (ycar && (1 << logZB) > p.n[2])) return hipErrorInvalidValue;
    const int threads = nseg << logZB;
    const CnTab tg = tab_of(p.cntab[axis][conjugate ? 1 : 0], L);
    const cx_coef k = cn_kappa(p, axis, conjugate);
    const cx<double> kappa = {k.re, k.im};
    const int blocks = cn_strided_blocks(p, axis, ycar != nullptr);
    const size_t asz = (p.imag ? sizeof(T) : sizeof(double)) * 2;
    // the carry-completing sweep stages its tables (lines it takes fit)
    const bool gt = p.lc.gtab[axis] && !ycar;
    const size_t sm = (size_t)(2 * threads + (gt ? 0 : 3 * nseg * (S + 1)) + 3 * nseg) * asz;
    const bool guard = (L % S) != 0;
    const cx<double>* ytab = (const cx<double>*)p.cntab[1][0];
#define DGPE_CN(SV, RCV, GV, YV)                                                                      \
    if (gt && !YV)                                                                                    \
        hipLaunchKernelGGL((k_cn_strided<T, SV, RCV, GV, false, true>), dim3(blocks), dim3(threads),  \
                           sm, p.stream, (cx<T>*)f, L, C, logZB, nseg, tg, kappa, norm_partials,      \
                           (const cx<T>*)ycar, ytab, p.n[1], p.n[2]);                                 \
    else                                                                                              \
    hipLaunchKernelGGL((k_cn_strided<T, SV, RCV, GV, YV, false>), dim3(blocks), dim3(threads), sm, p.stream, \
                       (cx<T>*)f, L, C, logZB, nseg, tg, kappa, norm_partials, (const cx<T>*)ycar,    \
                       ytab, p.n[1], p.n[2])
#define DGPE_CN_S(SV)                                  \
    if (p.imag) {                                      \
        if (ycar) {                                    \
            if (guard) DGPE_CN(SV, true, true, true);  \
            else DGPE_CN(SV, true, false, true);       \
        } else if (guard) DGPE_CN(SV, true, true, false); \
        else DGPE_CN(SV, true, false, false);          \
    } else {                                           \
        if (guard) DGPE_CN(SV, false, true, false);    \
        else DGPE_CN(SV, false, false, false);         \
    }
    if (S == 16) { DGPE_CN_S(16) }
    else return hipErrorInvalidValue;
#undef DGPE_CN_S
#undef DGPE_CN
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cn_ycarry(const Plan& p, void* car) {
    const int K = p.n[1] / 16;
    if (!p.imag || p.lc.seg[1] != 16 || p.n[1] % 16 || K > 16) return hipErrorInvalidValue;
    const int blocks = (p.n[0] * p.n[2] + 63) / 64;
    const cx<double>* ytab = (const cx<double>*)p.cntab[1][0];
    // the tiling of the pairs follows the x sweep that reads them
    const int lzb = cn_strided_logzb(p, 0, true);
    if (lzb < 0 || (1 << lzb) > p.n[2]) return hipErrorInvalidValue;
#define DGPE_YC(KMV)                                                                           \
    hipLaunchKernelGGL((k_cn_ycarry<T, true, KMV>), dim3(blocks), dim3(64), 0, p.stream,       \
                       (cx<T>*)car, p.n[0], p.n[1], p.n[2], ytab, lzb)
    if (K <= 4) DGPE_YC(4);
    else if (K <= 8) DGPE_YC(8);
    else if (p.n[2] % 32)  // the two-lane kernel takes 32 whole z columns per block
        return hipErrorInvalidValue;
    else  // two lanes per column
        hipLaunchKernelGGL((k_cn_ycarry2<T, true, 8>), dim3((p.n[0] * p.n[2] + 31) / 32), dim3(64), 0,
                           p.stream, (cx<T>*)car, p.n[0], p.n[1], p.n[2], ytab, lzb);
#undef DGPE_YC
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
    template hipError_t launch_cn_strided<T>(const Plan&, void*, int, bool, double*, const void*); \
    template hipError_t launch_cn_ycarry<T>(const Plan&, void*); \
    template hipError_t launch_cn_z<T>(const Plan&, void*, bool);
DGPE_INST(float)
DGPE_INST(double)
#undef DGPE_INST

}  // namespace dgpe
