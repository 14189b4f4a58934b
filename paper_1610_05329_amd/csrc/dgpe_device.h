// Device building blocks of libdgpe for gfx950 (CDNA4, wave64):
// complex arithmetic, radix-2/3/4/8 DFT butterflies, one Stockham stage on a
// batch of sequences resident in LDS, and cheap division by plan constants.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "dgpe_internal.h"

namespace dgpe {

// ---------------------------------------------------------------------------
// complex numbers: interleaved (re, im), 8 B (float) or 16 B (double)
// ---------------------------------------------------------------------------
template <typename T>
struct alignas(2 * sizeof(T)) cx {
    using value_type = T;
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) { return cx<T>{a, b}; }
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.x, s * a.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ T abs2(cx<T> a) { return a.x * a.x + a.y * a.y; }
// sin and cos of a phase angle.  Cody-Waite reduction: k = rint(2x/pi),
// r = (x - k P1) - k P2 with P2 = pi/2 - P1, then the Taylor series of sin and
// cos on |r| <= pi/4 and the quadrant's exchange and signs.  FP64: P1 = pi/2
// rounded to 33 significant bits (k P1 exact for |k| < 2^20).  FP32: P1 = pi/2
// rounded to FP32 and both steps fused multiply-adds; the first is exact (x and
// k P1 are multiples of ulp(P1) or of ulp(x) and their difference is below
// pi/4 + ulp, so it fits 24 bits) and the second rounds once; the omitted
// tail k (pi/2 - P1 - P2) is below 3e-15 |k|.  Truncation: the first omitted
// term is below 2e-9 (FP32: through r^9 and r^10) and below 1e-19 (FP64:
// through r^17 and r^18) relative to the result's scale.
namespace detail {
constexpr double kTwoOverPi = 0.6366197723675814;
constexpr double kPio2Hi = 1.5707963267341256;   // 0x3FF921FB54400000
constexpr double kPio2Lo = 6.077100506506192e-11;

__device__ __forceinline__ double reduce_pio2(double x, int* q) {
    const double k = rint(x * kTwoOverPi);
    *q = int(k) & 3;
    return fma(-k, kPio2Lo, fma(-k, kPio2Hi, x));
}

template <typename T>
__device__ __forceinline__ void quadrant(int q, T sr, T cr, T* s, T* c) {
    const T a = (q & 1) ? cr : sr;   // sin(r + q pi/2) up to sign
    const T b = (q & 1) ? sr : cr;   // cos(r + q pi/2) up to sign
    *s = (q & 2) ? -a : a;
    *c = ((q + 1) & 2) ? -b : b;
}
}  // namespace detail

// The reduced argument's sin r and cos r - 1 (the cosine series without its
// leading 1), and the quadrant q
__device__ __forceinline__ void sin_cosm1_reduced(float x, int* q, float* sr, float* cm1r) {
    const float k = rintf(x * 0.636619772f);
    *q = int(k) & 3;
    const float r = fmaf(-k, -4.37113883e-08f, fmaf(-k, 1.57079637f, x));
    const float r2 = r * r;
    // sin r = r (1 - r^2/3! + r^4/5! - r^6/7! + r^8/9!)
    float ps = 1.0f / 362880.0f;
    ps = fmaf(ps, r2, -1.0f / 5040.0f);
    ps = fmaf(ps, r2, 1.0f / 120.0f);
    ps = fmaf(ps, r2, -1.0f / 6.0f);
    *sr = fmaf(r * r2, ps, r);
    // cos r - 1 = -r^2/2! + r^4/4! - ... - r^10/10!
    float pc = -1.0f / 3628800.0f;
    pc = fmaf(pc, r2, 1.0f / 40320.0f);
    pc = fmaf(pc, r2, -1.0f / 720.0f);
    pc = fmaf(pc, r2, 1.0f / 24.0f);
    pc = fmaf(pc, r2, -0.5f);
    *cm1r = r2 * pc;
}

__device__ __forceinline__ void sin_cosm1_reduced(double x, int* q, double* sr, double* cm1r) {
    const double r = detail::reduce_pio2(x, q);
    const double r2 = r * r;
    // odd Taylor terms through r^17, even ones through r^18: coefficients
    // (-1)^n / (2n+1)! and (-1)^n / (2n)!
    constexpr double S[9] = {1.0, -1.0 / 6.0, 1.0 / 120.0, -1.0 / 5040.0, 1.0 / 362880.0,
                             -1.0 / 39916800.0, 1.0 / 6227020800.0, -1.0 / 1307674368000.0,
                             1.0 / 355687428096000.0};
    constexpr double C[10] = {1.0, -0.5, 1.0 / 24.0, -1.0 / 720.0, 1.0 / 40320.0,
                              -1.0 / 3628800.0, 1.0 / 479001600.0, -1.0 / 87178291200.0,
                              1.0 / 20922789888000.0, -1.0 / 6402373705728000.0};
    double ps = S[8];
#pragma unroll
    for (int i = 7; i >= 1; --i) ps = fma(ps, r2, S[i]);
    *sr = fma(r * r2, ps, r);
    double pc = C[9];
#pragma unroll
    for (int i = 8; i >= 1; --i) pc = fma(pc, r2, C[i]);
    *cm1r = r2 * pc;
}

template <typename T>
__device__ __forceinline__ void sin_cos(T x, T* s, T* c) {
    int q;
    T sr, cm1r;
    sin_cosm1_reduced(x, &q, &sr, &cm1r);
    detail::quadrant(q, sr, T(1) + cm1r, s, c);
}

// psi e^{-i theta} with theta = r + q pi/2, |r| <= pi/4: first the q quarter
// turns, (-i)^q psi, exactly (a swap of the components and sign changes), then
// the small angle as p + p (e^{-i r} - 1) with sin r and cos r - 1 from their
// series (cos r - 1 without the leading 1).  cos r itself, rounded to the
// state's precision near r = 0, is off by up to half an ulp of 1 with one sign
// over neighbouring points and steps: |e^{-i theta}| would then differ from 1
// by about that much and the real-time norm drift.  The increment keeps its
// full relative precision, so the modulus error is of order r^2 eps, and the
// result is rounded once.
template <typename T>
__device__ __forceinline__ cx<T> rotate_phase(cx<T> q, T th) {
    int qd;
    T sr, cm1r;
    sin_cosm1_reduced(th, &qd, &sr, &cm1r);
    // (-i)^q (x + i y): q = 1 (y, -x), 2 (-x, -y), 3 (-y, x)
    T a = (qd & 1) ? q.y : q.x;
    T b = (qd & 1) ? q.x : q.y;
    if (qd & 2) a = -a;
    if ((qd + 1) & 2) b = -b;
    return cx<T>{a + fma(b, sr, a * cm1r), b + fma(-a, sr, b * cm1r)};
}

// exp(x) = 2^(x log2 e) on the hardware base-2 exponential (v_exp_f32, about
// 1 ulp): the product's rounding adds |x| eps relative, negligible for the
// imaginary-time factors exp(-theta), theta = dt (...) << 1, and it takes 2
// instructions where the library expf takes about 8 (instruction issue is
// about two thirds of the fused z pass's time, next to its HBM traffic)
__device__ __forceinline__ float exp_of(float x) {
    return __builtin_amdgcn_exp2f(x * 1.44269504088896340736f);
}
__device__ __forceinline__ double exp_of(double x) { return exp(x); }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cx<T> rot90(cx<T> a) {
    return INV ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
}

// ---------------------------------------------------------------------------
// quotient by a plan constant d (2 <= d, n * d < 2^32): q = umulhi(n, ceil(2^32/d))
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) { return __umulhi(n, f.m); }

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with its own L2.  Remap so that each XCD works through one contiguous range
// of logical tiles: neighbouring tiles that share cache lines then meet in the
// same L2.  Identity when the grid is not a multiple of 8.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_swizzle(int bid, int nblocks) {
    if (nblocks % kXcds) return bid;
    return (bid % kXcds) * (nblocks / kXcds) + bid / kXcds;
}

// ---------------------------------------------------------------------------
// small DFTs, forward sign exp(-2 pi i jk/R); INV gives the conjugate kernel
// ---------------------------------------------------------------------------
template <typename T, bool INV>
__device__ __forceinline__ void dft2(cx<T>& a0, cx<T>& a1) {
    cx<T> t = a0 - a1;
    a0 = a0 + a1;
    a1 = t;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft3(cx<T>* v) {
    const T h = T(0.5);
    const T s = T(0.86602540378443864676372317075293618);
    cx<T> t1 = v[1] + v[2];
    cx<T> t2 = v[0] - h * t1;
    cx<T> d = s * (v[1] - v[2]);
    cx<T> t3 = rot90<T, INV>(d);
    v[0] = v[0] + t1;
    v[1] = t2 + t3;
    v[2] = t2 - t3;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
    cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = rot90<T, INV>(a1 - a3);
    a0 = t0 + t2;
    a2 = t0 - t2;
    a1 = t1 + t3;
    a3 = t1 - t3;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cx<T>* v) {
    const T c = T(0.70710678118654752440084436210484904);
    cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<T, INV>(e0, e1, e2, e3);
    dft4<T, INV>(o0, o1, o2, o3);
    // o_k *= W8^k, W8 = exp(-i pi/4) (conjugated for INV)
    cx<T> w1 = INV ? cx<T>{c, c} : cx<T>{c, -c};
    cx<T> w3 = INV ? cx<T>{-c, c} : cx<T>{-c, -c};
    o1 = cmul(o1, w1);
    o2 = rot90<T, INV>(o2);
    o3 = cmul(o3, w3);
    v[0] = e0 + o0;
    v[4] = e0 - o0;
    v[1] = e1 + o1;
    v[5] = e1 - o1;
    v[2] = e2 + o2;
    v[6] = e2 - o2;
    v[3] = e3 + o3;
    v[7] = e3 - o3;
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dftR(cx<T>* v) {
    if constexpr (R == 2) dft2<T, INV>(v[0], v[1]);
    else if constexpr (R == 3) dft3<T, INV>(v);
    else if constexpr (R == 4) dft4<T, INV>(v[0], v[1], v[2], v[3]);
    else dft8<T, INV>(v);
}

// ---------------------------------------------------------------------------
// One self-sorting (Stockham) radix-R stage over B = 2^logB sequences of
// length L held in LDS; element e of sequence b lives at buf[e * ES + b].
// Butterfly j (0 <= j < L/R) with k = j mod Ns reads elements j + r L/R,
// multiplies element r by W_L^{r k L/(Ns R)}, applies the R-point DFT and
// writes to ((j - k) R + k + r Ns).  All reads of a stage complete (barrier)
// before its writes, so the stage runs in place with registers as staging.
// Each thread owns at most MAXB butterflies (the launch guarantees it).
// ---------------------------------------------------------------------------
template <typename T, int R, bool INV, int MAXB>
__device__ __forceinline__ void fft_stage(cx<T>* buf, int ES, int L, int logB, int Ns, int logNs,
                                          const cx<T>* tw, int tid, int nthr) {
    const int LR = L / R;
    const int nb = LR << logB;
    const int tws = L / (Ns * R);
    const int bmask = (1 << logB) - 1;
    cx<T> v[MAXB][R];
    int obase[MAXB];
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int t = tid + q * nthr;
        if (t < nb) {
            const int b = t & bmask;
            const int j = t >> logB;
            const int k = logNs >= 0 ? (j & (Ns - 1)) : j % Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[(j + r * LR) * ES + b];
            if (k != 0) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cx<T> w = tw[r * k * tws];
                    v[q][r] = INV ? cmulc(v[q][r], w) : cmul(v[q][r], w);
                }
            }
            obase[q] = ((j - k) * R + k) * ES + b;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int t = tid + q * nthr;
        if (t < nb) {
            dftR<T, R, INV>(v[q]);
#pragma unroll
            for (int r = 0; r < R; ++r) buf[obase[q] + r * Ns * ES] = v[q][r];
        }
    }
    __syncthreads();
}

// Whole FFT of length f.L on the LDS batch (forward: exp(-2 pi i ...), INV:
// exp(+2 pi i ...), both unnormalised).  The caller synchronises before the
// first stage; the last stage ends with a barrier.  EMAX bounds the elements
// per thread: (L << logB) <= EMAX * nthr.
template <typename T, bool INV, int EMAX>
__device__ __forceinline__ void lds_fft(cx<T>* buf, int ES, const FftDesc& f, int logB,
                                        const cx<T>* tw, int tid, int nthr) {
    int Ns = 1, logNs = 0;
    for (int s = 0; s < f.nstages; ++s) {
        const int R = f.radix[s];
        if (R == 8) fft_stage<T, 8, INV, (EMAX + 7) / 8>(buf, ES, f.L, logB, Ns, logNs, tw, tid, nthr);
        else if (R == 4) fft_stage<T, 4, INV, (EMAX + 3) / 4>(buf, ES, f.L, logB, Ns, logNs, tw, tid, nthr);
        else if (R == 3) fft_stage<T, 3, INV, (EMAX + 2) / 3>(buf, ES, f.L, logB, Ns, logNs, tw, tid, nthr);
        else fft_stage<T, 2, INV, (EMAX + 1) / 2>(buf, ES, f.L, logB, Ns, logNs, tw, tid, nthr);
        Ns *= R;
        // Ns stays a power of two until the first radix-3 stage (radix 3 comes last)
        logNs = (R == 3 || logNs < 0) ? -1 : logNs + (R == 8 ? 3 : R == 4 ? 2 : 1);
    }
}

// ---------------------------------------------------------------------------
// block-wide FP64 sum (deterministic fixed tree: wave shuffles, then LDS)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sums v over the block; the result is valid in thread 0.  `scratch` holds
// one double per wave.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < nw; ++w) r += scratch[w];
    return r;
}

// Deterministic FP64 sum of n partials by one block (blockDim a multiple of
// 64): each thread a strided Neumaier sum, its loads issued in batches of 8,
// then block_sum.  The result is valid in thread 0; every thread must call.
__device__ __forceinline__ double block_sum_partials(const double* __restrict__ partials, int n,
                                                     double* scratch) {
    constexpr int kBatch = 8;
    const int nt = blockDim.x;
    double s = 0.0, c = 0.0;
    for (int b0 = threadIdx.x; b0 < n; b0 += kBatch * nt) {
        double vb[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            const int b = b0 + j * nt;
            vb[j] = b < n ? partials[b] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            if (b0 + j * nt >= n) break;
            const double v = vb[j];
            const double t = s + v;
            c += (fabs(s) >= fabs(v)) ? (s - t) + v : (v - t) + s;
            s = t;
        }
    }
    return block_sum(s + c, scratch);
}

}  // namespace dgpe

namespace dgpe {

// ---------------------------------------------------------------------------
// Crank-Nicolson solve of one line split into segments of S points.
//
// (1 - A D) x = (1 + A D) u on a line of N points with zero ghosts is a
// constant tridiagonal system tridiag(-A, 1 + 2A, -A).  Thomas elimination
// with pivots 1/m_i gives m_0 = 1/(1 + 2A), m_i = 1/(1 + 2A - A^2 m_{i-1});
// with alpha_i = A m_i both the forward and the backward recurrences use the
// same factor:
//   d_i = alpha_i (d_{i-1} + r'_i),  r'_i = u_{i-1} + u_{i+1} + kappa u_i,
//   kappa = 1/A - 2  (r' is the right-hand side divided by A),
//   x_i = d_i + alpha_i x_{i+1}.
// Each thread owns the segment [e0, e0 + cnt) of one line in registers (v,
// holding u on entry) and
//   1. forms r' from its points and the neighbours `left` (u_{e0-1}) and
//      `right` (u_{e0+cnt}), zero beyond the line;
//   2. runs the forward recurrence from a zero carry, publishes its last d;
//   3. adds P_i * (true d_{e0-1}), P_i = prod_{j=e0}^{i} alpha_j, where the
//      true value follows from the published ends of the segments on its left
//      through d_end(k) = dtilde_end(k) + Pend(k) d_end(k-1);
//   4. runs back substitution from a zero carry, publishes its first x, and
//      adds Q_i * (true x_{e0+cnt}), Q_i = prod_{j=i}^{e0+cnt-1} alpha_j.
// The result equals plain Thomas elimination up to rounding (no truncation).
// alpha, P, Q are plan tables (length N); pend/qbeg hold P at each segment's
// end and Q at each segment's start.  RC: real coefficients (imaginary time).
// GUARD: segments may be partial (cnt < S); otherwise every active thread has
// cnt == S.  All threads of the block call this (two barriers); threads
// without a segment pass cnt = 0.  dl and xf are LDS arrays of nseg * nlines
// entries, indexed [seg * nlines + line].
// ---------------------------------------------------------------------------
template <bool RC, typename T>
__device__ __forceinline__ cx<T> kmul(cx<T> k, cx<T> a) {
    if constexpr (RC) return cx<T>{k.x * a.x, k.x * a.y};
    else return cmul(k, a);
}
// c + k a, the products accumulated by fused multiply-adds (two per component
// for complex k, one for real k): the recurrences' multiply-then-add steps in
// half the instructions
template <bool RC, typename T>
__device__ __forceinline__ cx<T> kfma(cx<T> k, cx<T> a, cx<T> c) {
    if constexpr (RC) return cx<T>{fma(k.x, a.x, c.x), fma(k.x, a.y, c.y)};
    else return cx<T>{fma(k.x, a.x, fma(-k.y, a.y, c.x)), fma(k.x, a.y, fma(k.y, a.x, c.y))};
}

// Arithmetic type of the tridiagonal recurrences: the storage type in
// imaginary time (real coefficients; renormalised every step), FP64 in real
// time.  Rounding the Thomas factors to FP32 would make every step
// non-unitary by O(1e-7) with the same sign each step, a systematic norm drift
// over long runs; FP64 factors and recurrences leave only the unbiased rounding
// of the FP32 state.
template <typename T, bool RC>
using cn_acc_t = typename std::conditional<RC, T, double>::type;

template <typename A, typename T>
__device__ __forceinline__ cx<A> widen(cx<T> v) { return cx<A>{A(v.x), A(v.y)}; }
// 16-byte units of the state: two FP32 or one FP64 complex values
template <typename T>
struct unit16;
template <>
struct unit16<float> {
    using type = float4;
};
template <>
struct unit16<double> {
    using type = double2;
};

template <typename T>
__device__ __forceinline__ void load_unit(const cx<T>* p, cx<T>* out) {
    const auto q = *reinterpret_cast<const typename unit16<T>::type*>(p);
    if constexpr (sizeof(T) == 4) {
        out[0] = cx<T>{q.x, q.y};
        out[1] = cx<T>{q.z, q.w};
    } else {
        out[0] = cx<T>{q.x, q.y};
    }
}

template <typename T>
__device__ __forceinline__ void store_unit(cx<T>* p, const cx<T>* in) {
    typename unit16<T>::type q;
    if constexpr (sizeof(T) == 4) {
        q = float4{in[0].x, in[0].y, in[1].x, in[1].y};
    } else {
        q = double2{in[0].x, in[0].y};
    }
    *reinterpret_cast<typename unit16<T>::type*>(p) = q;
}

// Orders the LDS accesses of one wave (no cross-wave synchronisation)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


// A wave's LPW = 64 / nseg whole lines of Nz values (LPW * Nz consecutive
// values in HBM) in two layouts: the load layout (lane l holds the 16-byte
// units j * 64 + l, coalesced) and the segment layout (lane = segment of SZ
// consecutive points, the nseg segments of a line on consecutive lanes).  The
// transposes go through the wave's own LDS staging area, KR lines per round;
// a staged line is Nz values with one 16-byte unit of padding after each
// segment (the segment-wise accesses then spread over the banks).
template <typename T, int Nz, int SZ, int KR>
struct WaveLines {
    static constexpr int nseg = Nz / SZ;
    static constexpr int LPW = 64 / nseg;
    static constexpr int U = 16 / (int)sizeof(cx<T>);
    static constexpr int NU = SZ / U;           // units per lane
    static constexpr int SL = Nz + nseg * U;    // staged line
    static constexpr int JR = KR * Nz / (64 * U);  // unit loads per lane and round
    static_assert(LPW % KR == 0 && JR * 64 * U == KR * Nz, "rounds of whole unit loads");

    __device__ static int unit_pos(int j, int lane, int r) {
        const int c = (j * 64 + lane) * U - r * KR * Nz;
        const int e = c % Nz;
        return (c / Nz) * SL + e + (e / SZ) * U;
    }

    // v wider than the state: the values are widened after the rounds, so each
    // conversion is issued once rather than once per round
    template <typename A>
    __device__ static void to_segments(cx<T>* stg, const cx<T> (&a)[SZ], cx<A> (&v)[SZ], int lane) {
        if constexpr (std::is_same_v<A, T>) {
            stage_in(stg, a, v, lane);
        } else {
            cx<T> t[SZ];
            stage_in(stg, a, t, lane);
#pragma unroll
            for (int i = 0; i < SZ; ++i) v[i] = widen<A>(t[i]);
        }
    }

    template <typename A>
    __device__ static void store_from_segments(cx<T>* stg, const cx<A> (&v)[SZ], cx<T>* wp,
                                               int lane) {
        if constexpr (std::is_same_v<A, T>) {
            stage_out(stg, v, wp, lane);
        } else {
            cx<T> t[SZ];
#pragma unroll
            for (int i = 0; i < SZ; ++i) t[i] = cx<T>{T(v[i].x), T(v[i].y)};
            stage_out(stg, t, wp, lane);
        }
    }

    __device__ static void stage_in(cx<T>* stg, const cx<T> (&a)[SZ], cx<T> (&v)[SZ], int lane) {
        const int seg = lane % nseg, sl = lane / nseg;
#pragma unroll
        for (int r = 0; r < LPW / KR; ++r) {
            wave_sync();  // earlier reads of the staging area done
#pragma unroll
            for (int jj = 0; jj < JR; ++jj) {
                const int j = r * JR + jj;
                store_unit<T>(stg + unit_pos(j, lane, r), a + j * U);
            }
            wave_sync();
            if (sl / KR == r) {
                const cx<T>* sp = stg + (sl - r * KR) * SL + seg * (SZ + U);
#pragma unroll
                for (int j = 0; j < NU; ++j) load_unit<T>(sp + j * U, v + j * U);
            }
        }
    }

    __device__ static void stage_out(cx<T>* stg, const cx<T> (&v)[SZ], cx<T>* wp, int lane) {
        const int seg = lane % nseg, sl = lane / nseg;
#pragma unroll
        for (int r = 0; r < LPW / KR; ++r) {
            wave_sync();
            if (sl / KR == r) {
                cx<T>* sp = stg + (sl - r * KR) * SL + seg * (SZ + U);
#pragma unroll
                for (int j = 0; j < NU; ++j) store_unit<T>(sp + j * U, v + j * U);
            }
            wave_sync();
#pragma unroll
            for (int jj = 0; jj < JR; ++jj) {
                const int j = r * JR + jj;
                cx<T> t2[U];
                load_unit<T>(stg + unit_pos(j, lane, r), t2);
                store_unit<T>(wp + (j * 64 + lane) * U, t2);
            }
        }
    }
};

// Raw buffer access (vector memory instructions): a resource over `bytes`
// bytes from `base`, a per-lane 32-bit byte offset and a wave-uniform byte
// offset, so a lane keeps one address register however many strided values it
// moves.  Reads past the range return zero and writes past it are dropped.
// Third descriptor word: the gfx9 raw-buffer format.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}

template <typename T>
__device__ __forceinline__ cx<T> buf_load_cx(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    typedef unsigned v2u __attribute__((ext_vector_type(2)));
    typedef unsigned v4u __attribute__((ext_vector_type(4)));
    if constexpr (sizeof(T) == 4) {
        const v2u q = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0);
        return __builtin_bit_cast(cx<T>, q);
    } else {
        const v4u q = __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0);
        return __builtin_bit_cast(cx<T>, q);
    }
}

// Two FP32 complex values in one 16-byte access.  The loaded vector is
// reinterpreted whole: extracting its elements one by one after the builtin
// compiled to a single dword load replicated into all four.
template <typename T>
struct cx2 {
    cx<T> a, b;
};

template <typename T>
__device__ __forceinline__ cx2<T> buf_load_cx2(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    static_assert(sizeof(T) == 4, "16-byte pair of FP32 complex values");
    typedef unsigned v4u __attribute__((ext_vector_type(4)));
    const v4u q = __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0);
    return __builtin_bit_cast(cx2<T>, q);
}

template <typename T>
__device__ __forceinline__ void buf_store_cx(cx<T> v, __amdgpu_buffer_rsrc_t r, uint32_t vo,
                                             uint32_t so) {
    if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r, vo, so, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v), r, vo, so, 0);
}

// Small per-block tables (twiddles, Thomas factors) in registers: every load
// issued first, staged in LDS after the block's other loads are in flight.
template <typename V, int N, int NT>
struct TabRegs {
    static constexpr int R = (N + NT - 1) / NT;
    V v[R];
};

template <typename V, int N, int NT, typename S>
__device__ __forceinline__ void tab_issue(TabRegs<V, N, NT>& r, const S* __restrict__ src, int tid) {
#pragma unroll
    for (int u = 0; u < TabRegs<V, N, NT>::R; ++u) r.v[u] = src[min(tid + u * NT, N - 1)];
}

// Stages a TabRegs in LDS at dst[index(i)].  Every thread writes (threads past
// the end repeat the last entry, with its own value): a conditional write would
// let the compiler move the load down into the branch, and the wait for it
// would then also wait for the state loads issued after it.
template <typename V, int N, int NT, typename D, typename F>
__device__ __forceinline__ void tab_stage(const TabRegs<V, N, NT>& r, D* dst, int tid, F index) {
#pragma unroll
    for (int u = 0; u < TabRegs<V, N, NT>::R; ++u) dst[index(min(tid + u * NT, N - 1))] = widen<typename D::value_type>(r.v[u]);
}

// conversion between the arithmetic type and the segment values' type.  Values
// held narrower than the arithmetic (FP32 segments of the FP64 real-time
// recurrences) are rounded once each: the forward d, and each x from the true
// right carry (rounding r', or an x before its carry correction, was measured
// to drift the real-time norm by about 1e-8 per step at 128^3)
template <typename V, typename A>
__device__ __forceinline__ cx<V> to_store(cx<A> v) { return cx<V>{V(v.x), V(v.y)}; }

template <typename A>
__device__ __forceinline__ cx<A> shfl_up_c(cx<A> v, int d, int width) {
    return cx<A>{__shfl_up(v.x, d, width), __shfl_up(v.y, d, width)};
}
template <typename A>
__device__ __forceinline__ cx<A> shfl_down_c(cx<A> v, int d, int width) {
    return cx<A>{__shfl_down(v.x, d, width), __shfl_down(v.y, d, width)};
}

// Carry of the exact segmented Thomas solve from the published segment ends
// b_k = buf[k * nlines + line] and the segment products m_k, over k in
// [k0, k1): c = b_k + m_k c taken in increasing k (forward: the true d before
// segment k1) or decreasing k (backward: the true x after segment k0 - 1).
// CH segments per round (4 in FP32, 2 in FP64: registers), their LDS reads
// issued together.
template <typename A, bool RC, bool REV>
__device__ __forceinline__ cx<A> carry_chain(const cx<A>* buf, const cx<A>* m, int k0, int k1,
                                             int nlines, int line) {
    constexpr int CH = sizeof(A) == 4 ? 4 : 2;
    cx<A> c = {A(0), A(0)};
    const int n = k1 - k0;
    int r = 0;
    for (; r + CH <= n; r += CH) {
        cx<A> bv[CH], mv[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int k = REV ? k1 - 1 - (r + q) : k0 + r + q;
            bv[q] = buf[k * nlines + line];
            mv[q] = m[k];
        }
#pragma unroll
        for (int q = 0; q < CH; ++q) c = kfma<RC>(mv[q], c, bv[q]);
    }
    for (; r < n; ++r) {
        const int k = REV ? k1 - 1 - r : k0 + r;
        c = kfma<RC>(m[k], c, buf[k * nlines + line]);
    }
    return c;
}

// tg, hs (only for values stored narrower than A): the G table (indexed like
// ta) and H per segment, see dgpe_internal.h
template <typename T, int S, bool RC, bool GUARD, typename TT, typename VS, typename TH = double>
__device__ __forceinline__ void cn_segment_solve(cx<VS> (&v)[S], int cnt,
                                                 cx<cn_acc_t<T, RC>> left,
                                                 cx<cn_acc_t<T, RC>> right,
                                                 cx<cn_acc_t<T, RC>> kappa, const cx<TT>* ta,
                                                 const cx<TT>* tp, const cx<TT>* tq,
                                                 const cx<cn_acc_t<T, RC>>* pend,
                                                 const cx<cn_acc_t<T, RC>>* qbeg, int tb, int seg,
                                                 int nseg, cx<cn_acc_t<T, RC>>* dl,
                                                 cx<cn_acc_t<T, RC>>* xf, int line, int nlines,
                                                 const cx<TT>* tg = nullptr,
                                                 const cx<TH>* hs = nullptr) {
    using A = cn_acc_t<T, RC>;
    // FP32 recurrences keep the segment's alpha in registers; FP64 ones read it
    // where it is used (register budget)
    constexpr bool kPre = sizeof(A) == 4;
    const bool act = cnt > 0;
    cx<A> al[kPre ? S : 1];
    if constexpr (kPre) {
#pragma unroll
        for (int i = 0; i < S; ++i)
            if (act && (!GUARD || i < cnt)) al[i] = widen<A>(ta[tb + i]);
    }
    auto alpha = [&](int i) -> cx<A> {
        if constexpr (kPre) return al[kPre ? i : 0];
        else return widen<A>(ta[tb + i]);
    };
    // Values stored narrower than the arithmetic (FP32 state, FP64 real-time
    // recurrences) must be rounded once: storing the zero-carry x and adding
    // Q_i x_right afterwards rounds those values twice, and that double
    // rounding drifts the norm (about 6e-6 over 1000 real-time steps at 128^3;
    // rounding the forward d is harmless).  So the back substitution runs once,
    // from the true right carry, and the segment's first x from a zero right
    // carry, which the right carries need, is accumulated in the forward pass
    // instead: x_first = sum_i G_i d_i = sum_i G_i dloc_i + H c_left.
    constexpr bool kTwice = sizeof(VS) < sizeof(A);
    cx<A> xacc = {A(0), A(0)};
    // 1. forward recurrence from a zero carry, with r'_i = u_{i-1} + u_{i+1} +
    // kappa u_i formed on the fly from the input values (threads without a
    // segment read no table)
    if (act) {
        cx<A> dcur = {A(0), A(0)};
        cx<A> prev = left, cur = widen<A>(v[0]);
#pragma unroll
        for (int i = 0; i < S; ++i) {
            cx<A> nxt = right;
            if (i + 1 < S) {
                if (!GUARD || i + 1 < cnt) nxt = widen<A>(v[(i + 1 < S) ? i + 1 : i]);
            }
            if (!GUARD || i < cnt) {
                dcur = kmul<RC>(alpha(i), kfma<RC>(kappa, cur, (dcur + prev) + nxt));
                v[i] = to_store<VS>(dcur);
                // the segment's first x from zero carries on both sides
                if constexpr (kTwice) xacc = kfma<RC>(widen<A>(tg[tb + i]), dcur, xacc);
            }
            prev = cur;
            cur = nxt;
        }
        dl[seg * nlines + line] = dcur;
    }
    __syncthreads();
    cx<A> c = {A(0), A(0)};
    if (act) {
        // 2. true d before the segment's first point, from the segments on the
        // left (P correction), then back substitution from a zero carry
        c = carry_chain<A, RC, false>(dl, pend, 0, seg, nlines, line);
        if constexpr (kTwice) {
            xf[seg * nlines + line] = kfma<RC>(widen<A>(hs[seg]), c, xacc);
        } else {
            cx<A> xcur = {A(0), A(0)};
#pragma unroll
            for (int i = S - 1; i >= 0; --i) {
                if (!GUARD || i < cnt) {
                    const cx<A> d = kfma<RC>(widen<A>(tp[tb + i]), c, widen<A>(v[i]));
                    xcur = kfma<RC>(alpha(i), xcur, d);
                    v[i] = to_store<VS>(xcur);
                }
            }
            xf[seg * nlines + line] = xcur;
        }
    }
    __syncthreads();
    if (act) {
        const cx<A> cr = carry_chain<A, RC, true>(xf, qbeg, seg + 1, nseg, nlines, line);
        if constexpr (kTwice) {
            // 3. back substitution from the true x after the segment (the
            // factors read here, not held since the forward pass)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            cx<A> xcur = cr;
#pragma unroll
            for (int i = S - 1; i >= 0; --i) {
                if (!GUARD || i < cnt) {
                    const cx<A> d = kfma<RC>(widen<A>(tp[tb + i]), c, widen<A>(v[i]));
                    xcur = kfma<RC>(alpha(i), xcur, d);
                    v[i] = to_store<VS>(xcur);
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < S; ++i)
                if (!GUARD || i < cnt)
                    v[i] = to_store<VS>(kfma<RC>(widen<A>(tq[tb + i]), cr, widen<A>(v[i])));
        }
    }
}

}  // namespace dgpe

namespace dgpe {


// Lane shifts inside rows of 16 lanes (DPP row_shr:D, row_shl:D): lane l
// receives lane l - D (up) or l + D (down) of its row, a lane whose source
// lies outside its row receives 0.  For groups of W <= 16 consecutive lanes
// (W a power of two dividing 16) every source inside the lane's group is
// inside its row, which is all the wave solver uses: every lane whose source
// lies outside its group discards what it receives.  One VALU move per 32-bit
// word, instead of an LDS permute (with zero fill the move needs no copy of
// the old value first).
template <int CTRL>
__device__ __forceinline__ int dpp_word(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __int_as_float(dpp_word<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)dpp_word<CTRL>((int)(unsigned)b);
    const unsigned hi = (unsigned)dpp_word<CTRL>((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int D, typename A>
__device__ __forceinline__ cx<A> row_up(cx<A> v) {
    static_assert(D >= 1 && D <= 15, "row shift");
    return cx<A>{dpp_move<0x110 + D>(v.x), dpp_move<0x110 + D>(v.y)};
}
template <int D, typename A>
__device__ __forceinline__ cx<A> row_down(cx<A> v) {
    static_assert(D >= 1 && D <= 15, "row shift");
    return cx<A>{dpp_move<0x100 + D>(v.x), dpp_move<0x100 + D>(v.y)};
}

// Inclusive scans of the affine maps x -> a x + b over the segments of a line,
// (a2, b2) o (a1, b1) = (a2 a1, a2 b1 + b2): forward (segment s composes
// segments 0..s) and backward (segments s..NSEG-1), in log2(NSEG) steps.
template <int O, int NSEG, bool RC, typename A>
__device__ __forceinline__ void affine_scan_up(cx<A>& a, cx<A>& b, int seg) {
    if constexpr (O < NSEG) {
        const cx<A> ap = row_up<O>(a), bp = row_up<O>(b);
        if (seg >= O) {
            b = kfma<RC>(a, bp, b);
            a = kmul<RC>(a, ap);
        }
        affine_scan_up<2 * O, NSEG, RC>(a, b, seg);
    }
}
template <int O, int NSEG, bool RC, typename A>
__device__ __forceinline__ void affine_scan_down(cx<A>& a, cx<A>& b, int seg) {
    if constexpr (O < NSEG) {
        const cx<A> ap = row_down<O>(a), bp = row_down<O>(b);
        if (seg + O < NSEG) {
            b = kfma<RC>(a, bp, b);
            a = kmul<RC>(a, ap);
        }
        affine_scan_down<2 * O, NSEG, RC>(a, b, seg);
    }
}

// The same exact segmented Crank-Nicolson solve as cn_segment_solve, for
// lines whose NSEG segments sit on NSEG consecutive lanes of one wave (segment
// s on lane s of its group; NSEG a power of two up to 16; full segments).
// Neighbour values and carries move by DPP row shifts, and the carry
// recurrences d_end(k) = dtilde_end(k) + Pend(k) d_end(k-1) (and the backward
// one) are evaluated as inclusive scans of affine maps in log2(NSEG) steps.
// No LDS and no barriers.  Tables: alpha, P, Q (length N; ta, tp, tq point at
// this segment's S entries), pend and qbeg (per segment).  The segment values
// are held in the arithmetic type (holding the FP64 real-time values in FP32
// saves registers the pass cannot use, its occupancy being set by LDS, and
// costs conversions: measured slower).
template <typename T, int S, int NSEG, bool RC, typename TT, typename TS>
__device__ __forceinline__ void cn_segment_solve_wave(cx<cn_acc_t<T, RC>> (&v)[S],
                                                      cx<cn_acc_t<T, RC>> kappa, const TT* ta,
                                                      const TT* tp, const TT* tq, const TS* pend,
                                                      const TS* qbeg, int seg) {
    static_assert(NSEG >= 1 && NSEG <= 16 && (NSEG & (NSEG - 1)) == 0, "segments inside a row");
    using A = cn_acc_t<T, RC>;
    const cx<A> zero = {A(0), A(0)};
    // neighbours
    cx<A> left = zero, right = zero;
    if constexpr (NSEG > 1) {
        left = row_up<1>(v[S - 1]);
        right = row_down<1>(v[0]);
        if (seg == 0) left = zero;
        if (seg == NSEG - 1) right = zero;
    }
    // forward recurrence from a zero carry, r'_i = u_{i-1} + u_{i+1} + kappa u_i
    // formed on the fly from the input values
    cx<A> dcur = zero;
    {
        cx<A> prev = left, cur = v[0];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const cx<A> nxt = (i + 1 < S) ? v[(i + 1 < S) ? i + 1 : i] : right;
            dcur = kmul<RC>(widen<A>(ta[i]), kfma<RC>(kappa, cur, (dcur + prev) + nxt));
            v[i] = dcur;
            prev = cur;
            cur = nxt;
        }
    }
    // forward scan: d at the end of each segment; its left neighbour's is the
    // true d before the segment
    cx<A> a = widen<A>(pend[seg]), b = dcur;
    affine_scan_up<1, NSEG, RC>(a, b, seg);
    cx<A> c = zero;
    if constexpr (NSEG > 1) {
        c = row_up<1>(b);
        if (seg == 0) c = zero;
    }
    // P correction and back substitution from a zero carry.  FP64 factors are
    // read again here rather than kept live since the forward pass (64 registers)
    if constexpr (sizeof(A) == 8) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    cx<A> xcur = zero;
#pragma unroll
    for (int i = S - 1; i >= 0; --i) {
        const cx<A> d = kfma<RC>(widen<A>(tp[i]), c, v[i]);
        xcur = kfma<RC>(widen<A>(ta[i]), xcur, d);
        v[i] = xcur;
    }
    // backward scan: true x at the start of each segment; the right
    // neighbour's is the true x after the segment
    a = widen<A>(qbeg[seg]);
    b = xcur;
    affine_scan_down<1, NSEG, RC>(a, b, seg);
    cx<A> cr = zero;
    if constexpr (NSEG > 1) {
        cr = row_down<1>(b);
        if (seg == NSEG - 1) cr = zero;
    }
#pragma unroll
    for (int i = 0; i < S; ++i) v[i] = kfma<RC>(widen<A>(tq[i]), cr, v[i]);
}

}  // namespace dgpe
