// Register-resident DFTs and the two-factor FFT used by the fast spectral
// passes on gfx950.
//
// rdft<T, R, INV>: a DFT of size R (2^a 3^b, R <= 32) on R values in one
// thread's registers, natural order in and out, by a compile-time mixed-radix
// split R = P Q: with n = p + P q,
//   X[k + Q j] = sum_p W_P^{p j} W_R^{p k} sum_q x[p + P q] W_Q^{q k}.
// Twiddles are compile-time constants.
//
// Two-factor FFT of length L = R1 R2 on a sequence spread over R1 threads:
//   phase A: thread t holds x[t + R1 n2] (n2 < R2), applies rdft<R2> and the
//            twiddle W_L^{t k2}; the values go through LDS;
//   phase B: thread u (< R2) gathers the R1 values with index k2 = u, applies
//            rdft<R1> and holds X[u + R2 k1] (k1 < R1).
// The inverse transform of data laid out as after phase B is the same scheme
// with the roles of R1 and R2 exchanged, which returns the original layout.
#pragma once

#include "dgpe_device.h"

namespace dgpe {

// ---- compile-time twiddles exp(-2 pi i m / R) ------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;

// sin and cos of phi in [0, pi/2) by Taylor series (constant evaluation)
constexpr void taylor_sincos(double phi, double& s, double& c) {
    double term_s = phi, term_c = 1.0, ss = 0.0, cc = 0.0;
    const double p2 = phi * phi;
    for (int n = 0; n < 16; ++n) {
        ss += term_s;
        cc += term_c;
        term_s *= -p2 / ((2.0 * n + 2.0) * (2.0 * n + 3.0));
        term_c *= -p2 / ((2.0 * n + 1.0) * (2.0 * n + 2.0));
    }
    s = ss;
    c = cc;
}

template <int R>
struct TwiddleTable {
    double c[R];
    double s[R];  // -sin(2 pi m / R)
    constexpr TwiddleTable() : c(), s() {
        for (int m = 0; m < R; ++m) {
            // 2 pi m / R = q pi/2 + phi with 4m = q R + r, phi = pi r / (2R)
            const int q = (4 * m) / R, r = (4 * m) % R;
            double sp = 0.0, cp = 0.0;
            taylor_sincos(kPi * r / (2.0 * R), sp, cp);
            double cs = cp, sn = sp;
            if (q == 1) { cs = -sp; sn = cp; }
            else if (q == 2) { cs = -cp; sn = -sp; }
            else if (q == 3) { cs = sp; sn = -cp; }
            c[m] = cs;
            s[m] = -sn;
        }
    }
};

template <int R>
inline constexpr TwiddleTable<R> kTwiddle{};

template <typename T, int R, bool INV>
__device__ __forceinline__ cx<T> ctw(int m) {
    return cx<T>{T(kTwiddle<R>.c[m]), T(INV ? -kTwiddle<R>.s[m] : kTwiddle<R>.s[m])};
}

template <int R>
constexpr int rsplit() {
    return (R % 4 == 0 && R != 4) ? 4 : (R % 2 == 0 && R != 2) ? 2 : (R % 3 == 0 && R != 3) ? 3 : R;
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void rdft(cx<T>* v) {
    if constexpr (R == 1) {
        return;
    } else if constexpr (R == 2 || R == 3 || R == 4 || R == 8) {
        dftR<T, R, INV>(v);
    } else {
        constexpr int P = rsplit<R>();
        constexpr int Q = R / P;
        static_assert(P * Q == R && P < R, "radix must factor into 2 and 3");
        cx<T> u[P][Q];
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int q = 0; q < Q; ++q) u[p][q] = v[p + P * q];
#pragma unroll
        for (int p = 0; p < P; ++p) rdft<T, Q, INV>(u[p]);
#pragma unroll
        for (int p = 1; p < P; ++p)
#pragma unroll
            for (int k = 1; k < Q; ++k) u[p][k] = cmul(u[p][k], ctw<T, R, INV>(p * k));
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            cx<T> w[P];
#pragma unroll
            for (int p = 0; p < P; ++p) w[p] = u[p][k];
            rdft<T, P, INV>(w);
#pragma unroll
            for (int j = 0; j < P; ++j) v[k + Q * j] = w[j];
        }
    }
}

// Phase-A twiddle: v[k] *= W_L^{t k} (table tw[m] = W_L^m, conjugated for INV)
template <typename T, int R, bool INV>
__device__ __forceinline__ void twiddle_phase(cx<T>* v, int t, const cx<T>* tw) {
#pragma unroll
    for (int k = 1; k < R; ++k) {
        const cx<T> w = tw[t * k];
        v[k] = INV ? cmulc(v[k], w) : cmul(v[k], w);
    }
}

// (R1, R2) of the two-factor FFT for the lengths with a compiled fast path;
// {0, 0} otherwise.
struct Split2 {
    int r1, r2;
};
inline Split2 fast_split(int L) {
    switch (L) {
        case 16: return {4, 4};
        case 32: return {8, 4};
        case 48: return {8, 6};
        case 64: return {8, 8};
        case 96: return {12, 8};
        case 128: return {16, 8};
        case 192: return {16, 12};
        case 256: return {16, 16};
        case 384: return {24, 16};
        case 512: return {32, 16};
        default: return {0, 0};
    }
}

}  // namespace dgpe
