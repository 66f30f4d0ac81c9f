// Device helpers shared by the separable Gaussian-basis kernels: reads of
// uniform tables through the constant address space, the XCD-aware tile
// order, and the symmetric fold of the one-dimensional factors.
#pragma once

#include <type_traits>

#include "internal.hpp"

namespace svc {

// Read-only tables (factors, coefficients, sums) are read through the
// constant address space: every lane reads the same element, so the loads
// become scalar-cache loads into SGPRs that the FMAs take as operands.
template <class T>
using cptr = const __attribute__((address_space(4))) T*;
template <class T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
    return (cptr<T>)(p);
}

__device__ __forceinline__ int sep_xcd_remap(int bid, int n) {
    const int x8 = bid & 7, tt = bid >> 3, q8 = n >> 3, r8 = n & 7;
    return x8 * q8 + (x8 < r8 ? x8 : r8) + tt;
}

// Symmetric fold.  f_e(-w) = (-1)^e f_e(w) and f_e(0) = 0 for e >= 1, so a
// k-tap convolution of a window x is
//   sum_w f_e(w) x[o - w] = f_e(0) x[o] + sum_{w=1..h} f_e(w) (x[o-w] + (-1)^e x[o+w]):
// one add per tap pair, shared by the factors of one parity that use the
// window, and one FMA per factor.  fold_conv applies the NF factors
// f_e, f_{e+2}, ... of parity ODD to a window of NO + 2h samples: out[c][o]
// for the NO outputs; f points at the taps of f_e.  The centre tap is applied
// to the first factor of an even group (it is zero for every other factor).
template <int H, int NF, int NO, bool ODD>
__device__ __forceinline__ void fold_conv(const double (&x)[NO + 2 * H], cptr<double> f,
                                          double (&out)[NF][NO]) {
    constexpr int K = 2 * H + 1;
#pragma unroll
    for (int o = 0; o < NO; ++o) out[0][o] = ODD ? 0.0 : f[H] * x[o + H];
#pragma unroll
    for (int c = 1; c < NF; ++c)
#pragma unroll
        for (int o = 0; o < NO; ++o) out[c][o] = 0.0;
#pragma unroll
    for (int w = 1; w <= H; ++w) {
        double p[NO];
#pragma unroll
        for (int o = 0; o < NO; ++o) p[o] = ODD ? x[o + H - w] - x[o + H + w] : x[o + H - w] + x[o + H + w];
#pragma unroll
        for (int c = 0; c < NF; ++c) {
            const double fw = f[2 * c * K + H + w];
#pragma unroll
            for (int o = 0; o < NO; ++o) out[c][o] = fma(fw, p[o], out[c][o]);
        }
    }
}

// Calls fn(NF) with NF = nf (1 <= nf <= 4) as a compile-time constant.
template <class Fn>
__device__ __forceinline__ void with_nf(int nf, Fn&& fn) {
    switch (nf) {
        case 1: fn(std::integral_constant<int, 1>{}); break;
        case 2: fn(std::integral_constant<int, 2>{}); break;
        case 3: fn(std::integral_constant<int, 3>{}); break;
        default: fn(std::integral_constant<int, 4>{}); break;
    }
}

// Plain k-tap convolution of one factor (no fold): out[o] = sum_u f[u] x[o + 2h - u].
template <int H, int NO>
__device__ __forceinline__ void direct_conv(const double (&x)[NO + 2 * H], cptr<double> f,
                                            double (&out)[NO]) {
#pragma unroll
    for (int o = 0; o < NO; ++o) out[o] = 0.0;
#pragma unroll
    for (int u = 0; u < 2 * H + 1; ++u) {
        const double fu = f[u];
#pragma unroll
        for (int o = 0; o < NO; ++o) out[o] = fma(fu, x[o + 2 * H - u], out[o]);
    }
}

// Cy[q] = sum_ie c[m(ie, q)] xh^ie for q <= DSM, the coefficients of a
// spatial polynomial sum_m c_m P_m in yh at column x; the terms m are ordered
// by total degree, and within one by falling power of xh, and c is padded
// with zeros past the plan's terms, so every instance reads all its terms.
template <int DSM>
__device__ __forceinline__ void coef_in_x(cptr<double> c, const double (&xpow)[DSM + 1],
                                          double (&cy)[DSM + 1]) {
#pragma unroll
    for (int q = 0; q <= DSM; ++q) cy[q] = 0.0;
    int m = 0;
#pragma unroll
    for (int tt = 0; tt <= DSM; ++tt) {
#pragma unroll
        for (int ie = tt; ie >= 0; --ie) cy[tt - ie] = fma(c[m + tt - ie], xpow[ie], cy[tt - ie]);
        m += tt + 1;
    }
}

}  // namespace svc
