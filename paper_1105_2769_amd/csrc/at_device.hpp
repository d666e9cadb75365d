// Device-side building blocks of the Axilrod-Teller potential (Section 1).
//
// With squared side lengths a = r_ij^2, b = r_ik^2, c = r_jk^2 the law of
// cosines gives 8 a b c cos t_i cos t_j cos t_k = (a+b-c)(a-b+c)(-a+b+c), so
//
//   phi = q_a q_b q_c + 3/8 w_a w_b w_c P,   q_x = x^(-3/2), w_x = x^(-5/2),
//   P   = (a + b - c)(c^2 - (a - b)^2)      (any side may play c).
//
// Every pair of points therefore enters only through (x, q_x, w_x), which the
// kernels compute once per pair in binary64 and reuse across many triples.
#pragma once

#include <hip/hip_runtime.h>

namespace mb {

// Pair terms of one pair from its FP64 coordinate difference.  An invalid
// pair (a masked or padded slot) gets a = 1, q = w = 0, so every triple it
// takes part in evaluates to exactly zero without producing Inf or NaN.
__device__ __forceinline__ void pair_terms(double dx, double dy, double dz, bool valid, double &a,
                                           double &q, double &w, double &ia_out) {
    double aa = fma(dx, dx, fma(dy, dy, dz * dz));
    double ra = rsqrt(aa);  // 1 / r
    double ia = ra * ra;    // 1 / a
    double qq = ra * ia;    // a^(-3/2)
    double ww = qq * ia;    // a^(-5/2)
    a = valid ? aa : 1.0;
    q = valid ? qq : 0.0;
    w = valid ? ww : 0.0;
    ia_out = valid ? ia : 0.0;
}

// The same with a = |d|^2 formed in binary64 and rounded once to binary32,
// and q = a^(-3/2), w = a^(-5/2) in binary32 from the hardware reciprocal
// square root (about one ulp; the binary64 route costs three times the
// instructions).  a keeps the binary64-then-rounded value the law-of-cosines
// differences need; q and w are only factors of a triple's value.
__device__ __forceinline__ void pair_terms32(double dx, double dy, double dz, bool valid, float &a,
                                             float &q, float &w, float &ia_out) {
    const float aa = (float)fma(dx, dx, fma(dy, dy, dz * dz));
    const float ra = __builtin_amdgcn_rsqf(aa);  // 1 / r
    const float ia = ra * ra;
    const float qq = ra * ia;
    const float ww = qq * ia;
    a = valid ? aa : 1.0f;
    q = valid ? qq : 0.0f;
    w = valid ? ww : 0.0f;
    ia_out = valid ? ia : 0.0f;
}

// phi of one triangle from its three pair terms (the identity above).
template <typename T>
__device__ __forceinline__ T phi_from_pairs(T a, T qa, T wa, T b, T qb, T wb, T c, T qc, T wc) {
    T d = a - b;
    T t = (a + b) - c;
    T m = fma(-d, d, c * c);
    T P = t * m;
    return fma(T(0.375) * (wa * wb) * wc, P, (qa * qb) * qc);
}

}  // namespace mb
