// Three-body far-field expansion of order p <= 2 (Section 3.2) on the device.
//
// For a point x and two source nodes A, B with centres cA, cB (their
// centroids), the expansion is the degree-p Taylor polynomial of
// phi(x, cA + u, cB + v) in the displacements (u, v), summed over the
// sources: with moments about the centroids the first-order sums vanish, so
//
//   p = 0, 1 : nA nB phi(x, cA, cB)
//   p = 2    : + 1/2 nB tr(H_uu S_A) + 1/2 nA tr(H_vv S_B),
//
// where H_uu, H_vv are the second derivatives of phi in u and in v and S is
// a node's second-moment matrix sum (y - c)(y - c)^T.  The Taylor
// coefficients come from a second-order jet carried through the
// law-of-cosines form phi = (abc)^(-3/2) + 3/8 (abc)^(-5/2) P(a, b, c) with
// a = |x - cA - u|^2, b = |x - cB - v|^2, c = |cA + u - cB - v|^2: the
// value, the gradients in u and v and the u-u and v-v Hessian blocks are
// closed under sums, products and powers (the mixed block is not needed).
#pragma once

#include <hip/hip_runtime.h>

namespace mb {

// Symmetric 3 x 3 matrices are stored as (00, 01, 02, 11, 12, 22).
struct Jet2 {
    double v;
    double gu[3], gv[3];
    double hu[6], hv[6];
};

__device__ __forceinline__ Jet2 jet_const(double c) {
    Jet2 r;
    r.v = c;
    for (int i = 0; i < 3; ++i) r.gu[i] = r.gv[i] = 0.0;
    for (int i = 0; i < 6; ++i) r.hu[i] = r.hv[i] = 0.0;
    return r;
}

// s a + t b
__device__ __forceinline__ Jet2 jet_lin(double s, const Jet2 &a, double t, const Jet2 &b) {
    Jet2 r;
    r.v = s * a.v + t * b.v;
    for (int i = 0; i < 3; ++i) {
        r.gu[i] = s * a.gu[i] + t * b.gu[i];
        r.gv[i] = s * a.gv[i] + t * b.gv[i];
    }
    for (int i = 0; i < 6; ++i) {
        r.hu[i] = s * a.hu[i] + t * b.hu[i];
        r.hv[i] = s * a.hv[i] + t * b.hv[i];
    }
    return r;
}

// g k^T + k g^T in the symmetric storage
__device__ __forceinline__ void sym_outer2(const double *g, const double *k, double *o, double w) {
    o[0] += w * 2.0 * g[0] * k[0];
    o[1] += w * (g[0] * k[1] + k[0] * g[1]);
    o[2] += w * (g[0] * k[2] + k[0] * g[2]);
    o[3] += w * 2.0 * g[1] * k[1];
    o[4] += w * (g[1] * k[2] + k[1] * g[2]);
    o[5] += w * 2.0 * g[2] * k[2];
}

__device__ __forceinline__ Jet2 jet_mul(const Jet2 &a, const Jet2 &b) {
    Jet2 r;
    r.v = a.v * b.v;
    for (int i = 0; i < 3; ++i) {
        r.gu[i] = a.v * b.gu[i] + b.v * a.gu[i];
        r.gv[i] = a.v * b.gv[i] + b.v * a.gv[i];
    }
    for (int i = 0; i < 6; ++i) {
        r.hu[i] = a.v * b.hu[i] + b.v * a.hu[i];
        r.hv[i] = a.v * b.hv[i] + b.v * a.hv[i];
    }
    sym_outer2(a.gu, b.gu, r.hu, 1.0);
    sym_outer2(a.gv, b.gv, r.hv, 1.0);
    return r;
}

// s^e for s.v > 0: first derivative e s^(e-1), second e (e-1) s^(e-2)
__device__ __forceinline__ Jet2 jet_pow(const Jet2 &s, double e) {
    const double f0 = pow(s.v, e);
    const double f1 = e * f0 / s.v;
    const double f2 = (e - 1.0) * f1 / s.v;
    Jet2 r;
    r.v = f0;
    for (int i = 0; i < 3; ++i) {
        r.gu[i] = f1 * s.gu[i];
        r.gv[i] = f1 * s.gv[i];
    }
    for (int i = 0; i < 6; ++i) {
        r.hu[i] = f1 * s.hu[i];
        r.hv[i] = f1 * s.hv[i];
    }
    // f2 g g^T: half of sym_outer2(g, g)
    sym_outer2(s.gu, s.gu, r.hu, 0.5 * f2);
    sym_outer2(s.gv, s.gv, r.hv, 0.5 * f2);
    return r;
}

// |d + su u + sv v|^2 as a jet (su, sv in {-1, 0, 1})
__device__ __forceinline__ Jet2 jet_sqdist(const double d[3], double su, double sv) {
    Jet2 r = jet_const(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int i = 0; i < 3; ++i) {
        r.gu[i] = 2.0 * su * d[i];
        r.gv[i] = 2.0 * sv * d[i];
    }
    const double du = 2.0 * su * su, dv = 2.0 * sv * sv;
    r.hu[0] = r.hu[3] = r.hu[5] = du;
    r.hv[0] = r.hv[3] = r.hv[5] = dv;
    return r;
}

// tr(H S) for symmetric H and S in the storage above
__device__ __forceinline__ double sym_trace_prod(const double *h, const double *s) {
    return h[0] * s[0] + h[3] * s[3] + h[5] * s[5] + 2.0 * (h[1] * s[1] + h[2] * s[2] + h[4] * s[4]);
}

// The expansion of order p (0..2) at x due to nodes A (nA points, centroid
// ca, second moments sa) and B; see the top of this file.
__device__ __forceinline__ double farfield_value(const double x[3], const double ca[3],
                                                 const double cb[3], double na, double nb,
                                                 const double sa[6], const double sb[6], int p) {
    const double dxa[3] = {x[0] - ca[0], x[1] - ca[1], x[2] - ca[2]};
    const double dxb[3] = {x[0] - cb[0], x[1] - cb[1], x[2] - cb[2]};
    const double dab[3] = {ca[0] - cb[0], ca[1] - cb[1], ca[2] - cb[2]};
    const Jet2 a = jet_sqdist(dxa, -1.0, 0.0);  // |x - (ca + u)|^2
    const Jet2 b = jet_sqdist(dxb, 0.0, -1.0);  // |x - (cb + v)|^2
    const Jet2 c = jet_sqdist(dab, 1.0, -1.0);  // |(ca + u) - (cb + v)|^2
    const Jet2 abc = jet_mul(jet_mul(a, b), c);
    const Jet2 t1 = jet_lin(1.0, jet_lin(1.0, a, 1.0, b), -1.0, c);  // a + b - c
    const Jet2 t2 = jet_lin(1.0, jet_lin(1.0, a, -1.0, b), 1.0, c);  // a - b + c
    const Jet2 t3 = jet_lin(1.0, jet_lin(-1.0, a, 1.0, b), 1.0, c);  // -a + b + c
    const Jet2 pp = jet_mul(jet_mul(t1, t2), t3);
    const Jet2 phi = jet_lin(1.0, jet_pow(abc, -1.5), 0.375, jet_mul(jet_pow(abc, -2.5), pp));
    double v = na * nb * phi.v;
    if (p >= 2) v += 0.5 * (nb * sym_trace_prod(phi.hu, sa) + na * sym_trace_prod(phi.hv, sb));
    return v;
}

}  // namespace mb
