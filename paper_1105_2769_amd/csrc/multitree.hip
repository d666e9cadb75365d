// Triple-tree (multi-tree) traversal for the Axilrod-Teller potential on
// gfx950: MTPotentialCanonical (Algorithm 2) with the deterministic
// monopole prune (Section 4, Section 4.1) and the Monte Carlo prune
// (Algorithms 3-5), then the top-down pass (Section 3).
//
// The recursion becomes a device-resident LIFO stack of canonical node
// triples, processed in rounds: the host pops the top `chunk` triples and
// enqueues
//   1. classify   - one thread per triple: canonical case, T_i, distance
//                   bounds, deterministic test (a prune is applied at once
//                   with FP64 atomics on node accumulators), Monte Carlo
//                   eligibility, base case or split;
//   2. mc         - one workgroup per eligible triple: per-point sampling
//                   until the termination rule, commit if every point passes;
//                   a failed triple falls through to base case or split;
//   3. base       - one workgroup per leaf triple: exact sum through the
//                   pair-term tiles also used by the exhaustive kernel;
//   4. children   - the canonical children of split triples are compacted in
//                   order onto the stack where the popped triples were;
//   5. refresh    - the node summary statistic Phi^l(P) = min over x in P of
//                   the running lower bound of x is recomputed.
// Popping from the top processes the most recently split triples first, so
// the traversal is depth first across rounds, as the paper's recursion.
// Triples generated early (far apart, high in the tree) wait on the stack
// while the lower bounds of their points grow, which is what lets them be
// pruned when their turn comes.
//
// Readings for the Axilrod-Teller potential (sign-indefinite, not monotone):
// phi = R g with R = (r_12 r_13 r_23)^-3 and g = 1 + 3 cos cos cos is bounded
// over every triangle whose sides lie between the smallest and largest box
// distances d^l, d^u of the three node pairs (at_bounds below), giving
// [phi_lo, phi_hi]: the deterministic test compares phi_hi - phi_lo with the
// allowance and delta^l_i = T_i phi_lo (Section 4, Section 4.1).  The Monte
// Carlo stop rule is z sigma_mu <= (eps (Phi^l + T_i (mu - z sigma_mu)) +
// tau) / T_root with at least m_min samples.  Besides the paper's running
// lower bound (signed statistic) a two-sided statistic keeps a running upper
// bound too and certifies |Phi| from whichever side has settled.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "at_device.hpp"
#include "direct_tile.hpp"
#include "farfield.hpp"
#include "mb_internal.hpp"
#include "multitree.hpp"
#include "tree.hpp"

namespace mb {
namespace {

struct Item {
    int32_t p1, p2, p3, slot;  // canonical node triple; slot = index in the popped chunk
};

struct MtCounters {
    unsigned long long n_base, n_mc, n_units, n_short, n_far;
    unsigned long long det_prunes, mc_prunes, mc_failed, base_cases, base_triples,
        mc_samples;
};

struct MtConst {
    int n;
    double eps, tau, z, t_root;
    double r_min;  // closest pair distance of the point set: a floor for every d^l
    int m_limit, m_min;
    double zeta;
    uint32_t seed32;
    int use_mc;
    int want_cov;
    int two_sided;  // allowance from both running bounds (MB_BOUND_TWO_SIDED)
    int order;      // expansion order of a deterministic prune's estimate (0..2)
};

// A deterministically pruned node triple whose estimate is the far-field
// expansion at each point, with the bounds of its phi.
struct FarItem {
    int32_t p1, p2, p3, pad;
    double lo, hi;
};

// Node statistics of the prune rules, refreshed once per round: over the
// points x of the node, pos = min LB(x), neg = min -UB(x) and
// mix = min max(LB(x), -UB(x)), with LB, UB the running lower and upper
// bounds of what has been credited to x so far.
struct NodeStats {
    const double *pos, *neg, *mix;
};

struct NodeView {
    const int32_t *begin, *end, *left, *right;
    const double *lo, *hi, *centroid;
};

__device__ __forceinline__ int64_t comb2(int64_t n) { return n * (n - 1) / 2; }

__device__ __forceinline__ double box_min_dist(const double *lo1, const double *hi1,
                                               const double *lo2, const double *hi2) {
    double s2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double g = fmax(0.0, fmax(lo1[c] - hi2[c], lo2[c] - hi1[c]));
        s2 = fma(g, g, s2);
    }
    return sqrt(s2);
}

__device__ __forceinline__ double box_max_dist(const double *lo1, const double *hi1,
                                               const double *lo2, const double *hi2) {
    double s2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double g = fmax(fabs(hi2[c] - lo1[c]), fabs(hi1[c] - lo2[c]));
        s2 = fma(g, g, s2);
    }
    return sqrt(s2);
}

// Cosine of the angle between the sides of squared lengths a, b facing the
// side of squared length c (law of cosines).
__device__ __forceinline__ double cos_law(double a, double b, double c) {
    return (a + b - c) / (2.0 * sqrt(a * b));
}

// Range of cos_law over a in [a0, a1], b in [b0, b1], c in [c0, c1] (all
// positive).  cos_law falls with c.  For fixed c it has no stationary point
// inside the (a, b) box, and along an edge it falls then rises, with its
// only minimum where the angle facing the fixed side is right (b = a - c or
// a = b - c), value sqrt(1 - c / fixed side).  So the top is a corner at c0
// and the bottom a corner or such an edge point at c1.  Clipped to [-1, 1],
// where the cosines of real triangles lie.
__device__ __forceinline__ void cos_range(double a0, double a1, double b0, double b1, double c0,
                                          double c1, double &lo, double &hi) {
    hi = fmax(fmax(cos_law(a0, b0, c0), cos_law(a0, b1, c0)),
              fmax(cos_law(a1, b0, c0), cos_law(a1, b1, c0)));
    lo = fmin(fmin(cos_law(a0, b0, c1), cos_law(a0, b1, c1)),
              fmin(cos_law(a1, b0, c1), cos_law(a1, b1, c1)));
    const double ea[2] = {a0, a1}, eb[2] = {b0, b1};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const double bs = ea[e] - c1;  // edge a = ea[e]: right angle where b = a - c
        if (bs > b0 && bs < b1) lo = fmin(lo, sqrt(1.0 - c1 / ea[e]));
        const double as = eb[e] - c1;  // edge b = eb[e]
        if (as > a0 && as < a1) lo = fmin(lo, sqrt(1.0 - c1 / eb[e]));
    }
    lo = fmax(lo, -1.0);
    hi = fmin(hi, 1.0);
}

// [phi_lo, phi_hi] over every triangle whose sides r_12, r_13, r_23 lie in
// [l12, u12], [l13, u13], [l23, u23] (all > 0): phi = R g, R between
// (u12 u13 u23)^-3 and (l12 l13 l23)^-3; g = 1 + 3 c_1 c_2 c_3 from the
// cosine ranges at the three vertices (interval product over its eight
// corners), clipped to [-2, 11/8] (collinear, equilateral).
__device__ __forceinline__ void at_bounds(double l12, double l13, double l23, double u12,
                                          double u13, double u23, double &phi_lo,
                                          double &phi_hi) {
    const double a0 = l12 * l12, a1 = u12 * u12;
    const double b0 = l13 * l13, b1 = u13 * u13;
    const double c0 = l23 * l23, c1 = u23 * u23;
    double x0, x1, y0, y1, z0, z1;
    cos_range(a0, a1, b0, b1, c0, c1, x0, x1);  // vertex 1: sides 12, 13; facing 23
    cos_range(a0, a1, c0, c1, b0, b1, y0, y1);  // vertex 2: sides 12, 23; facing 13
    cos_range(b0, b1, c0, c1, a0, a1, z0, z1);  // vertex 3: sides 13, 23; facing 12
    const double p00 = x0 * y0, p01 = x0 * y1, p10 = x1 * y0, p11 = x1 * y1;
    const double q_lo = fmin(fmin(p00, p01), fmin(p10, p11));
    const double q_hi = fmax(fmax(p00, p01), fmax(p10, p11));
    const double pmin = fmin(fmin(q_lo * z0, q_lo * z1), fmin(q_hi * z0, q_hi * z1));
    const double pmax = fmax(fmax(q_lo * z0, q_lo * z1), fmax(q_hi * z0, q_hi * z1));
    const double g_lo = fmax(-2.0, fma(3.0, pmin, 1.0));
    const double g_hi = fmin(1.375, fma(3.0, pmax, 1.0));
    const double pl = l12 * l13 * l23, pu = u12 * u13 * u23;
    const double r_hi = 1.0 / (pl * pl * pl), r_lo = 1.0 / (pu * pu * pu);
    phi_lo = g_lo * (g_lo >= 0.0 ? r_lo : r_hi);
    phi_hi = g_hi * (g_hi >= 0.0 ? r_hi : r_lo);
}

// Lower bound on |Phi| of every point of node v once it is credited t tuples
// with values in [lo, hi].  Signed (the paper): Phi^l(v) + t lo.  Two-sided:
// the largest of min LB + t lo, min(-UB) - t hi and
// min max(LB, -UB) + min(t lo, -t hi), each a lower bound on the new
// max(LB, -UB) of every point; with all LB > 0 the first is the paper's.
// One node's statistics, read once.
struct NodeAllow {
    double pos, neg, mix;
};
__device__ __forceinline__ NodeAllow node_allow(const NodeStats &ns, int v) {
    return NodeAllow{ns.pos[v], ns.neg[v], ns.mix[v]};
}
__device__ __forceinline__ double certified(const MtConst &k, const NodeAllow &na, double t,
                                            double lo, double hi) {
    const double sg = na.pos + t * lo;
    if (!k.two_sided) return sg;
    return fmax(fmax(sg, na.neg - t * hi), na.mix + fmin(t * lo, -t * hi));
}
__device__ __forceinline__ double certified(const MtConst &k, const NodeStats &ns, int v, double t,
                                            double lo, double hi) {
    return certified(k, node_allow(ns, v), t, lo, hi);
}

// phi of three points from binary64 coordinates (law-of-cosines form).
__device__ __forceinline__ double phi3(const double *a, const double *b, const double *c) {
    double ab, qab, wab, iab, ac, qac, wac, iac, bc, qbc, wbc, ibc;
    pair_terms(b[0] - a[0], b[1] - a[1], b[2] - a[2], true, ab, qab, wab, iab);
    pair_terms(c[0] - a[0], c[1] - a[1], c[2] - a[2], true, ac, qac, wac, iac);
    pair_terms(c[0] - b[0], c[1] - b[1], c[2] - b[2], true, bc, qbc, wbc, ibc);
    return phi_from_pairs<double>(ab, qab, wab, ac, qac, wac, bc, qbc, wbc);
}

// Largest distance from node v's centroid to a corner of its box.
__device__ __forceinline__ double node_radius(const NodeView &nv, int v) {
    double s2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double m = nv.centroid[3 * v + c];
        const double d = fmax(nv.hi[3 * v + c] - m, m - nv.lo[3 * v + c]);
        s2 = fma(d, d, s2);
    }
    return sqrt(s2);
}

// The far-field expansion is a Taylor series in the displacements of the
// source points from their centres; it converges only for nodes small
// against their distances.  Accepted when every two nodes of the triple
// have r_a + r_b <= 1/2 |c_a - c_b|.
__device__ __forceinline__ bool well_separated(const NodeView &nv, int p1, int p2, int p3) {
    const int a[3] = {p1, p1, p2}, b[3] = {p2, p3, p3};
    for (int q = 0; q < 3; ++q) {
        const double *ca = nv.centroid + 3 * a[q], *cb = nv.centroid + 3 * b[q];
        const double dx = ca[0] - cb[0], dy = ca[1] - cb[1], dz = ca[2] - cb[2];
        const double d = sqrt(fma(dx, dx, fma(dy, dy, dz * dz)));
        if (node_radius(nv, a[q]) + node_radius(nv, b[q]) > 0.5 * d) return false;
    }
    return true;
}

// Distinct nodes of a canonical triple, each with its T_i and its first slot.
struct Roles {
    int n_roles;
    int node[3];
    int slot[3];
    int64_t t[3];
};

__device__ __forceinline__ char canonical_case(int p1, int p2, int p3) {
    if (p1 == p2 && p2 == p3) return 'a';
    if (p1 == p2) return 'b';
    if (p2 == p3) return 'c';
    return 'd';
}

__device__ __forceinline__ Roles roles_of(int p1, int p2, int p3, int64_t n1, int64_t n2,
                                          int64_t n3) {
    Roles r;
    const char cs = canonical_case(p1, p2, p3);
    if (cs == 'a') {
        r.n_roles = 1;
        r.node[0] = p1; r.slot[0] = 0; r.t[0] = comb2(n1 - 1);
    } else if (cs == 'b') {
        r.n_roles = 2;
        r.node[0] = p1; r.slot[0] = 0; r.t[0] = (n1 - 1) * n3;
        r.node[1] = p3; r.slot[1] = 2; r.t[1] = comb2(n1);
    } else if (cs == 'c') {
        r.n_roles = 2;
        r.node[0] = p1; r.slot[0] = 0; r.t[0] = comb2(n2);
        r.node[1] = p2; r.slot[1] = 1; r.t[1] = n1 * (n2 - 1);
    } else {
        r.n_roles = 3;
        r.node[0] = p1; r.slot[0] = 0; r.t[0] = n2 * n3;
        r.node[1] = p2; r.slot[1] = 1; r.t[1] = n1 * n3;
        r.node[2] = p3; r.slot[2] = 2; r.t[2] = n1 * n2;
    }
    return r;
}

// Canonical children (every non-leaf node split, one copy per pair of equal
// nodes): written to out[0..count), returns count (<= 8).
__device__ int canonical_children(const NodeView &nv, int p1, int p2, int p3, Item *out) {
    auto opts = [&](int v, int *o) -> int {
        if (nv.left[v] < 0) {
            o[0] = v;
            return 1;
        }
        o[0] = nv.left[v];
        o[1] = nv.right[v];
        return 2;
    };
    const char cs = canonical_case(p1, p2, p3);
    int cnt = 0;
    int oa[2], ob[2];
    if (cs == 'a') {
        const int na = opts(p1, oa);
        for (int x = 0; x < na; ++x)
            for (int y = x; y < na; ++y)
                for (int z = y; z < na; ++z) out[cnt++] = Item{oa[x], oa[y], oa[z], 0};
    } else if (cs == 'b') {
        const int na = opts(p1, oa), nb = opts(p3, ob);
        for (int x = 0; x < na; ++x)
            for (int y = x; y < na; ++y)
                for (int z = 0; z < nb; ++z) out[cnt++] = Item{oa[x], oa[y], ob[z], 0};
    } else if (cs == 'c') {
        const int na = opts(p1, oa), nb = opts(p2, ob);
        for (int x = 0; x < na; ++x)
            for (int y = 0; y < nb; ++y)
                for (int z = y; z < nb; ++z) out[cnt++] = Item{oa[x], ob[y], ob[z], 0};
    } else {
        int oc[2];
        const int na = opts(p1, oa), nb = opts(p2, ob), nc = opts(p3, oc);
        for (int x = 0; x < na; ++x)
            for (int y = 0; y < nb; ++y)
                for (int z = 0; z < nc; ++z) out[cnt++] = Item{oa[x], ob[y], oc[z], 0};
    }
    return cnt;
}

__device__ __forceinline__ void emit_children(const NodeView &nv, const Item &it, int slot,
                                              Item *__restrict__ child_buf,
                                              uint8_t *__restrict__ child_flag) {
    Item ch[8];
    const int c = canonical_children(nv, it.p1, it.p2, it.p3, ch);
    for (int q = 0; q < 8; ++q) {
        if (q < c) child_buf[8 * slot + q] = ch[q];
        child_flag[8 * slot + q] = q < c ? 1 : 0;
    }
}

// A slot of a list for every lane of the wave with `want`, by one atomic
// per wave: the lanes that ask are numbered in lane order from the count the
// first of them takes.  Every lane of the wave calls it (convergent); the
// result is meaningful only where want is true.
__device__ __forceinline__ unsigned long long wave_append(unsigned long long *counter, bool want) {
    const unsigned long long mask = __ballot(want);
    if (mask == 0) return 0;
    const int lane = threadIdx.x & 63;
    const int first = __ffsll((long long)mask) - 1;
    unsigned long long base = 0;
    if (lane == first) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)base, first);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(base >> 32), first);
    base = ((unsigned long long)hi << 32) | lo;
    return base + (unsigned long long)__popcll(mask & ((1ull << lane) - 1ull));
}

// counter += the sum of v over the lanes of the wave, by one atomic per
// wave (every lane calls it)
__device__ __forceinline__ void wave_add(unsigned long long *counter, unsigned long long v) {
    const unsigned long long mask = __ballot(v != 0);
    if (mask == 0) return;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    if ((threadIdx.x & 63) == __ffsll((long long)mask) - 1) atomicAdd(counter, v);
}

// What classification decided for a triple; the list appends are made by
// the caller, a wave at a time.
enum Outcome : int { kNone, kSplit, kDeferred, kFar, kPruned, kToMc, kToBase };

// 1. classification of one popped triple (slot `slot` of the round)
__device__ __forceinline__ int classify_one(
    Item &it, int slot, const NodeView &nv, const NodeStats &ns, double *__restrict__ node_acc,
    double *__restrict__ node_lo, double *__restrict__ node_hi,
    unsigned long long *__restrict__ node_cov, const MtConst &k, Item *__restrict__ child_buf,
    uint8_t *__restrict__ child_flag, double spread_limit, Item *__restrict__ defer_buf,
    uint8_t *__restrict__ defer_flag, double &far_lo, double &far_hi) {
    for (int q = 0; q < 8; ++q) child_flag[8 * slot + q] = 0;
    defer_flag[slot] = 0;
    const int p1 = it.p1, p2 = it.p2, p3 = it.p3;
    const int64_t n1 = nv.end[p1] - nv.begin[p1], n2 = nv.end[p2] - nv.begin[p2],
                  n3 = nv.end[p3] - nv.begin[p3];
    const Roles r = roles_of(p1, p2, p3, n1, n2, n3);
    const double *lo = nv.lo, *hi = nv.hi;
    // box distances of the distinct node pairs
    double d12 = 0.0, d13 = 0.0, d23 = 0.0;
    if (r.n_roles == 3) {
        d12 = box_min_dist(lo + 3 * p1, hi + 3 * p1, lo + 3 * p2, hi + 3 * p2);
        d13 = box_min_dist(lo + 3 * p1, hi + 3 * p1, lo + 3 * p3, hi + 3 * p3);
        d23 = box_min_dist(lo + 3 * p2, hi + 3 * p2, lo + 3 * p3, hi + 3 * p3);
    } else if (r.n_roles == 2) {
        d12 = box_min_dist(lo + 3 * r.node[0], hi + 3 * r.node[0], lo + 3 * r.node[1],
                           hi + 3 * r.node[1]);
    }
    // spread: the largest box distance between two nodes of the triple; it
    // never decreases when a triple is split, so triples can be taken in
    // bands of increasing spread
    if (fmax(d12, fmax(d13, d23)) > spread_limit) {
        defer_buf[slot] = it;
        defer_flag[slot] = 1;
        return kDeferred;
    }

    // bounds on phi over the triple: no two points are closer than r_min, so
    // every d^l is raised to it (a node paired with itself has d^l = 0); d^u
    // is the farthest pair of box corners
    const int pa[3] = {p1, p1, p2}, pb[3] = {p2, p3, p3};
    double dl[3], du[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double *la = lo + 3 * pa[q], *ha = hi + 3 * pa[q], *lb = lo + 3 * pb[q],
                     *hb = hi + 3 * pb[q];
        dl[q] = fmax(pa[q] == pb[q] ? 0.0 : box_min_dist(la, ha, lb, hb), k.r_min);
        du[q] = fmax(box_max_dist(la, ha, lb, hb), dl[q]);
    }
    double phi_lo, phi_hi;
    at_bounds(dl[0], dl[1], dl[2], du[0], du[1], du[2], phi_lo, phi_hi);

    // deterministic prune (three distinct nodes)
    if (r.n_roles == 3) {
        double allow = INFINITY;
        for (int q = 0; q < 3; ++q)
            allow = fmin(allow, certified(k, ns, r.node[q], (double)r.t[q], phi_lo, phi_hi));
        if (phi_hi - phi_lo <= (k.eps * allow + k.tau) / k.t_root) {
            const bool far = k.order >= 1 && well_separated(nv, p1, p2, p3);
            if (far) {
                // the far-field expansion at each point (far_kernel)
                far_lo = phi_lo;
                far_hi = phi_hi;
            } else {
                // monopole estimate at the centroids, kept inside the bound interval
                double phic =
                    phi3(nv.centroid + 3 * p1, nv.centroid + 3 * p2, nv.centroid + 3 * p3);
                phic = isfinite(phic) ? fmin(fmax(phic, phi_lo), phi_hi) : 0.5 * (phi_lo + phi_hi);
                for (int q = 0; q < 3; ++q)
                    atomicAdd(&node_acc[r.node[q]], (double)r.t[q] * phic);
            }
            for (int q = 0; q < 3; ++q) {
                atomicAdd(&node_lo[r.node[q]], (double)r.t[q] * phi_lo);
                atomicAdd(&node_hi[r.node[q]], (double)r.t[q] * phi_hi);
                if (k.want_cov) atomicAdd(&node_cov[r.node[q]], (unsigned long long)r.t[q]);
            }
            return far ? kFar : kPruned;
        }
    }
    // Monte Carlo candidate.  A point can pass the stop rule only if its
    // allowance is >= 0 (z sigma_mu >= 0); the allowance is largest for a
    // sample mean inside [phi_lo, phi_hi] with sigma_mu = 0, so a node whose
    // allowance is negative even then fails for certain and the triple skips
    // the sampling.
    if (k.use_mc) {
        int64_t tmin = r.t[0];
        for (int q = 1; q < r.n_roles; ++q) tmin = min(tmin, r.t[q]);
        bool can_pass = tmin > 0 && k.zeta * (double)k.m_limit <= (double)tmin;
        for (int q = 0; q < r.n_roles && can_pass; ++q) {
            const int v = r.node[q];
            const double t = (double)r.t[q];
            double best = ns.pos[v] + t * phi_hi;
            if (k.two_sided) best = fmax(fmax(best, ns.neg[v] - t * phi_lo), ns.mix[v]);
            can_pass = k.eps * best + k.tau >= 0.0;
        }
        if (can_pass) return kToMc;
    }
    const bool all_leaves = nv.left[p1] < 0 && nv.left[p2] < 0 && nv.left[p3] < 0;
    if (all_leaves) return kToBase;
    emit_children(nv, it, slot, child_buf, child_flag);
    return kSplit;
}

__global__ __launch_bounds__(256) void classify_kernel(
    const Item *__restrict__ items, int n_items, NodeView nv, NodeStats ns,
    double *__restrict__ node_acc, double *__restrict__ node_lo, double *__restrict__ node_hi,
    unsigned long long *__restrict__ node_cov, MtConst k, MtCounters *__restrict__ ctr,
    Item *__restrict__ mc_list, Item *__restrict__ base_list, Item *__restrict__ child_buf,
    uint8_t *__restrict__ child_flag, double spread_limit, Item *__restrict__ defer_buf,
    uint8_t *__restrict__ defer_flag, FarItem *__restrict__ far_list) {
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    int outcome = kNone;
    Item it{};
    double far_lo = 0.0, far_hi = 0.0;
    if (slot < n_items) {
        it = items[slot];
        it.slot = slot;
        outcome = classify_one(it, slot, nv, ns, node_acc, node_lo, node_hi, node_cov, k,
                               child_buf, child_flag, spread_limit, defer_buf, defer_flag, far_lo,
                               far_hi);
    }
    // list appends and the prune count, one atomic per wave each
    const unsigned long long pf = wave_append(&ctr->n_far, outcome == kFar);
    if (outcome == kFar) far_list[pf] = FarItem{it.p1, it.p2, it.p3, 0, far_lo, far_hi};
    const unsigned long long pm = wave_append(&ctr->n_mc, outcome == kToMc);
    if (outcome == kToMc) mc_list[pm] = it;
    const unsigned long long pb = wave_append(&ctr->n_base, outcome == kToBase);
    if (outcome == kToBase) base_list[pb] = it;
    wave_add(&ctr->det_prunes, outcome == kPruned || outcome == kFar ? 1ull : 0ull);
}

// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32 -> 64-bit
// multiplications with key bumps by the Weyl constants in between.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
    }
}

// Unordered pair (u < v) of [0, m) from its index t in [0, C(m, 2)), v-major.
__device__ __forceinline__ void pair_from_index(uint64_t t, int64_t &u, int64_t &v) {
    int64_t vv = (int64_t)floor((1.0 + sqrt(1.0 + 8.0 * (double)t)) * 0.5);
    while (vv * (vv - 1) / 2 > (int64_t)t) --vv;
    while ((vv + 1) * vv / 2 <= (int64_t)t) ++vv;
    v = vv;
    u = (int64_t)t - vv * (vv - 1) / 2;
}

// How one uniform 64-bit integer r picks the two partners of a point x
// (offset xl inside its node, at slot `slot` of the node triple): the
// T_i partner tuples are numbered 0..range-1, t = floor(r range / 2^64), and
// t is decoded either as an unordered pair of one node (pair_from_index) or
// as (t / div, t mod div) over two nodes, skipping x itself where a partner
// comes from x's own node.  Set up once per point.
struct PartnerMap {
    uint64_t range;
    double inv;       // 1 / div
    int32_t div;      // product decode: second partner's range
    int32_t skip_u, skip_v;  // a partner offset >= skip is moved up by one
    int32_t pair;     // 1: unordered pair of one node
    int32_t su, sv;   // slots of the partners' nodes
};

__device__ __forceinline__ PartnerMap partner_map(char cs, int slot, int64_t xl, int64_t n1,
                                                  int64_t n2, int64_t n3) {
    constexpr int32_t kNone = INT32_MAX;
    PartnerMap m;
    m.div = 1;
    m.skip_u = m.skip_v = kNone;
    if (cs == 'a') {  // a pair of A minus x
        m.pair = 1; m.range = (uint64_t)comb2(n1 - 1); m.su = m.sv = 0;
        m.skip_u = m.skip_v = (int32_t)xl;
    } else if (cs == 'b' && slot == 0) {  // x in A: one partner in A minus x, one in B
        m.pair = 0; m.range = (uint64_t)((n1 - 1) * n3); m.div = (int32_t)n3; m.su = 0; m.sv = 2;
        m.skip_u = (int32_t)xl;
    } else if (cs == 'b') {  // x in B: a pair of A
        m.pair = 1; m.range = (uint64_t)comb2(n1); m.su = m.sv = 0;
    } else if (cs == 'c' && slot == 0) {  // x in A: a pair of B
        m.pair = 1; m.range = (uint64_t)comb2(n2); m.su = m.sv = 1;
    } else if (cs == 'c') {  // x in B: one partner in A, one in B minus x
        m.pair = 0; m.range = (uint64_t)(n1 * (n2 - 1)); m.div = (int32_t)(n2 - 1); m.su = 0;
        m.sv = 1;
        m.skip_v = (int32_t)xl;
    } else {  // three distinct nodes: one partner in each of the other two
        m.su = slot == 0 ? 1 : 0;
        m.sv = slot == 2 ? 1 : 2;
        const int64_t na = m.su == 0 ? n1 : n2, nb = m.sv == 1 ? n2 : n3;
        m.pair = 0; m.range = (uint64_t)(na * nb); m.div = (int32_t)nb;
    }
    m.inv = 1.0 / (double)m.div;
    return m;
}

// Partner offsets (u, v) inside their nodes for one uniform integer r.  The
// quotient t / div comes from binary64 (t < 2^53, so the estimate is off by
// at most one) and is corrected exactly.
__device__ __forceinline__ void partners(const PartnerMap &m, uint64_t r, int64_t &u, int64_t &v) {
    const uint64_t t = __umul64hi(r, m.range);
    if (m.pair) {
        pair_from_index(t, u, v);
    } else {
        int64_t q = (int64_t)((double)t * m.inv);
        int64_t rem = (int64_t)t - q * m.div;
        if (rem < 0) {
            --q;
            rem += m.div;
        } else if (rem >= m.div) {
            ++q;
            rem -= m.div;
        }
        u = q;
        v = rem;
    }
    u += u >= m.skip_u;
    v += v >= m.skip_v;
}

constexpr int kMcThreads = 256;
#ifndef MB_MC_WAVES
#define MB_MC_WAVES 3  // waves per SIMD the sampler's registers must allow
#endif
constexpr int kMcCache = 2048;  // points whose (mu, lower bound) stay in LDS between passes

struct McPoint {
    bool pass;
    double mean, sig;
    int drawn;
};

// v from lane l - D of the same row of 16 lanes (DPP row_shr:D); the first
// D lanes of a row receive 0.
template <int D>
__device__ __forceinline__ double row_shr(double v) {
    static_assert(D >= 1 && D <= 15, "row shift");
    const unsigned long long b = __double_as_longlong(v);
    // bound_ctrl: a lane whose source lies before its row reads 0
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, 0x110 + D, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), 0x110 + D, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned)lo));
}

// Inclusive prefix sum over each aligned group of W lanes (4, 8 or 16; gl:
// lane in group).  A row shift fills the first lanes of a 16-lane row with
// 0; a smaller group masks what it would take from the group before it.
template <int W>
__device__ __forceinline__ double group_incl_scan(double v, int gl) {
    static_assert(W == 4 || W == 8 || W == 16, "a DPP row or a part of one");
    double u = row_shr<1>(v);
    v += (W == 16 || gl >= 1) ? u : 0.0;
    u = row_shr<2>(v);
    v += (W == 16 || gl >= 2) ? u : 0.0;
    if constexpr (W >= 8) {
        u = row_shr<4>(v);
        v += (W == 16 || gl >= 4) ? u : 0.0;
    }
    if constexpr (W == 16) v += row_shr<8>(v);
    return v;
}

// phi of the triangle (x, a, b) from binary64 coordinates, evaluated in
// binary32 after an exact power-of-two rescaling: the squared sides are
// formed in binary64 and divided by 4^e so that the longest lies in [1, 4)
// (the triangle inequality keeps a second side >= 1/4 of it), and since phi
// is homogeneous of degree -9/2 in the squared sides the binary32 value is
// multiplied back by 2^(-9 e).  Monte Carlo samples only: their relative
// error (about 1e-6 away from collinear triangles) is far below the
// statistical error they are averaged into.
__device__ __forceinline__ double phi_sample(double x0, double x1, double x2, const double *a,
                                             const double *b) {
    const double dx = a[0] - x0, dy = a[1] - x1, dz = a[2] - x2;
    const double ex = b[0] - x0, ey = b[1] - x1, ez = b[2] - x2;
    const double fx = b[0] - a[0], fy = b[1] - a[1], fz = b[2] - a[2];
    const double s_ab = fma(dx, dx, fma(dy, dy, dz * dz));
    const double s_ac = fma(ex, ex, fma(ey, ey, ez * ez));
    const double s_bc = fma(fx, fx, fma(fy, fy, fz * fz));
    const double mx = fmax(s_ab, fmax(s_ac, s_bc));
    const int e = (__builtin_amdgcn_frexp_exp(mx) - 1) >> 1;  // 4^e <= mx < 4^(e+1)
    const float A = (float)__builtin_amdgcn_ldexp(s_ab, -2 * e);
    const float B = (float)__builtin_amdgcn_ldexp(s_ac, -2 * e);
    const float C = (float)__builtin_amdgcn_ldexp(s_bc, -2 * e);
    auto terms = [](float v, float &q, float &w) {
        const float r = __builtin_amdgcn_rsqf(v);
        const float iv = r * r;
        q = r * iv;
        w = q * iv;
    };
    float qa, wa, qb, wb, qc, wc;
    terms(A, qa, wa);
    terms(B, qb, wb);
    terms(C, qc, wc);
    const float f = phi_from_pairs<float>(A, qa, wa, B, qb, wb, C, qc, wc);
    return __builtin_amdgcn_ldexp((double)f, -9 * e);
}

// Algorithm 4 for one point, by a group of kMcGroup lanes of a wave:
// samples are drawn kMcBatch at a time, lane l of the group taking samples
// kMcPer l .. kMcPer l + kMcPer - 1 of the batch, two from each Philox block
// (sample s uses counter s / 2, half s mod 2); prefix sums give
// the running mean and unbiased variance after every sample, and the first
// sample count m at which the sequential loop would stop - the termination
// rule holding with m >= m_min, or m = m_limit - is found with a ballot.
// The decision depends only on the sample sequence, not on the group width;
// the width sets how many samples past the stop are drawn (a point that
// stops at m_min = 30 draws 32).  Every lane of the group returns the same
// result.  `failed` (nullable) aborts between batches.  gl: lane in the
// group, g0: the group's first lane in the wave.
#ifndef MB_MC_PER
#define MB_MC_PER 4
#endif
constexpr int kMcPer = MB_MC_PER;        // samples per lane per batch (even)
constexpr int kMcBatch = 32;              // samples per batch of a point
constexpr int kMcGroup = kMcBatch / kMcPer;  // lanes per point

// Running statistics after sample count m (m >= 1) from the shifted sums
// t1 = sum (f - f0), t2 = sum (f - f0)^2.
//
// The rule z s <= (eps C(mu - z s, mu + z s) + tau) / T_root, s = sigma_mu,
// is tested without a square root or a division: every term of the credit
// C is linear in z s with slope -T_i (`certified`), C = C0 - T_i z s, so the
// rule reads z s <= R = (eps C0 + tau) / (T_root + eps T_i), i.e.
// R >= 0 and z^2 s^2 <= R^2; den = 1 / (T_root + eps T_i) is set per point.
struct McStat {
    bool ok, stop;
    double mean, var_mu;  // running mean and sigma_mu^2
};
__device__ __forceinline__ McStat mc_stat(double f0, double t1, double t2, int m, double t,
                                          const NodeAllow &na, const MtConst &k, double den) {
    const double dm = (double)m;
    double im = __builtin_amdgcn_rcp(dm);  // 1/m: hardware estimate, one Newton step
    im = fma(fma(-dm, im, 1.0), im, im);
    double im1 = __builtin_amdgcn_rcp(dm - 1.0);
    im1 = fma(fma(-(dm - 1.0), im1, 1.0), im1, im1);
    McStat r;
    r.mean = fma(t1, im, f0);
    r.var_mu = m >= 2 ? fmax(fma(-t1 * t1, im, t2), 0.0) * im1 * im : 0.0;
    const double tm = t * r.mean;
    double c0 = na.pos + tm;
    if (k.two_sided) c0 = fmax(fmax(c0, na.neg - tm), na.mix - fabs(tm));
    const double R = (k.eps * c0 + k.tau) * den;
    const bool cond = m >= 2 && R >= 0.0 && k.z * k.z * r.var_mu <= R * R;
    r.ok = cond && m >= k.m_min;
    r.stop = r.ok || m == k.m_limit;
    return r;
}

// Algorithm 4 for one point in progress, held by a group: the point, its
// partner map and node statistics, and the sums over the batches so far.
struct McRun {
    PartnerMap pm;
    NodeAllow na;
    int32_t xr, bu, bv;
    double x0, x1, x2, t, den;
    double f0, s1, s2;
    int base;
};

__device__ __forceinline__ void mc_begin(McRun &r, const PartnerMap &pm, int64_t xr,
                                         const int64_t nb[3], const double *__restrict__ xs,
                                         double t, const NodeStats &ns, int node,
                                         const MtConst &k) {
    r.pm = pm;
    r.na = node_allow(ns, node);
    r.xr = (int32_t)xr;
    r.bu = pm.su == 0 ? nb[0] : (pm.su == 1 ? nb[1] : nb[2]);
    r.bv = pm.sv == 0 ? nb[0] : (pm.sv == 1 ? nb[1] : nb[2]);
    r.x0 = xs[3 * xr];
    r.x1 = xs[3 * xr + 1];
    r.x2 = xs[3 * xr + 2];
    r.t = t;
    r.den = 1.0 / (k.t_root + k.eps * t);
    r.f0 = r.s1 = r.s2 = 0.0;
    r.base = 0;
}

// One batch of kMcBatch samples of the point in r.  Returns true when the
// test of the point has ended, with its result in res.
__device__ __forceinline__ bool mc_batch(McRun &r, const Item &it, const double *__restrict__ xs,
                                         const MtConst &k, int gl, int g0, McPoint &res) {
    constexpr int W = kMcGroup, E = kMcPer;
    const int base = r.base;
    const int sa = base + E * gl;  // this lane's samples sa .. sa + E - 1
    double f[E];
    bool v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        v[e] = sa + e < k.m_limit;
        f[e] = 0.0;
    }
    if (v[0]) {
        // all the lane's partner tuples first, so that their point loads are
        // in flight together (a tuple is valid even when its sample lies
        // past m_limit; its value is then unused)
        int64_t u[E], w[E];
#pragma unroll
        for (int h = 0; h < E / 2; ++h) {
            uint32_t c[4] = {(uint32_t)r.xr, (uint32_t)((sa >> 1) + h), (uint32_t)it.p1,
                             (uint32_t)it.p2};
            philox4x32_10(c, (uint32_t)it.p3, k.seed32);
            partners(r.pm, ((uint64_t)c[1] << 32) | c[0], u[2 * h], w[2 * h]);
            partners(r.pm, ((uint64_t)c[3] << 32) | c[2], u[2 * h + 1], w[2 * h + 1]);
        }
        double pu[E][3], pw[E][3];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const double *a = xs + 3 * (r.bu + u[e]), *b = xs + 3 * (r.bv + w[e]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                pu[e][c] = a[c];
                pw[e][c] = b[c];
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const double fe = phi_sample(r.x0, r.x1, r.x2, pu[e], pw[e]);
            f[e] = v[e] ? fe : 0.0;
        }
    }
    if (base == 0) r.f0 = __shfl(f[0], g0);  // shift for numerically stable sums
    double g[E], l1 = 0.0, l2 = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        g[e] = v[e] ? f[e] - r.f0 : 0.0;
        l1 += g[e];
        l2 = fma(g[e], g[e], l2);
    }
    const double p1 = group_incl_scan<W>(l1, gl), p2 = group_incl_scan<W>(l2, gl);
    // sums through each of the lane's samples, from the last one down
    McStat S[E];
    bool stop[E];
    {
        double q1 = r.s1 + p1, q2 = r.s2 + p2;
#pragma unroll
        for (int e = E - 1; e >= 0; --e) {
            S[e] = mc_stat(r.f0, q1, q2, sa + e + 1, r.t, r.na, k, r.den);
            stop[e] = v[e] && S[e].stop;
            q1 -= g[e];
            q2 = fma(-g[e], g[e], q2);
        }
    }
    bool any = false;
    int first = E - 1;
#pragma unroll
    for (int e = E - 1; e >= 0; --e)
        if (stop[e]) {
            any = true;
            first = e;
        }
    // this group's bits of the wave's ballot
    const unsigned long long bal = (__ballot(any) >> g0) & ((1ull << W) - 1ull);
    const int drawn = min(base + kMcBatch, k.m_limit);
    if (bal) {
        const int L = g0 + __ffsll((long long)bal) - 1;
        bool ok = false;
        double mean = 0.0, var_mu = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (e == first) {
                ok = S[e].ok;
                mean = S[e].mean;
                var_mu = S[e].var_mu;
            }
        res.pass = __shfl((int)ok, L) != 0;
        res.mean = __shfl(mean, L);
        res.sig = sqrt(__shfl(var_mu, L));
        res.drawn = drawn;
        return true;
    }
    if (drawn >= k.m_limit) {
        res.pass = false;
        res.mean = res.sig = 0.0;
        res.drawn = drawn;
        return true;
    }
    r.s1 += __shfl(p1, g0 + W - 1);
    r.s2 += __shfl(p2, g0 + W - 1);
    r.base = base + kMcBatch;
    return false;
}

// Algorithm 4 for one point from start to end; `failed` (nullable) is
// checked between batches and ends the test as a failure once set.
__device__ McPoint mc_point_group(const Item &it, const PartnerMap &pm, int64_t xr,
                                  const int64_t nb[3], const double *__restrict__ xs, double t,
                                  const NodeStats &ns, int node, const MtConst &k,
                                  const volatile int *failed, int gl, int g0) {
    McRun run;
    mc_begin(run, pm, xr, nb, xs, t, ns, node, k);
    McPoint res;
    while (!mc_batch(run, it, xs, k, gl, g0, res)) {
        if (failed && *failed) {
            res.pass = false;
            res.mean = res.sig = 0.0;
            res.drawn = run.base;
            break;
        }
    }
    return res;
}

// 2. Monte Carlo test and commit (Algorithms 3-5), one workgroup per triple.
// Groups of kMcGroup lanes take the points of the distinct nodes in turn;
// the triple is summarized only if every point passes (any failure ends the
// test), in which case the points are credited T_i mu and
// T_i (mu - z sigma_mu).
__global__ __launch_bounds__(kMcThreads, MB_MC_WAVES) void mc_kernel(
    const Item *__restrict__ mc_list, NodeView nv, const double *__restrict__ xs, NodeStats ns,
    double *__restrict__ est, double *__restrict__ dev,
    unsigned long long *__restrict__ node_cov, MtConst k, MtCounters *__restrict__ ctr,
    Item *__restrict__ base_list, Item *__restrict__ child_buf, uint8_t *__restrict__ child_flag) {
    __shared__ int failed;
    __shared__ double c_mean[kMcCache], c_dev[kMcCache];
    const int lane = threadIdx.x & 63;
    // groups of kMcGroup lanes, each sampling its own points
    constexpr int kGroups = kMcThreads / kMcGroup;
    const int grp = threadIdx.x / kMcGroup;
    const int gl = lane % kMcGroup, g0 = lane - gl;
    const unsigned long long n_mc = ctr->n_mc;
    // counters, summed over this workgroup's triples and added once at the end
    unsigned long long drawn = 0, my_failed = 0, my_prunes = 0;
    for (unsigned long long w = blockIdx.x; w < n_mc; w += gridDim.x) {
        const Item it = mc_list[w];
        const int64_t nb[3] = {nv.begin[it.p1], nv.begin[it.p2], nv.begin[it.p3]};
        const int64_t n1 = nv.end[it.p1] - nv.begin[it.p1], n2 = nv.end[it.p2] - nv.begin[it.p2],
                      n3 = nv.end[it.p3] - nv.begin[it.p3];
        const Roles r = roles_of(it.p1, it.p2, it.p3, n1, n2, n3);
        const char cs = canonical_case(it.p1, it.p2, it.p3);
        int64_t sz[3] = {0, 0, 0}, total = 0;
        for (int q = 0; q < r.n_roles; ++q) {
            sz[q] = nv.end[r.node[q]] - nv.begin[r.node[q]];
            total += sz[q];
        }
        // points of the node with the smallest allowance first: a triple that
        // fails usually fails there, and the test ends at the first failure.
        // The order changes no point's samples or result.
        int qo[3] = {0, 1, 2};
        double key[3];
        for (int q = 0; q < r.n_roles; ++q) key[q] = certified(k, ns, r.node[q], 0.0, 0.0, 0.0);
        for (int a = 1; a < r.n_roles; ++a)
            for (int b = a; b > 0 && key[qo[b]] < key[qo[b - 1]]; --b) {
                const int tmp = qo[b];
                qo[b] = qo[b - 1];
                qo[b - 1] = tmp;
            }
        const int64_t szo[3] = {sz[qo[0]], sz[qo[1]], sz[qo[2]]};
        __syncthreads();
        if (threadIdx.x == 0) failed = 0;
        __syncthreads();
        for (int64_t e = grp; e < total; e += kGroups) {
            if (*(volatile int *)&failed) break;
            int qq = 0;
            int64_t off = e;
            while (off >= szo[qq]) off -= szo[qq++];
            const int q = qo[qq];
            const McPoint res = mc_point_group(it, partner_map(cs, r.slot[q], off, n1, n2, n3),
                                               nv.begin[r.node[q]] + off, nb, xs, (double)r.t[q],
                                               ns, r.node[q], k, &failed, gl, g0);
            drawn += res.drawn;
            if (!res.pass) {
                if (gl == 0) failed = 1;
                break;
            }
            if (e < kMcCache && gl == 0) {
                c_mean[e] = res.mean;
                c_dev[e] = k.z * res.sig;
            }
        }
        __syncthreads();
        if (failed) {
            if (threadIdx.x == 0) {
                ++my_failed;
                if (nv.left[it.p1] < 0 && nv.left[it.p2] < 0 && nv.left[it.p3] < 0)
                    base_list[atomicAdd(&ctr->n_base, 1ull)] = it;
                else
                    emit_children(nv, it, it.slot, child_buf, child_flag);
            }
            continue;
        }
        for (int64_t e = grp; e < total; e += kGroups) {
            int qq = 0;
            int64_t off = e;
            while (off >= szo[qq]) off -= szo[qq++];
            const int q = qo[qq];
            const int64_t xr = nv.begin[r.node[q]] + off;
            const double t = (double)r.t[q];
            double mean, half;
            if (e < kMcCache) {
                mean = c_mean[e];
                half = c_dev[e];
            } else {
                const PartnerMap pm = partner_map(cs, r.slot[q], off, n1, n2, n3);
                const McPoint res =
                    mc_point_group(it, pm, xr, nb, xs, t, ns, r.node[q], k, nullptr, gl, g0);
                mean = res.mean;
                half = k.z * res.sig;
            }
            // Algorithm 5: the estimate gains T_i mu; the running bounds gain
            // T_i (mu -+ z sigma_mu), kept as est -+ dev
            if (gl == 0) {
                atomicAdd(&est[xr], t * mean);
                atomicAdd(&dev[xr], t * half);
            }
        }
        if (threadIdx.x == 0) {
            ++my_prunes;
            if (k.want_cov)
                for (int q = 0; q < r.n_roles; ++q)
                    atomicAdd(&node_cov[r.node[q]], (unsigned long long)r.t[q]);
        }
    }
    if (gl == 0 && drawn) atomicAdd(&ctr->mc_samples, drawn);
    if (threadIdx.x == 0) {
        if (my_failed) atomicAdd(&ctr->mc_failed, my_failed);
        if (my_prunes) atomicAdd(&ctr->mc_prunes, my_prunes);
    }
}

// 3. Exhaustive base cases (MTPotentialBase) through the tile code of the
// exhaustive sum.  A leaf triple (P1, P2, P3) holds the particle triples
// i in P1, j in P2, k in P3 with depth-first ranks i < j < k, so it is a
// work unit of that code with an I block of P1's points, a J block of P2's
// and a K tile of P3's; since the tile's K dimension (one k per lane) is
// wider than a leaf, the leaf triples of a round are sorted by (P1, P2) and
// up to 256 / (leaf width) of them with the same (P1, P2) form one unit,
// their P3 leaves side by side in the K tile.  The unit's (i, j) terms go to
// a table that the tile code reads with scalar loads, as in the exhaustive
// sum.
constexpr int kLeafMax = 32;  // points per leaf at most (leaf_size <= 32)

// Tile shapes of the base-case units: an I block of 32 slots (IPW * NW) and a
// J block of 32; KR k per lane: a K tile of 256 for full units and of 128 for
// the short last unit of a run.  Binary32 units form their (i, k) and (j, k)
// powers in binary32 (pair_terms32): with I and J blocks of one leaf those
// pair terms are a sixth of the work, three times that in binary64.
template <typename T, int KR_> struct LeafShape;
template <int KR_> struct LeafShape<float, KR_> {
    static constexpr int IPW = 8, NW = 4, KR = KR_, JC = 16;
    static constexpr bool kPair32 = true;
    static constexpr bool kLdsBB = false;  // two workgroups per CU fit the LDS without it
};
template <int KR_> struct LeafShape<double, KR_> {
    static constexpr int IPW = 4, NW = 8, KR = KR_, JC = 16;
    static constexpr bool kPair32 = false;
    static constexpr bool kLdsBB = true;
};
template <typename T, int KR>
using LeafLds = DirectLds<T, kLeafMax, LeafShape<T, KR>>;
static_assert(LeafLds<float, 4>::IB == kLeafMax && LeafLds<double, 4>::IB == kLeafMax,
              "I block = leaf");
constexpr int kLeafKT = LeafLds<float, 4>::KT;  // K tile of a full unit
static_assert(LeafLds<double, 4>::KT == kLeafKT && LeafLds<float, 2>::KT == kLeafKT / 2,
              "K tiles of full and short units");
constexpr int kLeafTab = kLeafMax * kLeafMax * kPairVals;  // (i, j) table numbers per unit
constexpr int kUnitBatch = 131072;  // units whose tables are held at most (1 GiB in binary32)
constexpr int kUnitStart = 8192;    // table capacity a traversal starts with

// Ranks of a unit's slots, filled into LDS before the tile code runs.
struct LeafIndex {
    const int *r;  // LDS, one entry per slot of the unit
    __device__ __forceinline__ int rank(int p) const { return r[p]; }
    __device__ __forceinline__ int ri(int il) const { return r[il]; }
    __device__ __forceinline__ int rj(int jl) const { return r[kLeafMax + jl]; }
    __device__ __forceinline__ int rk(int kl) const { return r[2 * kLeafMax + kl]; }
};

// Sort keys of the round's leaf triples: (P1, P2) as p1 * M + p2, P3 as the
// value; slots past the round's count get the largest key.  Also the base
// case statistics (and, for the coverage check, the tuples per node).
__global__ void leaf_keys_kernel(const Item *__restrict__ base_list, int cap, NodeView nv, int M,
                                 MtConst k, MtCounters *__restrict__ ctr,
                                 unsigned long long *__restrict__ node_cov,
                                 unsigned long long *__restrict__ keys, int *__restrict__ vals) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int n_base = (int)ctr->n_base;
    unsigned long long tri = 0;
    if (e < cap && e >= n_base) {
        keys[e] = ~0ull;
        vals[e] = -1;
    } else if (e < cap) {
        const Item it = base_list[e];
        keys[e] = (unsigned long long)it.p1 * (unsigned long long)M + (unsigned long long)it.p2;
        vals[e] = it.p3;
        const int64_t n1 = nv.end[it.p1] - nv.begin[it.p1],
                      n2 = nv.end[it.p2] - nv.begin[it.p2],
                      n3 = nv.end[it.p3] - nv.begin[it.p3];
        const char cs = canonical_case(it.p1, it.p2, it.p3);
        if (cs == 'a') tri = (unsigned long long)(n1 * (n1 - 1) * (n1 - 2) / 6);
        else if (cs == 'b') tri = (unsigned long long)(comb2(n1) * n3);
        else if (cs == 'c') tri = (unsigned long long)(n1 * comb2(n2));
        else tri = (unsigned long long)(n1 * n2 * n3);
        if (k.want_cov) {
            const Roles r = roles_of(it.p1, it.p2, it.p3, n1, n2, n3);
            for (int q = 0; q < r.n_roles; ++q)
                atomicAdd(&node_cov[r.node[q]], (unsigned long long)r.t[q]);
        }
    }
    // the base-case statistics, one atomic per wave each (every lane here)
    const bool real = e < cap && e < n_base;
    wave_add(&ctr->base_cases, real ? 1ull : 0ull);
    wave_add(&ctr->base_triples, tri);
}

// Units from the sorted keys: each run of equal (P1, P2) is cut into full
// units of per_unit leaf triples; a remainder of more than per_unit / 2
// makes one more full unit, a smaller one a short unit (half the K tile).
// The first thread of the run writes them.
__global__ void leaf_units_kernel(const unsigned long long *__restrict__ keys, int cap,
                                  MtCounters *__restrict__ ctr, int per_unit,
                                  int *__restrict__ u_start, int *__restrict__ u_count,
                                  int *__restrict__ h_start, int *__restrict__ h_count) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int n_base = (int)ctr->n_base;
    if (e >= n_base || e >= cap) return;
    const unsigned long long key = keys[e];
    if (e > 0 && keys[e - 1] == key) return;
    int len = 1;
    while (e + len < n_base && keys[e + len] == key) ++len;
    int full = len / per_unit;
    const int rest = len - full * per_unit;
    const bool short_rest = rest > 0 && 2 * rest <= per_unit;
    if (rest > 0 && !short_rest) ++full;
    if (full > 0) {
        const int base = (int)atomicAdd(&ctr->n_units, (unsigned long long)full);
        for (int q = 0; q < full; ++q) {
            u_start[base + q] = e + q * per_unit;
            u_count[base + q] = min(per_unit, len - q * per_unit);
        }
    }
    if (short_rest) {
        const int h = (int)atomicAdd(&ctr->n_short, 1ull);
        h_start[h] = e + len - rest;
        h_count[h] = rest;
    }
}

// (i, j) tables of the units [u0, u0 + batch) that exist: [jl][il][a, w]
// for i in P1, j in P2, masked unless both exist and rank i < rank j (P1 = P2
// in cases (a) and (b)); coordinates times `scale`.
template <typename T>
__global__ __launch_bounds__(256) void leaf_table_kernel(
    const unsigned long long *__restrict__ keys, const int *__restrict__ u_start,
    const unsigned long long *__restrict__ count, int u0, int batch, int M, NodeView nv,
    const double *__restrict__ xs, double scale, T *__restrict__ tab) {
    __shared__ double xa[3][kLeafMax], xb[3][kLeafMax];
    const int tid = threadIdx.x;
    const int n_units = min((int)*count - u0, batch);
    for (int w = blockIdx.x; w < n_units; w += gridDim.x) {
        const unsigned long long key = keys[u_start[u0 + w]];
        const int p1 = (int)(key / (unsigned long long)M), p2 = (int)(key % (unsigned long long)M);
        const int b1 = nv.begin[p1], b2 = nv.begin[p2];
        const int n1 = nv.end[p1] - b1, n2 = nv.end[p2] - b2;
        __syncthreads();  // the previous unit is done with xa, xb
        if (tid < kLeafMax) {
            for (int c = 0; c < 3; ++c)
                xa[c][tid] = tid < n1 ? xs[3 * (int64_t)(b1 + tid) + c] * scale : 0.0;
        } else if (tid < 2 * kLeafMax) {
            const int o = tid - kLeafMax;
            for (int c = 0; c < 3; ++c)
                xb[c][o] = o < n2 ? xs[3 * (int64_t)(b2 + o) + c] * scale : 0.0;
        }
        __syncthreads();
        T *out = tab + (int64_t)w * kLeafTab;
        for (int e = tid; e < kLeafMax * kLeafMax; e += 256) {
            const int jl = e / kLeafMax, il = e % kLeafMax;
            table_entry(xb[0][jl] - xa[0][il], xb[1][jl] - xa[1][il], xb[2][jl] - xa[2][il],
                        il < n1 && jl < n2 && b1 + il < b2 + jl, out + kPairVals * e);
        }
    }
}

// The units [u0, u0 + batch) that exist (of *count) through the tile code;
// the K tile holds the P3 leaves of a unit's items, `width` slots each (the
// largest leaf).  The tables were written by the previous launch and are
// only read.
template <typename T, int KR>
__global__ __launch_bounds__((LeafLds<T, KR>::TPB)) void leaf_tile_kernel(
    const unsigned long long *__restrict__ keys, const int *__restrict__ vals,
    const int *__restrict__ u_start, const int *__restrict__ u_count,
    const unsigned long long *__restrict__ count, int u0, int batch, int M, NodeView nv,
    const double *__restrict__ xs, const T *__restrict__ tab, int width, double scale,
    double out_scale, double *__restrict__ est) {
    using Lds = LeafLds<T, KR>;
    __shared__ Lds s;
    __shared__ int rk[Lds::XS];
    using CT = __attribute__((address_space(4))) const T;
    constexpr int TPB = Lds::TPB;
    const int n_units = min((int)*count - u0, batch);
    for (int w = blockIdx.x; w < n_units; w += gridDim.x) {
        const int u = u0 + w;
        const int e0 = u_start[u], cnt = u_count[u];
        const unsigned long long key = keys[e0];
        const int p1 = (int)(key / (unsigned long long)M), p2 = (int)(key % (unsigned long long)M);
        const int b1 = nv.begin[p1], b2 = nv.begin[p2];
        const int n1 = nv.end[p1] - b1, n2 = nv.end[p2] - b2;
        __syncthreads();  // the previous unit is done with rk and the LDS
        for (int p = threadIdx.x; p < Lds::XS; p += TPB) {
            int r = -1;
            if (p < kLeafMax) {
                if (p < n1) r = b1 + p;
            } else if (p < 2 * kLeafMax) {
                if (p - kLeafMax < n2) r = b2 + p - kLeafMax;
            } else {
                const int q = (p - 2 * kLeafMax) / width, o = (p - 2 * kLeafMax) % width;
                if (q < cnt) {
                    const int v = vals[e0 + q];
                    if (o < nv.end[v] - nv.begin[v]) r = nv.begin[v] + o;
                }
            }
            rk[p] = r;
        }
        __syncthreads();
        const LeafIndex ix{rk};
        tile_unit<T, kLeafMax, LeafShape<T, KR>>(s, xs, ix, (CT *)tab + (int64_t)w * kLeafTab,
                                                 scale, out_scale, est);
    }
}

// Far-field estimates of the round's far items: one workgroup per item; each
// point x of each node gets the expansion of order k.order due to the other
// two nodes (farfield.hpp), kept inside [T phi_lo, T phi_hi], in fest[x].
__global__ __launch_bounds__(256) void far_kernel(const FarItem *__restrict__ far_list,
                                                  NodeView nv, const double *__restrict__ xs,
                                                  const double *__restrict__ smom, MtConst k,
                                                  const MtCounters *__restrict__ ctr,
                                                  double *__restrict__ fest) {
    const int n_far = (int)ctr->n_far;
    for (int w = blockIdx.x; w < n_far; w += gridDim.x) {
        const FarItem it = far_list[w];
        const int pn[3] = {it.p1, it.p2, it.p3};
        const int b0 = nv.begin[pn[0]], b1 = nv.begin[pn[1]], b2 = nv.begin[pn[2]];
        const int c0 = nv.end[pn[0]] - b0, c1 = nv.end[pn[1]] - b1, c2 = nv.end[pn[2]] - b2;
        const int total = c0 + c1 + c2;
        for (int e = threadIdx.x; e < total; e += blockDim.x) {
            const int q = e < c0 ? 0 : (e < c0 + c1 ? 1 : 2);
            const int r = q == 0 ? b0 + e : (q == 1 ? b1 + e - c0 : b2 + e - c0 - c1);
            const int va = pn[q == 0 ? 1 : 0], vb = pn[q == 2 ? 1 : 2];
            const double na = (double)(nv.end[va] - nv.begin[va]);
            const double nb = (double)(nv.end[vb] - nv.begin[vb]);
            const double x[3] = {xs[3 * (int64_t)r], xs[3 * (int64_t)r + 1], xs[3 * (int64_t)r + 2]};
            double f = farfield_value(x, nv.centroid + 3 * va, nv.centroid + 3 * vb, na, nb,
                                      smom + 6 * va, smom + 6 * vb, k.order);
            const double t = na * nb;
            f = isfinite(f) ? fmin(fmax(f, t * it.lo), t * it.hi) : 0.5 * t * (it.lo + it.hi);
            atomicAdd(&fest[r], f);
        }
    }
}

// Second-moment matrices sum (y - c)(y - c)^T of every node about its
// centroid: leaves from their points, then parents by the parallel-axis
// rule, depth by depth in one workgroup.
__global__ void leaf_moments_kernel(const int32_t *__restrict__ leaves, int n_leaves,
                                    const int32_t *__restrict__ begin,
                                    const int32_t *__restrict__ end,
                                    const double *__restrict__ xs,
                                    const double *__restrict__ centroid,
                                    double *__restrict__ smom) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_leaves) return;
    const int v = leaves[e];
    const double *c = centroid + 3 * v;
    double m[6] = {0, 0, 0, 0, 0, 0};
    for (int r = begin[v]; r < end[v]; ++r) {
        const double d0 = xs[3 * (int64_t)r] - c[0], d1 = xs[3 * (int64_t)r + 1] - c[1],
                     d2 = xs[3 * (int64_t)r + 2] - c[2];
        m[0] += d0 * d0;
        m[1] += d0 * d1;
        m[2] += d0 * d2;
        m[3] += d1 * d1;
        m[4] += d1 * d2;
        m[5] += d2 * d2;
    }
    for (int i = 0; i < 6; ++i) smom[6 * v + i] = m[i];
}

__global__ __launch_bounds__(1024) void up_moments_kernel(const int32_t *__restrict__ depth_nodes,
                                                          const int *__restrict__ depth_off,
                                                          int n_depths,
                                                          const int32_t *__restrict__ left,
                                                          const int32_t *__restrict__ right,
                                                          const int32_t *__restrict__ begin,
                                                          const int32_t *__restrict__ end,
                                                          const double *__restrict__ centroid,
                                                          double *__restrict__ smom) {
    for (int d = n_depths - 1; d >= 0; --d) {
        for (int e = depth_off[d] + threadIdx.x; e < depth_off[d + 1]; e += blockDim.x) {
            const int v = depth_nodes[e];
            if (left[v] < 0) continue;
            double m[6] = {0, 0, 0, 0, 0, 0};
            for (const int ch : {left[v], right[v]}) {
                const double w = (double)(end[ch] - begin[ch]);
                const double d0 = centroid[3 * ch] - centroid[3 * v];
                const double d1 = centroid[3 * ch + 1] - centroid[3 * v + 1];
                const double d2 = centroid[3 * ch + 2] - centroid[3 * v + 2];
                const double *s = smom + 6 * ch;
                m[0] += s[0] + w * d0 * d0;
                m[1] += s[1] + w * d0 * d1;
                m[2] += s[2] + w * d0 * d2;
                m[3] += s[3] + w * d1 * d1;
                m[4] += s[4] + w * d1 * d2;
                m[5] += s[5] + w * d2 * d2;
            }
            for (int i = 0; i < 6; ++i) smom[6 * v + i] = m[i];
        }
        __syncthreads();
    }
}

__global__ void reset_round_kernel(MtCounters *ctr) {
    ctr->n_base = 0;
    ctr->n_mc = 0;
    ctr->n_units = 0;
    ctr->n_short = 0;
    ctr->n_far = 0;
}

__global__ void zero_u64_kernel(unsigned long long *__restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__global__ void zero_counters_kernel(MtCounters *ctr) {
    ctr->n_base = ctr->n_mc = ctr->n_units = ctr->n_short = ctr->n_far = 0;
    ctr->det_prunes = ctr->mc_prunes = 0;
    ctr->mc_failed = ctr->base_cases = ctr->base_triples = ctr->mc_samples = 0;
}

// 5. Node statistics.  Per point, LB(x) = est[x] - dev[x] + (node
// lower-bound increments of x's leaf and its ancestors) and UB(x) = est[x] +
// dev[x] + (node upper-bound increments): exact base-case values and Monte
// Carlo means are in est, the Monte Carlo half-widths T_i z sigma_mu in dev,
// the deterministic prunes' T_i phi_lo and T_i phi_hi on the nodes.  Top-down
// path sums and bottom-up minima run in one workgroup, depth by depth.
__global__ __launch_bounds__(1024) void refresh_down_kernel(const int32_t *__restrict__ depth_nodes,
                                                            const int *__restrict__ depth_off,
                                                            int n_depths,
                                                            const int32_t *__restrict__ parent,
                                                            const double *__restrict__ node_lo,
                                                            const double *__restrict__ node_hi,
                                                            double *__restrict__ cum_lo,
                                                            double *__restrict__ cum_hi) {
    for (int d = 0; d < n_depths; ++d) {
        for (int e = depth_off[d] + threadIdx.x; e < depth_off[d + 1]; e += blockDim.x) {
            const int v = depth_nodes[e];
            const int u = parent[v];
            cum_lo[v] = node_lo[v] + (u >= 0 ? cum_lo[u] : 0.0);
            cum_hi[v] = node_hi[v] + (u >= 0 ? cum_hi[u] : 0.0);
        }
        __syncthreads();
    }
}

// Leaf statistics: minima over the leaf's points of LB, -UB and max(LB, -UB).
__global__ void refresh_leaf_kernel(const int32_t *__restrict__ leaves, int n_leaves,
                                    const int32_t *__restrict__ begin,
                                    const int32_t *__restrict__ end, const double *__restrict__ est,
                                    const double *__restrict__ dev,
                                    const double *__restrict__ cum_lo,
                                    const double *__restrict__ cum_hi, double *__restrict__ pos,
                                    double *__restrict__ neg, double *__restrict__ mix) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_leaves) return;
    const int v = leaves[e];
    double mp = INFINITY, mn = INFINITY, mm = INFINITY;
    for (int r = begin[v]; r < end[v]; ++r) {
        const double l = est[r] - dev[r] + cum_lo[v];
        const double u = est[r] + dev[r] + cum_hi[v];
        mp = fmin(mp, l);
        mn = fmin(mn, -u);
        mm = fmin(mm, fmax(l, -u));
    }
    pos[v] = mp;
    neg[v] = mn;
    mix[v] = mm;
}

__global__ __launch_bounds__(1024) void refresh_up_kernel(const int32_t *__restrict__ depth_nodes,
                                                          const int *__restrict__ depth_off,
                                                          int n_depths,
                                                          const int32_t *__restrict__ left,
                                                          const int32_t *__restrict__ right,
                                                          double *__restrict__ pos,
                                                          double *__restrict__ neg,
                                                          double *__restrict__ mix) {
    for (int d = n_depths - 1; d >= 0; --d) {
        for (int e = depth_off[d] + threadIdx.x; e < depth_off[d + 1]; e += blockDim.x) {
            const int v = depth_nodes[e];
            const int a = left[v], b = right[v];
            if (a >= 0) {
                pos[v] = fmin(pos[a], pos[b]);
                neg[v] = fmin(neg[a], neg[b]);
                mix[v] = fmin(mix[a], mix[b]);
            }
        }
        __syncthreads();
    }
}

// 6. Top-down (Section 3): node accumulators to points, back to input order.
__global__ void topdown_kernel(int n, const int32_t *__restrict__ leaf_of,
                               const int32_t *__restrict__ parent, const int32_t *__restrict__ perm,
                               const double *__restrict__ est, const double *__restrict__ fest,
                               const double *__restrict__ node_acc,
                               const unsigned long long *__restrict__ node_cov,
                               double *__restrict__ phi, int64_t *__restrict__ coverage) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double acc = est[r] + fest[r];
    unsigned long long cv = 0;
    for (int v = leaf_of[r]; v >= 0; v = parent[v]) {
        acc += node_acc[v];
        if (coverage) cv += node_cov[v];
    }
    phi[perm[r]] = acc;
    if (coverage) coverage[perm[r]] = (int64_t)cv;
}

// Whether the tree's depth-first copy of the points is the caller's x in the
// tree's order, bit for bit: flag[0] is set at any difference.
__global__ void same_points_kernel(const double *__restrict__ x, const int32_t *__restrict__ perm,
                                   const double *__restrict__ xs, int n, int *__restrict__ flag) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t i = perm[r];
    bool diff = false;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        diff |= __double_as_longlong(x[3 * i + c]) != __double_as_longlong(xs[3 * (int64_t)r + c]);
    if (diff) atomicOr(flag, 1);
}

template <typename T>
mb_status dalloc(Scratch &sc, T **p, size_t count, hipStream_t s) {
    mb_status st = sc.alloc(sizeof(T) * (count ? count : 1), s);
    *p = sc.as<T>();
    return st;
}

}  // namespace

mb_status tree_matches_points(const DeviceTree *t, const double *x, int64_t n, hipStream_t s,
                              bool *same) {
    *same = false;
    if (t->h.n != n) return MB_OK;
    if (n == 0) {
        *same = true;
        return MB_OK;
    }
    Scratch sc;
    int *flag;
    mb_status st = dalloc(sc, &flag, 1, s);
    if (st != MB_OK) return st;
    MB_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    same_points_kernel<<<(int)((n + 255) / 256), 256, 0, s>>>(x, t->perm, t->xs, (int)n, flag);
    MB_HIP(hipGetLastError());
    int h = 1;
    MB_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    MB_HIP(hipStreamSynchronize(s));
    *same = h == 0;
    return MB_OK;
}

double normal_quantile_upper(double alpha_half) {
    // z with P(Z > z) = alpha_half, by Newton's method on erfc
    if (!(alpha_half > 0.0 && alpha_half < 0.5)) return 0.0;
    double z = 1.0;
    for (int it = 0; it < 100; ++it) {
        const double f = 0.5 * std::erfc(z / std::sqrt(2.0)) - alpha_half;
        const double df = -std::exp(-0.5 * z * z) / std::sqrt(2.0 * M_PI);
        const double step = f / df;
        z -= step;
        if (std::fabs(step) < 1e-16 * std::fabs(z)) break;
    }
    return z;
}

mb_status multitree_run(const DeviceTree *t, const MtParams &prm, double *phi, int64_t *coverage,
                        MtStats *stats, hipStream_t s) {
    const int n = (int)t->h.n;
    const int M = t->h.n_nodes;
    mb_status st;
    auto t0 = std::chrono::steady_clock::now();
    if (n < 3) {
        if ((st = zero_doubles(phi, n, s)) != MB_OK) return st;
        if (coverage && n > 0) MB_HIP(hipMemsetAsync(coverage, 0, sizeof(int64_t) * n, s));
        MB_HIP(hipStreamSynchronize(s));
        return MB_OK;
    }
    // host lists: leaves, depth offsets
    std::vector<int32_t> leaves;
    for (int v = 0; v < M; ++v)
        if (t->h.left[v] < 0) leaves.push_back(v);
    const int n_depths = t->h.max_depth + 1;

    // per point: est (exact values and Monte Carlo means), dev (Monte Carlo
    // half-widths); per node: accumulators, bound increments, statistics and
    // path sums of the increments
    Scratch s_pt, s_nd, s_cov, s_ctr, s_leaves, s_doff;
    double *pt, *nd;
    unsigned long long *node_cov;
    MtCounters *ctr;
    int32_t *d_leaves;
    int *d_doff;
    if ((st = dalloc(s_pt, &pt, 3 * (size_t)n, s)) || (st = dalloc(s_nd, &nd, 14 * (size_t)M, s)) ||
        (st = dalloc(s_cov, &node_cov, M, s)) || (st = dalloc(s_ctr, &ctr, 1, s)) ||
        (st = dalloc(s_leaves, &d_leaves, leaves.size(), s)) ||
        (st = dalloc(s_doff, &d_doff, t->depth_off.size(), s)))
        return st;
    double *est = pt, *dev = pt + n, *fest = pt + 2 * (size_t)n;  // fest: far-field estimates
    double *node_acc = nd, *node_lo = nd + M, *node_hi = nd + 2 * (size_t)M;
    double *st_pos = nd + 3 * (size_t)M, *st_neg = nd + 4 * (size_t)M, *st_mix = nd + 5 * (size_t)M;
    double *cum_lo = nd + 6 * (size_t)M, *cum_hi = nd + 7 * (size_t)M;
    double *smom = nd + 8 * (size_t)M;  // second moments, 6 per node
    const NodeStats ns{st_pos, st_neg, st_mix};
    MB_HIP(hipMemcpyAsync(d_leaves, leaves.data(), sizeof(int32_t) * leaves.size(),
                          hipMemcpyHostToDevice, s));
    MB_HIP(hipMemcpyAsync(d_doff, t->depth_off.data(), sizeof(int) * t->depth_off.size(),
                          hipMemcpyHostToDevice, s));
    if ((st = zero_doubles(pt, 3 * (int64_t)n, s)) != MB_OK) return st;
    if ((st = zero_doubles(nd, 14 * (int64_t)M, s)) != MB_OK) return st;
    if (prm.order >= 2) {
        leaf_moments_kernel<<<((int)leaves.size() + 255) / 256, 256, 0, s>>>(
            d_leaves, (int)leaves.size(), t->begin, t->end, t->xs, t->centroid, smom);
        up_moments_kernel<<<1, 1024, 0, s>>>(t->depth_nodes, d_doff, n_depths, t->left, t->right,
                                             t->begin, t->end, t->centroid, smom);
        MB_HIP(hipGetLastError());
    }
    zero_u64_kernel<<<(M + 255) / 256, 256, 0, s>>>(node_cov, M);
    zero_counters_kernel<<<1, 1, 0, s>>>(ctr);

    const int chunk = std::max(1, prm.chunk);
    // two LIFO stacks: the near stack is drained first; triples whose three
    // boxes are pairwise apart are deferred to the far stack meanwhile
    int64_t cap = std::max<int64_t>(16 * (int64_t)chunk, 1 << 16);
    int64_t fcap = cap;
    Scratch s_stack, s_far, s_mc, s_base, s_child, s_flag, s_dbuf, s_dflag, s_num, s_tmp, s_flist;
    Item *stack, *far, *mc_list, *base_list, *child_buf, *defer_buf;
    FarItem *far_list;
    uint8_t *child_flag, *defer_flag;
    int *d_num;
    if ((st = dalloc(s_stack, &stack, cap, s)) || (st = dalloc(s_far, &far, fcap, s)) ||
        (st = dalloc(s_mc, &mc_list, chunk, s)) || (st = dalloc(s_base, &base_list, chunk, s)) ||
        (st = dalloc(s_child, &child_buf, 8 * (size_t)chunk, s)) ||
        (st = dalloc(s_flag, &child_flag, 8 * (size_t)chunk, s)) ||
        (st = dalloc(s_dbuf, &defer_buf, chunk, s)) || (st = dalloc(s_dflag, &defer_flag, chunk, s)) ||
        (st = dalloc(s_num, &d_num, 2, s)) ||
        (st = dalloc(s_flist, &far_list, prm.order >= 1 ? chunk : 1, s)))
        return st;
    size_t tmp_bytes = 0;
    MB_HIP(hipcub::DeviceSelect::Flagged(nullptr, tmp_bytes, child_buf, child_flag, stack, d_num,
                                         8 * chunk, s));
    if ((st = s_tmp.alloc(tmp_bytes, s)) != MB_OK) return st;

    // base cases: sort keys and values of the round's leaf triples (two
    // copies each), units, and the (i, j) tables of up to `ubatch` units
    const bool base64 = prm.base_prec == MB_FP64;
    int width = 1;  // K-tile slots per leaf: the largest leaf
    for (int32_t v : leaves) width = std::max(width, t->h.end[v] - t->h.begin[v]);
    const int per_unit = kLeafKT / width;
    // table capacity in units: starts small and grows to the largest round
    // seen (up to kUnitBatch); units beyond it run in further batches
    int ubatch = std::min(chunk, kUnitStart);
    Scratch s_keys, s_vals, s_ust, s_ucnt, s_hst, s_hcnt, s_tab, s_htab, s_stmp;
    unsigned long long *keys;
    int *vals, *u_start, *u_count, *h_start, *h_count;
    char *tab, *htab;
    const size_t unit_tab_bytes = (size_t)kLeafTab * (base64 ? 8 : 4);
    const size_t tab_bytes = (size_t)ubatch * unit_tab_bytes;
    if ((st = dalloc(s_keys, &keys, 2 * (size_t)chunk, s)) ||
        (st = dalloc(s_vals, &vals, 2 * (size_t)chunk, s)) ||
        (st = dalloc(s_ust, &u_start, chunk, s)) || (st = dalloc(s_ucnt, &u_count, chunk, s)) ||
        (st = dalloc(s_hst, &h_start, chunk, s)) || (st = dalloc(s_hcnt, &h_count, chunk, s)) ||
        (st = dalloc(s_tab, &tab, tab_bytes, s)) || (st = dalloc(s_htab, &htab, tab_bytes, s)))
        return st;
    const unsigned long long key_max = (unsigned long long)M * (unsigned long long)M - 1ull;
    const int end_bit = std::max(1, 64 - __builtin_clzll(std::max(key_max, 1ull)));
    size_t stmp_bytes = 0;
    MB_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, stmp_bytes, keys, keys + chunk, vals,
                                              vals + chunk, chunk, 0, end_bit, s));
    if ((st = s_stmp.alloc(stmp_bytes, s)) != MB_OK) return st;
    // binary32 tiles work on coordinates scaled by a power of two that puts
    // the closest pair in [1, 2) (exact), as in the exhaustive sum
    const double lscale = base64 || !(prm.r_min > 0.0) ? 1.0 : unit_scale(prm.r_min * prm.r_min);
    const double lout = std::pow(lscale, 9.0);
    const NodeView nv{t->begin, t->end, t->left, t->right, t->lo, t->hi, t->centroid};
    // one batch of full units and one of short units, from unit u0 of each
    auto leaf_batch = [&](int u0) -> mb_status {
        const unsigned grid = (unsigned)std::min(ubatch, 2048);
        const unsigned long long *nf = &ctr->n_units, *nh = &ctr->n_short;
        if (base64) {
            leaf_table_kernel<double><<<grid, 256, 0, s>>>(keys + chunk, u_start, nf, u0, ubatch,
                                                          M, nv, t->xs, lscale, (double *)tab);
            leaf_tile_kernel<double, 4><<<grid, LeafLds<double, 4>::TPB, 0, s>>>(
                keys + chunk, vals + chunk, u_start, u_count, nf, u0, ubatch, M, nv, t->xs,
                (const double *)tab, width, lscale, lout, est);
            leaf_table_kernel<double><<<grid, 256, 0, s>>>(keys + chunk, h_start, nh, u0, ubatch,
                                                          M, nv, t->xs, lscale, (double *)htab);
            leaf_tile_kernel<double, 2><<<grid, LeafLds<double, 2>::TPB, 0, s>>>(
                keys + chunk, vals + chunk, h_start, h_count, nh, u0, ubatch, M, nv, t->xs,
                (const double *)htab, width, lscale, lout, est);
        } else {
            leaf_table_kernel<float><<<grid, 256, 0, s>>>(keys + chunk, u_start, nf, u0, ubatch,
                                                         M, nv, t->xs, lscale, (float *)tab);
            leaf_tile_kernel<float, 4><<<grid, LeafLds<float, 4>::TPB, 0, s>>>(
                keys + chunk, vals + chunk, u_start, u_count, nf, u0, ubatch, M, nv, t->xs,
                (const float *)tab, width, lscale, lout, est);
            leaf_table_kernel<float><<<grid, 256, 0, s>>>(keys + chunk, h_start, nh, u0, ubatch,
                                                         M, nv, t->xs, lscale, (float *)htab);
            leaf_tile_kernel<float, 2><<<grid, LeafLds<float, 2>::TPB, 0, s>>>(
                keys + chunk, vals + chunk, h_start, h_count, nh, u0, ubatch, M, nv, t->xs,
                (const float *)htab, width, lscale, lout, est);
        }
        MB_HIP(hipGetLastError());
        return MB_OK;
    };

    const Item root{0, 0, 0, 0};
    MB_HIP(hipMemcpyAsync(stack, &root, sizeof(Item), hipMemcpyHostToDevice, s));
    int64_t top = 1, far_top = 0;
    // bands of spread: 0 (all boxes touching), then unit * 2^(phase - 1)
    int phase = 0;
    auto spread_limit = [&](int ph) {
        return ph == 0 ? 0.0 : prm.spread_unit * std::ldexp(1.0, ph - 1);
    };

    MtConst k;
    k.n = n;
    k.eps = prm.eps;
    k.tau = prm.tau;
    k.z = prm.alpha > 0.0 ? normal_quantile_upper(prm.alpha / 2.0) : 0.0;
    k.t_root = (double)(n - 1) * (double)(n - 2) / 2.0;
    k.r_min = prm.r_min;
    k.m_limit = prm.m_limit;
    k.m_min = prm.m_min;
    k.zeta = prm.zeta;
    k.seed32 = (uint32_t)(prm.seed ^ (prm.seed >> 32));
    k.use_mc = prm.alpha > 0.0 ? 1 : 0;
    k.want_cov = coverage ? 1 : 0;
    k.two_sided = prm.bound == MB_BOUND_TWO_SIDED ? 1 : 0;
    k.order = prm.order;

    auto grow = [&](Scratch &sc, Item *&buf, int64_t &c, int64_t keep, int64_t need) -> mb_status {
        if (need <= c) return MB_OK;
        const int64_t nc = std::max<int64_t>(2 * c, need);
        Scratch s2;
        Item *b2;
        mb_status e = dalloc(s2, &b2, nc, s);
        if (e != MB_OK) return e;
        if (keep > 0) {
            hipError_t he = hipMemcpyAsync(b2, buf, sizeof(Item) * keep, hipMemcpyDeviceToDevice, s);
            if (he != hipSuccess) return hip_fail(he, "stack copy");
        }
        std::swap(sc.ptr, s2.ptr);
        buf = b2;
        c = nc;
        return MB_OK;
    };

    int64_t max_stack = 1, rounds = 0, visited = 0;
    // device time of the phases of each round: classification (with the
    // far-field estimates), Monte Carlo, base cases (sort, units, tiles)
    struct Events {
        hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
        ~Events() {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } evs;
    hipEvent_t *ev = evs.e;
    for (int q = 0; q < 4; ++q) MB_HIP(hipEventCreate(&ev[q]));
    double phase_ms[3] = {0.0, 0.0, 0.0};
    const bool trace = std::getenv("MB_TRACE") != nullptr;
    auto last_print = std::chrono::steady_clock::now();
    for (;;) {
        if (top == 0) {
            if (far_top == 0) break;
            // this band is done: the deferred triples become the stack
            if (trace) {
                MtCounters hc;
                MB_HIP(hipMemcpy(&hc, ctr, sizeof hc, hipMemcpyDeviceToHost));
                std::vector<double> pl(M);
                MB_HIP(hipMemcpy(pl.data(), st_pos, sizeof(double) * M, hipMemcpyDeviceToHost));
                std::vector<double> lv;
                for (int32_t v : leaves) lv.push_back(pl[v]);
                std::sort(lv.begin(), lv.end());
                std::fprintf(stderr,
                             "[mb multitree] end of band %d (spread <= %g): round %lld visited %lld "
                             "det %llu mc %llu/%llu base %llu base triples %llu; leaf Phi^l min %g "
                             "median %g max %g; deferred %lld\n",
                             phase, phase == 0 ? 0.0 : spread_limit(phase), (long long)rounds,
                             (long long)visited, hc.det_prunes, hc.mc_prunes, hc.mc_failed, hc.base_cases,
                             hc.base_triples, lv.front(), lv[lv.size() / 2], lv.back(),
                             (long long)far_top);
            }
            ++phase;
            std::swap(s_stack.ptr, s_far.ptr);
            std::swap(stack, far);
            std::swap(cap, fcap);
            top = far_top;
            far_top = 0;
            continue;
        }
        const double limit = (prm.spread_unit > 0.0 && phase < 64) ? spread_limit(phase) : INFINITY;
        const int B = (int)std::min<int64_t>(top, chunk);
        Item *items = stack + (top - B);
        MB_HIP(hipEventRecord(ev[0], s));
        reset_round_kernel<<<1, 1, 0, s>>>(ctr);
        classify_kernel<<<(B + 255) / 256, 256, 0, s>>>(items, B, nv, ns, node_acc, node_lo,
                                                       node_hi, node_cov, k, ctr, mc_list,
                                                       base_list, child_buf, child_flag, limit,
                                                       defer_buf, defer_flag, far_list);
        if (k.order >= 1)
            far_kernel<<<std::min(B, 2048), 256, 0, s>>>(far_list, nv, t->xs, smom, k, ctr, fest);
        MB_HIP(hipEventRecord(ev[1], s));
        if (k.use_mc)
            mc_kernel<<<std::min(B, 4096), kMcThreads, 0, s>>>(mc_list, nv, t->xs, ns, est, dev,
                                                               node_cov, k, ctr, base_list,
                                                               child_buf, child_flag);
        MB_HIP(hipEventRecord(ev[2], s));
        // base cases: sort by (P1, P2), cut into units, tables, tiles
        leaf_keys_kernel<<<(B + 255) / 256, 256, 0, s>>>(base_list, B, nv, M, k, ctr, node_cov,
                                                        keys, vals);
        MB_HIP(hipcub::DeviceRadixSort::SortPairs(s_stmp.ptr, stmp_bytes, keys, keys + chunk, vals,
                                                  vals + chunk, B, 0, end_bit, s));
        leaf_units_kernel<<<(B + 255) / 256, 256, 0, s>>>(keys + chunk, B, ctr, per_unit, u_start,
                                                         u_count, h_start, h_count);
        if ((st = leaf_batch(0)) != MB_OK) return st;
        MB_HIP(hipGetLastError());
        MB_HIP(hipEventRecord(ev[3], s));
        // children of split triples, in order, onto the stack where the chunk was;
        // deferred far triples, in order, onto the far stack
        if ((st = grow(s_stack, stack, cap, top - B, top - B + 8 * (int64_t)B)) != MB_OK) return st;
        MB_HIP(hipcub::DeviceSelect::Flagged(s_tmp.ptr, tmp_bytes, child_buf, child_flag,
                                             stack + (top - B), d_num, 8 * B, s));
        if (limit < INFINITY) {
            if ((st = grow(s_far, far, fcap, far_top, far_top + B)) != MB_OK) return st;
            MB_HIP(hipcub::DeviceSelect::Flagged(s_tmp.ptr, tmp_bytes, defer_buf, defer_flag,
                                                 far + far_top, d_num + 1, B, s));
        }
        int num[2] = {0, 0};
        MB_HIP(hipMemcpyAsync(num, d_num, sizeof(num), hipMemcpyDeviceToHost, s));
        unsigned long long n_units[2] = {0, 0};  // full and short units (adjacent counters)
        MB_HIP(hipMemcpyAsync(n_units, &ctr->n_units, sizeof n_units, hipMemcpyDeviceToHost, s));
        // Phi^l refresh for the next round
        refresh_down_kernel<<<1, 1024, 0, s>>>(t->depth_nodes, d_doff, n_depths, t->parent,
                                               node_lo, node_hi, cum_lo, cum_hi);
        refresh_leaf_kernel<<<((int)leaves.size() + 255) / 256, 256, 0, s>>>(
            d_leaves, (int)leaves.size(), t->begin, t->end, est, dev, cum_lo, cum_hi, st_pos,
            st_neg, st_mix);
        refresh_up_kernel<<<1, 1024, 0, s>>>(t->depth_nodes, d_doff, n_depths, t->left, t->right,
                                             st_pos, st_neg, st_mix);
        MB_HIP(hipGetLastError());
        MB_HIP(hipStreamSynchronize(s));
        float ms[3];
        for (int q = 0; q < 3; ++q) MB_HIP(hipEventElapsedTime(&ms[q], ev[q], ev[q + 1]));
        phase_ms[0] += ms[0];
        phase_ms[1] += ms[1];
        phase_ms[2] += ms[2];
        // units beyond the first batch (their credits reach the statistics
        // one round later, which only delays prunes)
        const unsigned long long n_units_max = std::max(n_units[0], n_units[1]);
        if (n_units_max > (unsigned long long)ubatch) {
            MB_HIP(hipEventRecord(ev[0], s));
            for (int u0 = ubatch; (unsigned long long)u0 < n_units_max; u0 += ubatch)
                if ((st = leaf_batch(u0)) != MB_OK) return st;
            MB_HIP(hipEventRecord(ev[1], s));
            MB_HIP(hipStreamSynchronize(s));
            MB_HIP(hipEventElapsedTime(&ms[0], ev[0], ev[1]));
            phase_ms[2] += ms[0];
            // larger tables for the next rounds
            if (ubatch < std::min(chunk, kUnitBatch)) {
                int cap = ubatch;
                while ((unsigned long long)cap < n_units_max && cap < kUnitBatch) cap *= 2;
                cap = std::min({cap, chunk, kUnitBatch});
                Scratch n1, n2;
                char *t1, *t2;
                if ((st = dalloc(n1, &t1, (size_t)cap * unit_tab_bytes, s)) ||
                    (st = dalloc(n2, &t2, (size_t)cap * unit_tab_bytes, s)))
                    return st;
                std::swap(s_tab.ptr, n1.ptr);
                std::swap(s_htab.ptr, n2.ptr);
                tab = t1;
                htab = t2;
                ubatch = cap;
            }
        }
        top = top - B + num[0];
        visited += B - (limit < INFINITY ? num[1] : 0);
        if (limit < INFINITY) far_top += num[1];
        max_stack = std::max(max_stack, top + far_top);
        ++rounds;
        if (trace && std::chrono::steady_clock::now() - last_print > std::chrono::seconds(5)) {
            last_print = std::chrono::steady_clock::now();
            MtCounters hc;
            MB_HIP(hipMemcpy(&hc, ctr, sizeof hc, hipMemcpyDeviceToHost));
            std::fprintf(stderr,
                         "[mb multitree] round %lld phase %d stack %lld far %lld visited %lld det %llu "
                         "mc %llu/%llu base %llu\n",
                         (long long)rounds, phase, (long long)top, (long long)far_top, (long long)visited,
                         hc.det_prunes, hc.mc_prunes, hc.mc_failed, hc.base_cases);
        }
    }
    topdown_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, t->leaf_of, t->parent, t->perm, est, fest,
                                                   node_acc, node_cov, phi, coverage);
    MB_HIP(hipGetLastError());
    MtCounters hc;
    MB_HIP(hipMemcpyAsync(&hc, ctr, sizeof hc, hipMemcpyDeviceToHost, s));
    MB_HIP(hipStreamSynchronize(s));
    if (stats) {
        stats->visited = visited;
        stats->det_prunes = (int64_t)hc.det_prunes;
        stats->mc_prunes = (int64_t)hc.mc_prunes;
        stats->mc_failed = (int64_t)hc.mc_failed;
        stats->base_cases = (int64_t)hc.base_cases;
        stats->base_triples = (int64_t)hc.base_triples;
        stats->mc_samples = (int64_t)hc.mc_samples;
        stats->max_stack = max_stack;
        stats->rounds = rounds;
        stats->classify_ms = phase_ms[0];
        stats->mc_ms = phase_ms[1];
        stats->base_ms = phase_ms[2];
        stats->traverse_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return MB_OK;
}

}  // namespace mb
