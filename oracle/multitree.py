"""Triple-tree (multi-tree) Axilrod-Teller potential on the CPU - oracle side.

TEST INFRASTRUCTURE ONLY.

This is the paper's algorithm written out in its own order, for n = 3:

  1. bottom-up: BuildKdTree (Algorithm 1, ``oracle.kdtree``); at expansion
     order p = 0 a node's moment is its point count (Section 4);
  2. approximation: MTPotentialCanonical over node triples (Algorithm 2),
     started at (root, root, root).  For each canonical triple, in order:
       a. deterministic prune (Section 4 and Section 4.1, the hybrid rule of
          the deterministic-prune equation): Summarize adds T_i * phi(c1,c2,c3)
          to node P_i and raises the running lower bound by
          delta^l_i = T_i * phi_lo;
       b. Monte Carlo prune (Algorithms 3 and 4 with the relative-error
          termination rule, committed by Algorithm 5);
       c. if all three nodes are leaves: the exhaustive base case
          MTPotentialBase;
       d. otherwise: split and recurse on the canonical children;
  3. top-down: node accumulators are pushed to their points (Section 3).

Readings taken where the paper is silent, garbled or does not fit the
Axilrod-Teller potential:
  * Canonical triples.  A triple (P1, P2, P3) is kept in depth-first order
    with every two nodes equal or disjoint; its case is (a) all equal,
    (b) P1 = P2 < P3, (c) P1 < P2 = P3, (d) all distinct (the four-case
    figure of Section 3).  The redundancy rule of Section 3 is printed with
    the inequality reversed; triples that it is meant to discard are never
    generated here, because children are emitted only in canonical order.
  * Splitting.  Every non-leaf node of the triple is split at once and the
    children are emitted in canonical order ((a) -> LLL, LLR, LRR, RRR;
    (b) -> {LL, LR, RR} x {B_L, B_R}; ...).  This partitions the particle
    triples exactly, as the proofs of Section 5 assume (up to 8 sub-calls).
  * T_i (tuples through a fixed point of P_i, Section 4.1):
        (a) C(n-1, 2);
        (b) x in A: (n_A - 1) n_B, x in B: C(n_A, 2);
        (c) x in A: C(n_B, 2), x in B: n_A (n_B - 1);
        (d) the product of the other two counts;
    T_root = C(N - 1, 2).
  * Bounds for Axilrod-Teller.  The paper's bound (Section 4) takes a
    monotone potential at the largest and smallest node distances d^u, d^l;
    Axilrod-Teller is neither monotone nor of one sign.  ``at_bounds``
    bounds phi = R g over all triangles whose sides lie between d^l and d^u
    of the three node pairs: R = (r_12 r_13 r_23)^-3 between its values at
    d^u and d^l, and the angular factor g = 1 + 3 cos cos cos from the exact
    range of each cosine over the box of squared sides, clipped to
    [-2, 11/8] (collinear, equilateral).  phi_lo takes the role of the
    paper's phi(d^u) and phi_hi that of phi(d^l): the prune test compares
    phi_hi - phi_lo with the allowance and delta^l_i = T_i phi_lo.  Every
    d^l is raised to the closest-pair distance of the set.  Only case (d)
    is tested (a node paired with itself has d^l = 0).
  * Running lower bound Phi^l.  LB(x) accumulates the lower bounds of
    everything already credited to x (exact base-case values, delta^l of
    deterministic prunes, T_i (mu - z sigma_mu) of Monte Carlo prunes);
    Phi^l(P) = min over x in P of LB(x).  For a sign-indefinite potential
    this is the paper's running sum, not a bound on the final total.
  * Monte Carlo termination (relative form): stop once m >= m_min and
        z sigma_mu <= (eps (Phi^l(P_i) + T_i (mu - z sigma_mu)) + tau) / T_root,
    i.e. the per-tuple error allowance of the deterministic rule; the
    printed equation drops T_i from the eps term while the proof of
    Theorem 5.2 keeps it.  A point passes iff this holds with m >= m_min
    samples, m <= m_limit.  MC is tried only if alpha > 0 and
    zeta * m_limit <= min_i T_i.  Defaults: m_limit = 128, zeta = 4,
    m_min = 30 (the rule of thumb quoted after Theorem 4.1).
  * z = z_{alpha/2}, the two-sided normal quantile; beta = alpha in
    Algorithm 5.
  * Samples are i.i.d. with replacement, each uniform over the T_i tuples of
    the node triple that contain x, drawn from Philox4x32-10 with
    counter (x, s, p1, p2) and key (p3, seed ^ seed >> 32), where x is the
    depth-first rank of the point, s the sample number and p1..p3 the node
    numbers.  A 64-bit uniform integer r is (w1 << 32 | w0); an index in
    [0, M) is floor(r * M / 2^64).
  * Test order: deterministic, then Monte Carlo, then base case or split.
  * Sign-indefinite potentials.  The running lower bound of a point whose
    Phi is negative stays negative, and the paper's relative rule then never
    prunes a triple holding that point.  With bound="two_sided" a running
    upper bound UB(x) is kept beside LB(x) (same credits with the upper ends
    of the intervals) and the allowance bounds max(LB, -UB) from below: the
    relative bound of Definition 2.2 is on |Phi|, and once the sign of a
    point's running total is settled either side certifies its size.  For a
    non-negative potential it is the paper's rule.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from statistics import NormalDist

import numpy as np

from .farfield import farfield
from .kdtree import KdTree, box_max_dist, box_min_dist, build_kdtree
from .philox import philox4x32_10_np


def comb2(n):
    return n * (n - 1) // 2


def at_phi_np(xi: np.ndarray, xj: np.ndarray, xk: np.ndarray) -> np.ndarray:
    """Vectorized Axilrod-Teller phi (Section 1), cosines from dot products."""
    dij = xj - xi
    dik = xk - xi
    djk = xk - xj
    rij = np.sqrt(np.einsum("...d,...d->...", dij, dij))
    rik = np.sqrt(np.einsum("...d,...d->...", dik, dik))
    rjk = np.sqrt(np.einsum("...d,...d->...", djk, djk))
    ci = np.einsum("...d,...d->...", dij, dik) / (rij * rik)
    cj = -np.einsum("...d,...d->...", dij, djk) / (rij * rjk)
    ck = np.einsum("...d,...d->...", dik, djk) / (rik * rjk)
    r3 = (rij * rik * rjk) ** 3
    return (1.0 + 3.0 * ci * cj * ck) / r3


def canonical_case(p1: int, p2: int, p3: int) -> str:
    if p1 == p2 == p3:
        return "a"
    if p1 == p2:
        return "b"
    if p2 == p3:
        return "c"
    return "d"


def distinct_roles(p: tuple[int, int, int], n: tuple[int, int, int]) -> list[tuple[int, int, int]]:
    """(node, T_i, slot) for each distinct node of a canonical triple, in order.

    ``slot`` is the first position (0, 1, 2) the node takes in the triple.
    """
    p1, p2, p3 = p
    n1, n2, n3 = n
    case = canonical_case(p1, p2, p3)
    if case == "a":
        return [(p1, comb2(n1 - 1), 0)]
    if case == "b":
        return [(p1, (n1 - 1) * n3, 0), (p3, comb2(n1), 2)]
    if case == "c":
        return [(p1, comb2(n2), 0), (p2, n1 * (n2 - 1), 1)]
    return [(p1, n2 * n3, 0), (p2, n1 * n3, 1), (p3, n1 * n2, 2)]


def triple_index_arrays(case: str, r1: np.ndarray, r2: np.ndarray, r3: np.ndarray):
    """All canonical particle triples (i, j, k) of a node triple, as rank arrays."""
    if case == "a":
        a = r1
        if a.size < 3:
            e = np.zeros(0, dtype=np.int64)
            return e, e, e
        ii, jj, kk = np.meshgrid(a, a, a, indexing="ij")
        m = (ii < jj) & (jj < kk)
        return ii[m], jj[m], kk[m]
    if case == "b":
        ii, jj, kk = np.meshgrid(r1, r1, r3, indexing="ij")
        m = ii < jj
        return ii[m], jj[m], kk[m]
    if case == "c":
        ii, jj, kk = np.meshgrid(r1, r2, r2, indexing="ij")
        m = jj < kk
        return ii[m], jj[m], kk[m]
    ii, jj, kk = np.meshgrid(r1, r2, r3, indexing="ij")
    return ii.ravel(), jj.ravel(), kk.ravel()


def canonical_children(tree: KdTree, p: tuple[int, int, int]) -> list[tuple[int, int, int]]:
    """Split every non-leaf node; children in canonical (depth-first) order."""
    opts = []
    for node in p:
        opts.append([node] if tree.is_leaf(node) else [int(tree.left[node]), int(tree.right[node])])
    seen = set()
    out = []
    for a in opts[0]:
        for b in opts[1]:
            for c in opts[2]:
                t = tuple(sorted((a, b, c), key=lambda v: (tree.begin[v], v)))
                if t in seen:
                    continue
                seen.add(t)
                out.append(t)
    out.sort(key=lambda t: (tree.begin[t[0]], tree.begin[t[1]], tree.begin[t[2]]))
    return out


def mc_draw(seed: int, p: tuple[int, int, int], x_rank: int, s: np.ndarray) -> np.ndarray:
    """64-bit uniform integers for samples s of point x in node triple p.

    One Philox block (four 32-bit words) serves two consecutive samples:
    sample s uses counter (x, s // 2, p1, p2), key (p3, seed), and words
    (0, 1) for even s, (2, 3) for odd s.
    """
    s = s.astype(np.uint64)
    m = s.shape[0]
    ctr = np.zeros((m, 4), dtype=np.uint64)
    ctr[:, 0] = x_rank
    ctr[:, 1] = s >> np.uint64(1)
    ctr[:, 2] = p[0]
    ctr[:, 3] = p[1]
    key = np.zeros((m, 2), dtype=np.uint64)
    key[:, 0] = p[2]
    key[:, 1] = (seed ^ (seed >> 32)) & 0xFFFFFFFF
    w = philox4x32_10_np(ctr, key).astype(np.uint64)
    odd = (s & np.uint64(1)).astype(bool)
    lo = np.where(odd, w[:, 2], w[:, 0])
    hi = np.where(odd, w[:, 3], w[:, 1])
    return (hi << np.uint64(32)) | lo


def uniform_index(r: np.ndarray, m: int) -> np.ndarray:
    """floor(r * m / 2^64) for 64-bit r and 0 < m < 2^63 (the high word of r * m)."""
    mask = np.uint64(0xFFFFFFFF)
    sh = np.uint64(32)
    r = r.astype(np.uint64)
    rh, rl = r >> sh, r & mask
    mh, ml = np.uint64(m) >> sh, np.uint64(m) & mask
    t = (rl * ml) >> sh
    t1 = rh * ml + t
    t2 = rl * mh + (t1 & mask)
    return (rh * mh + (t1 >> sh) + (t2 >> sh)).astype(np.int64)


def pair_from_index(t: np.ndarray, m: int) -> tuple[np.ndarray, np.ndarray]:
    """Unordered pair (u < v) of [0, m) from its index t in [0, C(m, 2)), v-major."""
    v = np.floor((1.0 + np.sqrt(1.0 + 8.0 * t.astype(np.float64))) / 2.0).astype(np.int64)
    v = np.where(v * (v - 1) // 2 > t, v - 1, v)
    v = np.where((v + 1) * v // 2 <= t, v + 1, v)
    u = t - v * (v - 1) // 2
    return u, v


def sample_partners(case: str, slot: int, x_local: np.ndarray, n: tuple[int, int, int],
                    r: np.ndarray) -> tuple[np.ndarray, np.ndarray, int, int]:
    """Map uniform integers to the two partners of x (uniform over the T_i tuples).

    ``slot`` is the triple position of x's node, ``x_local`` the offset of x
    inside it (broadcast against ``r``).  Returns the partners' offsets
    inside their nodes and the triple positions of those nodes.
    """
    n1, n2, n3 = n
    if case == "a":  # a pair of distinct points of A minus x
        u, v = pair_from_index(uniform_index(r, comb2(n1 - 1)), n1 - 1)
        return u + (u >= x_local), v + (v >= x_local), 0, 0
    if case == "b":
        if slot == 0:  # x in A: one partner in A minus x, one in B
            t = uniform_index(r, (n1 - 1) * n3)
            u, v = t // n3, t % n3
            return u + (u >= x_local), v, 0, 2
        u, v = pair_from_index(uniform_index(r, comb2(n1)), n1)  # x in B: a pair in A
        return u, v, 0, 0
    if case == "c":
        if slot == 0:  # x in A: a pair in B
            u, v = pair_from_index(uniform_index(r, comb2(n2)), n2)
            return u, v, 1, 1
        t = uniform_index(r, n1 * (n2 - 1))  # x in B: one partner in A, one in B minus x
        u, v = t // (n2 - 1), t % (n2 - 1)
        return u, v + (v >= x_local), 0, 1
    others = [s_ for s_ in (0, 1, 2) if s_ != slot]
    nb = n[others[1]]
    t = uniform_index(r, n[others[0]] * nb)
    return t // nb, t % nb, others[0], others[1]


def cos_range(a: tuple[float, float], b: tuple[float, float],
              c: tuple[float, float]) -> tuple[float, float]:
    """Range of the cosine of a triangle's angle over boxes of squared sides.

    The angle lies between the sides of squared lengths a and b; c is the
    squared length of the side opposite it; each is given as an interval
    (lower, upper).  By the law of cosines cos = h(a, b, c) with
    h = (a + b - c) / (2 sqrt(a b)).

    * h falls as c grows, so the largest value has c at its lower end and the
      smallest has c at its upper end.
    * For fixed c, with s = sqrt(a), t = sqrt(b): dh/dt = (t^2 - s^2 + c) /
      (2 s t^2), so along an edge of the (a, b) box h first falls, then rises
      (a single minimum at b = a - c, when a > c, where h = sqrt(1 - c/a):
      the angle facing the side a is right); by symmetry the same holds in a.
      Both derivatives vanish together only if c = 0, so for c > 0 there is
      no critical point inside the box.
    * Hence the maximum is at one of the four corners (c low), and the
      minimum at a corner or at an edge point b = a - c or a = b - c (c high).

    The box may hold (a, b, c) that are not triangles; cosines of real
    triangles lie in [-1, 1], so the range is clipped there.
    """
    def h(a_, b_, c_):
        return (a_ + b_ - c_) / (2.0 * math.sqrt(a_ * b_))

    top = max(h(a_, b_, c[0]) for a_ in a for b_ in b)
    cands = [h(a_, b_, c[1]) for a_ in a for b_ in b]
    for a_ in a:  # edge a fixed, b free
        bs = a_ - c[1]
        if b[0] < bs < b[1]:
            cands.append(math.sqrt(1.0 - c[1] / a_))
    for b_ in b:  # edge b fixed, a free
        as_ = b_ - c[1]
        if a[0] < as_ < a[1]:
            cands.append(math.sqrt(1.0 - c[1] / b_))
    return max(-1.0, min(cands)), min(1.0, top)


def at_bounds(lo: tuple[float, float, float], up: tuple[float, float, float]) -> tuple[float, float]:
    """(phi_lo, phi_hi) over every triangle whose sides lie between lo and up.

    lo = (d^l_12, d^l_13, d^l_23) and up = (d^u_12, d^u_13, d^u_23), the
    smallest and largest distances between the three node pairs (the
    distance bounds of Section 3).  Section 4 bounds a monotone potential by
    its values at d^u and d^l; the Axilrod-Teller phi is neither monotone nor
    of one sign, so it is bounded as the product of two factors,

        phi = R * g,  R = (r_12 r_13 r_23)^-3,  g = 1 + 3 cos t_1 cos t_2 cos t_3,

    each over its own range: R lies in [R(d^u), R(d^l)]; each cosine lies in
    the range of ``cos_range`` (t_1 is the angle at node 1, between sides 12
    and 13, facing side 23); the product of three intervals is taken over
    its eight corners; and g is clipped to [-2, 11/8], its values at a
    collinear and an equilateral triangle, the extremes over all triangles.
    phi_lo pairs the lower end of g with the R that makes it smallest, and
    phi_hi likewise.  The result never lies outside [-2 R(d^l), 11/8 R(d^l)].
    """
    a = (lo[0] ** 2, up[0] ** 2)  # side 12
    b = (lo[1] ** 2, up[1] ** 2)  # side 13
    c = (lo[2] ** 2, up[2] ** 2)  # side 23
    r_hi = 1.0 / (lo[0] * lo[1] * lo[2]) ** 3
    r_lo = 1.0 / (up[0] * up[1] * up[2]) ** 3
    c1 = cos_range(a, b, c)  # at node 1: sides 12, 13; opposite 23
    c2 = cos_range(a, c, b)  # at node 2: sides 12, 23; opposite 13
    c3 = cos_range(b, c, a)  # at node 3: sides 13, 23; opposite 12
    prods = [u * v * w for u in c1 for v in c2 for w in c3]
    g_lo = max(-2.0, 1.0 + 3.0 * min(prods))
    g_hi = min(1.375, 1.0 + 3.0 * max(prods))
    phi_lo = g_lo * (r_lo if g_lo >= 0.0 else r_hi)
    phi_hi = g_hi * (r_hi if g_hi >= 0.0 else r_lo)
    return phi_lo, phi_hi


def node_radius(tree: KdTree, v: int) -> float:
    """Largest distance from the centroid of node v to a corner of its box."""
    c = tree.centroid[v]
    d = np.maximum(tree.hi[v] - c, c - tree.lo[v])
    return float(np.sqrt(d @ d))


def well_separated(tree: KdTree, p: tuple[int, int, int], theta: float = 0.5) -> bool:
    """Whether every two nodes of the triple satisfy r_a + r_b <= theta |c_a - c_b|.

    The far-field expansion of Section 3.2 is a Taylor series in the
    displacements of P2's and P3's points from their centres; it converges
    only when the nodes are small against their distances (a multipole
    acceptance criterion).  Triples that fail it keep the p = 0 estimate.
    """
    for u, v in ((p[0], p[1]), (p[0], p[2]), (p[1], p[2])):
        d = tree.centroid[u] - tree.centroid[v]
        if node_radius(tree, u) + node_radius(tree, v) > theta * float(np.sqrt(d @ d)):
            return False
    return True


def closest_pair(x: np.ndarray) -> float:
    """Smallest distance between two points of the set (brute force over all pairs)."""
    best = math.inf
    for i in range(x.shape[0] - 1):
        d = x[i + 1:] - x[i]
        best = min(best, float(np.einsum("ij,ij->i", d, d).min()))
    return math.sqrt(best)


def node_triple_bounds(tree: KdTree, p: tuple[int, int, int], r_min: float) -> tuple[float, float]:
    """at_bounds of a node triple; every d^l is raised to the closest-pair
    distance r_min of the whole set (no two points are closer)."""
    p1, p2, p3 = p
    pairs = ((p1, p2), (p1, p3), (p2, p3))
    lo = tuple(max(box_min_dist(tree.lo[u], tree.hi[u], tree.lo[v], tree.hi[v]), r_min)
               for u, v in pairs)
    up = tuple(max(box_max_dist(tree.lo[u], tree.hi[u], tree.lo[v], tree.hi[v]), l_)
               for (u, v), l_ in zip(pairs, lo))
    return at_bounds(lo, up)


def certified(bound: str, stat, t, lo, hi):
    """Lower bound on |Phi(x)| for every x of a node after it is credited t
    tuples whose values lie in [lo, hi] (numbers or arrays).

    ``stat`` holds the node's statistics before the credit:
      "signed"    (the paper, Section 4.1): stat = Phi^l(P) = min_x LB(x);
                  the result is Phi^l(P) + t lo (lo plays delta^l / t);
      "two_sided" (a reading for sign-indefinite potentials): stat =
                  (min_x LB(x), min_x -UB(x), min_x max(LB(x), -UB(x))) with
                  UB the running upper bound; after the credit
                  max(LB + t lo, -(UB + t hi)) is at least each of
                  min LB + t lo, min(-UB) - t hi and
                  min max(LB, -UB) + min(t lo, -t hi), so their largest is a
                  lower bound.  When every LB is positive the first term
                  wins and this is the paper's rule.
    """
    if bound == "signed":
        return stat + t * lo
    a_pos, a_neg, a_mix = stat
    return np.maximum(np.maximum(a_pos + t * lo, a_neg - t * hi),
                      a_mix + np.minimum(t * lo, -t * hi))


def mc_try(tree: KdTree, xs: np.ndarray, p: tuple[int, int, int], roles, cnt, phil,
           eps: float, tau: float, t_root: int, z: float, seed: int, m_limit: int, m_min: int,
           bound: str = "signed"):
    """Monte Carlo test of one node triple (Algorithm 3, Algorithm 4 per point).

    For every point x of every distinct node P_i (``roles`` = (node, T_i,
    slot), ``phil`` = Phi^l(P_i)), samples are drawn one at a time and the
    running mean and unbiased variance updated; x stops at the first m with
    m >= m_min and
        z sigma_mu <= (eps (Phi^l(P_i) + T_i (mu - z sigma_mu)) + tau) / T_root,
    and passes if that holds, else fails at m = m_limit.  ``phil`` holds
    the node statistics of ``bound`` and the credit is ``certified`` with the
    interval [mu - z sigma_mu, mu + z sigma_mu] per tuple (for "signed" the
    printed rule above).  Points are scanned
    in order and the scan ends at the first failure.  Returns (all passed,
    [(first rank, T_i, mu per point, sigma_mu per point)], samples used).
    """
    case = canonical_case(*p)
    commits = []
    used_total = 0
    for (node, t, slot), plo in zip(roles, phil):
        base = int(tree.begin[node])
        npts = cnt[slot]
        xl = np.arange(npts, dtype=np.int64)[:, None]
        xr = base + xl
        r = np.stack([mc_draw(seed, p, int(base + q), np.arange(m_limit, dtype=np.uint64))
                      for q in range(npts)])
        u, v, su, sv = sample_partners(case, slot, xl, cnt, r)
        f = at_phi_np(xs[xr], xs[tree.begin[p[su]] + u], xs[tree.begin[p[sv]] + v])
        mean = np.zeros(npts)
        m2 = np.zeros(npts)
        stop_m = np.full(npts, -1, dtype=np.int64)
        mu_s = np.zeros(npts)
        sg_s = np.zeros(npts)
        passed = np.zeros(npts, dtype=bool)
        for k in range(m_limit):
            m = k + 1
            d = f[:, k] - mean
            mean = mean + d / m
            m2 = m2 + d * (f[:, k] - mean)
            if m < 2:
                continue
            sig_mu = np.sqrt(m2 / (m - 1) / m)
            credit = certified(bound, plo, t, mean - z * sig_mu, mean + z * sig_mu)
            cond = z * sig_mu <= (eps * credit + tau) / t_root
            fresh = (stop_m < 0) & ((cond & (m >= m_min)) | (m == m_limit))
            stop_m[fresh] = m
            mu_s[fresh] = mean[fresh]
            sg_s[fresh] = sig_mu[fresh]
            passed[fresh] = cond[fresh] & (m >= m_min)
        fail = np.nonzero(~passed)[0]
        used = stop_m if fail.size == 0 else stop_m[: fail[0] + 1]
        used_total += int(used.sum())
        if fail.size:
            return False, [], used_total
        commits.append((base, t, mu_s, sg_s))
    return True, commits, used_total


@dataclass
class MTResult:
    phi: np.ndarray                # estimate, input order
    lower: np.ndarray              # running lower bound LB(x), input order
    coverage: np.ndarray           # tuples credited per point, input order (int64)
    tree: KdTree
    stats: dict = field(default_factory=dict)


def multitree(x, eps: float, alpha: float, leaf_size: int, tau: float = 0.0, seed: int = 0,
              m_limit: int = 128, zeta: float = 4.0, m_min: int = 30,
              bound: str = "signed", order: int = 0) -> MTResult:
    """The traversal.  ``bound`` chooses the node statistic of the prune rules:

    * "signed": the paper's running lower bound Phi^l (Section 4.1);
    * "two_sided" (a reading for sign-indefinite potentials): running lower
      and upper bounds LB, UB per point, and the allowance is a lower bound
      on max(LB, -UB), i.e. on |Phi| when its sign is settled (see
      ``certified``); for potentials >= 0 it is the paper's rule.

    ``order`` is the expansion order p of a deterministic prune's estimate:
    0 is the monopole of Section 4 (every point of P_i gets T_i phi(c1, c2,
    c3)); p >= 1 is the truncated three-body far-field expansion of Section
    3.2 at each point x of P_i due to the other two nodes (``farfield``),
    kept inside [T_i phi_lo, T_i phi_hi], for node triples where it
    converges (``well_separated``; others keep the monopole).  The prune
    test itself is the same for every p (the paper states no error bound for
    p > 0).
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    if eps < 0 or tau < 0 or not (0.0 <= alpha < 1.0) or leaf_size < 1 or order < 0:
        raise ValueError("bad multitree parameters")
    if bound not in ("signed", "two_sided"):
        raise ValueError("bound must be 'signed' or 'two_sided'")
    tree = build_kdtree(x, leaf_size)
    xs = x[tree.perm]  # depth-first order
    r_min = closest_pair(x)
    t_root = comb2(n - 1) if n >= 1 else 0
    z = NormalDist().inv_cdf(1.0 - alpha / 2.0) if alpha > 0 else math.inf
    est = np.zeros(n)
    lb = np.zeros(n)
    ub = np.zeros(n)   # running upper bound (two_sided)
    cov = np.zeros(n, dtype=np.int64)
    node_acc = np.zeros(tree.n_nodes)
    st = dict(visited=0, det_prunes=0, mc_prunes=0, mc_failed=0, base_cases=0, base_triples=0,
              mc_samples=0)
    if n < 3:
        return MTResult(np.zeros(n), np.zeros(n), cov, tree, st)

    def pts(node):
        return slice(int(tree.begin[node]), int(tree.end[node]))

    def phi_l(node):
        if bound == "signed":
            return float(lb[pts(node)].min())
        lo_, up_ = lb[pts(node)], ub[pts(node)]
        return float(lo_.min()), float((-up_).min()), float(np.maximum(lo_, -up_).min())

    stack = [(0, 0, 0)]
    while stack:
        p = stack.pop()
        st["visited"] += 1
        p1, p2, p3 = p
        case = canonical_case(p1, p2, p3)
        cnt = (int(tree.count[p1]), int(tree.count[p2]), int(tree.count[p3]))
        roles = distinct_roles(p, cnt)

        # (a) deterministic prune, case (d) only
        if case == "d":
            phi_lo, phi_hi = node_triple_bounds(tree, p, r_min)
            allow = min(certified(bound, phi_l(node), t, phi_lo, phi_hi) for node, t, _ in roles)
            if phi_hi - phi_lo <= (eps * allow + tau) / t_root:
                phic = float(at_phi_np(tree.centroid[p1], tree.centroid[p2], tree.centroid[p3]))
                use_ff = order > 0 and well_separated(tree, p)
                for node, t, slot in roles:
                    if not use_ff:
                        node_acc[node] += t * phic
                    else:
                        oth = [xs[pts(v)] for q_, v in enumerate(p) if q_ != slot]
                        for r_ in range(int(tree.begin[node]), int(tree.end[node])):
                            f = farfield(xs[r_], oth[0], oth[1], order)
                            est[r_] += min(max(f, t * phi_lo), t * phi_hi)
                    lb[pts(node)] += t * phi_lo
                    ub[pts(node)] += t * phi_hi
                    cov[pts(node)] += t
                st["det_prunes"] += 1
                continue

        # (b) Monte Carlo prune (Algorithm 3 over the distinct nodes, Algorithm 4 per point)
        if alpha > 0 and zeta * m_limit <= min(t for _, t, _ in roles):
            ok, commits, used = mc_try(tree, xs, p, roles, cnt, [phi_l(node) for node, _, _ in roles],
                                       eps, tau, t_root, z, seed, m_limit, m_min, bound)
            st["mc_samples"] += used
            if ok:
                for base, t, mu_s, sg_s in commits:
                    sl = slice(base, base + mu_s.shape[0])
                    est[sl] += t * mu_s
                    lb[sl] += t * (mu_s - z * sg_s)
                    ub[sl] += t * (mu_s + z * sg_s)
                    cov[sl] += t
                st["mc_prunes"] += 1
                continue
            st["mc_failed"] += 1

        # (c) base case
        if tree.is_leaf(p1) and tree.is_leaf(p2) and tree.is_leaf(p3):
            ri, rj, rk = triple_index_arrays(case, np.arange(*pts(p1).indices(n)),
                                             np.arange(*pts(p2).indices(n)),
                                             np.arange(*pts(p3).indices(n)))
            if ri.size:
                f = at_phi_np(xs[ri], xs[rj], xs[rk])
                for r_ in (ri, rj, rk):
                    np.add.at(est, r_, f)
                    np.add.at(lb, r_, f)
                    np.add.at(ub, r_, f)
                    np.add.at(cov, r_, 1)
            st["base_cases"] += 1
            st["base_triples"] += int(ri.size)
            continue

        # (d) split: push children so that the first canonical child is processed first
        kids = canonical_children(tree, p)
        for c in reversed(kids):
            stack.append(c)

    # top-down: node accumulators to their points
    for node in range(tree.n_nodes):
        if node_acc[node] != 0.0:
            est[pts(node)] += node_acc[node]
    out = np.empty(n)
    out[tree.perm] = est
    low = np.empty(n)
    low[tree.perm] = lb
    cv = np.empty(n, dtype=np.int64)
    cv[tree.perm] = cov
    return MTResult(out, low, cv, tree, st)
