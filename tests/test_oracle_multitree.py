"""Pins of the CPU tree and traversal oracle (no GPU).

What fixes each part without another implementation to compare against:
  * the kd-tree: the invariants of Algorithm 1 with the median-by-count
    reading (partition, tight boxes, centroids, widest-dimension split,
    leaf threshold, pre-order numbering);
  * canonical children: recursing from (root, root, root) to leaf triples
    lists every unordered particle triple exactly once (brute force);
  * T_i per canonical case: brute-force counting of the tuples through each
    point of a node triple;
  * the Monte Carlo sampler: every draw is a valid tuple through the point,
    and all T_i tuples are drawn with equal frequency (chi-square);
  * the 64-bit index map and the pair index: exact integer arithmetic;
  * the traversal: eps = 0, alpha = 0 is the exhaustive sum (and each
    particle is credited with C(N-1, 2) tuples); with alpha = 0 every
    particle is within eps (Theorem 5.1, positive Phi); with alpha > 0 at
    least a 1 - alpha fraction is (Theorem 5.2).
"""
import itertools
import math

import numpy as np
import pytest

import workloads
from oracle import direct as oracle_direct
from oracle import kdtree as okd
from oracle import multitree as omt


def blobs(n_per: int, centers, seed: int) -> np.ndarray:
    parts = [workloads.jittered_lattice(n_per, seed=seed + q) + np.asarray(c, float)
             for q, c in enumerate(centers)]
    return np.concatenate(parts)


def test_kdtree_invariants():
    x = workloads.uniform_cube(500, seed=3) * np.array([1.0, 3.0, 2.0])
    t = okd.build_kdtree(x, 8)
    assert sorted(t.perm.tolist()) == list(range(500))
    assert t.begin[0] == 0 and t.end[0] == 500
    xs = x[t.perm]
    for v in range(t.n_nodes):
        b, e = int(t.begin[v]), int(t.end[v])
        pts = xs[b:e]
        np.testing.assert_array_equal(t.lo[v], pts.min(0))
        np.testing.assert_array_equal(t.hi[v], pts.max(0))
        np.testing.assert_allclose(t.centroid[v], pts.mean(0), rtol=1e-15, atol=1e-15)
        if e - b <= 8:
            assert t.left[v] < 0 and t.right[v] < 0
            continue
        lc, rc = int(t.left[v]), int(t.right[v])
        assert lc == v + 1 and t.parent[lc] == v and t.parent[rc] == v
        assert t.begin[lc] == b and t.end[lc] == b + (e - b) // 2
        assert t.begin[rc] == t.end[lc] and t.end[rc] == e
        d = int(np.argmax(t.hi[v] - t.lo[v]))
        keys_l = [(x[i, d], i) for i in t.perm[b:t.end[lc]]]
        keys_r = [(x[i, d], i) for i in t.perm[t.begin[rc]:e]]
        assert max(keys_l) < min(keys_r)


def leaf_triples(t, p=(0, 0, 0)):
    if all(t.is_leaf(v) for v in p):
        yield p
        return
    for c in omt.canonical_children(t, p):
        yield from leaf_triples(t, c)


@pytest.mark.parametrize("n,leaf", [(14, 2), (23, 3), (9, 1)])
def test_canonical_children_cover_each_triple_once(n, leaf):
    x = workloads.uniform_cube(n, seed=n)
    t = okd.build_kdtree(x, leaf)
    seen = {}
    for p in leaf_triples(t):
        case = omt.canonical_case(*p)
        r = [np.arange(t.begin[v], t.end[v]) for v in p]
        for tri in zip(*omt.triple_index_arrays(case, *r)):
            key = tuple(sorted(int(v) for v in tri))
            assert len(set(key)) == 3
            seen[key] = seen.get(key, 0) + 1
    assert len(seen) == math.comb(n, 3)
    assert set(seen.values()) == {1}


@pytest.mark.parametrize("case,n", [("a", (6, 6, 6)), ("b", (5, 5, 4)), ("c", (3, 6, 6)),
                                    ("d", (4, 5, 3))])
def test_t_i_counts_brute_force(case, n):
    # node ranges laid out in depth-first order: equal nodes share a range
    starts = {"a": (0, 0, 0), "b": (0, 0, 10), "c": (0, 10, 10), "d": (0, 10, 20)}[case]
    r = [np.arange(s, s + k) for s, k in zip(starts, n)]
    ii, jj, kk = omt.triple_index_arrays(case, *r)
    through = {}
    for tri in zip(ii, jj, kk):
        for v in tri:
            through[int(v)] = through.get(int(v), 0) + 1
    ids = {"a": (1, 1, 1), "b": (1, 1, 2), "c": (1, 2, 2), "d": (1, 2, 3)}[case]
    for node, t_i, slot in omt.distinct_roles(ids, n):
        for v in r[slot]:
            assert through[int(v)] == t_i


def valid_partners(case, slot, xl, n):
    """Brute-force set of (slot_u, u, slot_v, v) tuples through point xl of slot."""
    starts = {"a": (0, 0, 0), "b": (0, 0, 100), "c": (0, 100, 100), "d": (0, 100, 200)}[case]
    r = [np.arange(s, s + k) for s, k in zip(starts, n)]
    x_rank = starts[slot] + xl
    out = set()
    for tri in zip(*omt.triple_index_arrays(case, *r)):
        tri = [int(v) for v in tri]
        if x_rank in tri:
            rest = sorted(v for v in tri if v != x_rank)
            out.add(tuple(rest))
    return out, starts


@pytest.mark.parametrize("case,slot,n", [("a", 0, (6, 6, 6)), ("b", 0, (5, 5, 4)),
                                         ("b", 2, (5, 5, 4)), ("c", 0, (3, 5, 5)),
                                         ("c", 1, (3, 5, 5)), ("d", 0, (3, 4, 5)),
                                         ("d", 1, (3, 4, 5)), ("d", 2, (3, 4, 5))])
def test_sampler_valid_and_uniform(case, slot, n):
    rng = workloads.rng(7)
    draws = 40000
    for xl in (0, n[slot] - 1):
        valid, starts = valid_partners(case, slot, xl, n)
        r = rng.integers(0, 2**64, size=draws, dtype=np.uint64)
        u, v, su, sv = omt.sample_partners(case, slot, np.int64(xl), n, r)
        got = {}
        for a, b in zip(u, v):
            key = tuple(sorted((starts[su] + int(a), starts[sv] + int(b))))
            got[key] = got.get(key, 0) + 1
        assert set(got) == valid
        counts = np.array(list(got.values()), dtype=float)
        expect = draws / len(valid)
        chi2 = float(((counts - expect) ** 2 / expect).sum())
        dof = len(valid) - 1
        # 5 sigma of the chi-square distribution: a skewed map fails by far
        assert chi2 < dof + 5 * math.sqrt(2 * dof)


def test_uniform_index_exact():
    rng = workloads.rng(8)
    r = rng.integers(0, 2**64, size=2000, dtype=np.uint64)
    for m in (1, 2, 3, 1000, 2**31 - 1, 2**40 + 17, 2**62 + 5):
        got = omt.uniform_index(r, m)
        want = [(int(a) * m) >> 64 for a in r]
        assert got.tolist() == want


def test_pair_index_bijection():
    for m in range(2, 60):
        t = np.arange(m * (m - 1) // 2)
        u, v = omt.pair_from_index(t, m)
        pairs = set(zip(u.tolist(), v.tolist()))
        assert len(pairs) == t.size
        assert all(0 <= a < b < m for a, b in pairs)


@pytest.mark.parametrize("n,leaf", [(40, 4), (57, 3)])
def test_eps0_equals_exhaustive(n, leaf):
    x = workloads.jittered_lattice(n, seed=n)
    res = omt.multitree(x, eps=0.0, alpha=0.0, leaf_size=leaf)
    np.testing.assert_allclose(res.phi, oracle_direct.phi(x), rtol=1e-12)
    assert np.all(res.coverage == math.comb(n - 1, 2))
    assert res.stats["det_prunes"] == 0 and res.stats["mc_prunes"] == 0


def test_deterministic_mode_within_eps():
    # five compact clusters far apart: triples across three clusters prune
    x = blobs(24, [(0, 0, 0), (40, 0, 0), (0, 40, 0), (0, 0, 40), (40, 40, 40)], seed=11)
    eps = 0.05
    res = omt.multitree(x, eps=eps, alpha=0.0, leaf_size=4)
    ref = oracle_direct.phi(x)
    rel = np.abs(res.phi - ref) / np.abs(ref)
    assert res.stats["det_prunes"] > 0
    assert np.all(res.coverage == math.comb(x.shape[0] - 1, 2))
    assert rel.max() <= eps


def test_monte_carlo_mode_fraction_within_eps():
    x = blobs(48, [(0, 0, 0), (9, 0, 0), (0, 9, 0), (0, 0, 9)], seed=21)
    eps, alpha = 0.05, 0.1
    res = omt.multitree(x, eps=eps, alpha=alpha, leaf_size=4, m_limit=64, zeta=2.0, seed=5)
    ref = oracle_direct.phi(x)
    rel = np.abs(res.phi - ref) / np.abs(ref)
    assert res.stats["mc_prunes"] > 0
    assert np.all(res.coverage == math.comb(x.shape[0] - 1, 2))
    assert np.mean(rel <= eps) >= 1.0 - alpha


def _cos_grid(a, b, c, m=161):
    """Extremes of (a + b - c) / (2 sqrt(ab)) on a dense grid of the box (brute force)."""
    ga = np.linspace(a[0], a[1], m)[:, None, None]
    gb = np.linspace(b[0], b[1], m)[None, :, None]
    gc = np.linspace(c[0], c[1], 7)[None, None, :]
    h = (ga + gb - gc) / (2.0 * np.sqrt(ga * gb))
    return float(h.min()), float(h.max())


@pytest.mark.parametrize("a,b,c", [
    ((4.0, 9.0), (0.5, 6.0), (1.0, 2.0)),     # minimum inside the edge a = 4 (b = a - c)
    ((0.5, 6.0), (4.0, 9.0), (1.0, 2.0)),     # the same with a and b exchanged
    ((1.0, 1.2), (1.1, 1.3), (0.9, 1.05)),    # small box near the equilateral triangle
    ((9.0, 10.0), (0.2, 0.3), (8.0, 9.5)),    # thin triangle, cosines near +-1
    ((2.0, 50.0), (3.0, 40.0), (0.5, 60.0)),  # wide box: both clips are active
])
def test_cos_range_is_the_exact_range_over_the_box(a, b, c):
    lo, hi = omt.cos_range(a, b, c)
    glo, ghi = _cos_grid(a, b, c)
    # every grid value inside, and the ends attained to within the grid step
    assert lo <= max(glo, -1.0) + 1e-15 and hi >= min(ghi, 1.0) - 1e-15
    assert lo == pytest.approx(max(glo, -1.0), abs=2e-4)
    assert hi == pytest.approx(min(ghi, 1.0), abs=2e-4)


def _box_triple(rng, spread, width):
    c = rng.uniform(0, spread, size=(3, 3))
    w = rng.uniform(0.05, 1.0, size=(3, 3)) * width
    return c - w / 2, c + w / 2


def _dist_bounds(lo, hi):
    pairs = ((0, 1), (0, 2), (1, 2))
    dl = tuple(okd.box_min_dist(lo[u], hi[u], lo[v], hi[v]) for u, v in pairs)
    du = tuple(okd.box_max_dist(lo[u], hi[u], lo[v], hi[v]) for u, v in pairs)
    return dl, du


def test_box_max_dist_is_the_farthest_corner_pair():
    rng = workloads.rng(30)
    for _ in range(50):
        lo, hi = _box_triple(rng, 10.0, 2.0)
        corners = [np.array([(hi if (m >> d) & 1 else lo)[q][d] for d in range(3)])
                   for q in range(2) for m in range(8)]
        far = max(np.linalg.norm(corners[i] - corners[8 + j]) for i in range(8) for j in range(8))
        assert okd.box_max_dist(lo[0], hi[0], lo[1], hi[1]) == pytest.approx(far, rel=1e-14)
        p = rng.uniform(lo[0], hi[0], size=(300, 3))
        q = rng.uniform(lo[1], hi[1], size=(300, 3))
        assert np.linalg.norm(p - q, axis=1).max() <= far


@pytest.mark.parametrize("layout", ["random", "collinear", "equilateral", "close"])
def test_at_bounds_enclose_phi_of_points_in_the_boxes(layout):
    rng = workloads.rng({"random": 31, "collinear": 32, "equilateral": 33, "close": 34}[layout])
    checked = 0
    for _ in range(60):
        if layout == "random":
            lo, hi = _box_triple(rng, 12.0, rng.choice([0.02, 0.2, 1.0]))
        else:
            if layout == "collinear":  # boxes along a line: near-collinear triangles
                t = np.sort(rng.uniform(0, 10, size=3))
                c = np.outer(t, rng.normal(size=3)) + rng.normal(size=3)
            elif layout == "equilateral":
                s = rng.uniform(1, 5)
                c = np.array([[0, 0, 0], [s, 0, 0], [s / 2, s * math.sqrt(0.75), 0]])
            else:  # two boxes almost touching, the third farther
                c = np.array([[0, 0, 0], [1.0, 0, 0], rng.uniform(2, 6, size=3)])
            w = rng.uniform(0.02, 0.6, size=(3, 3))
            lo, hi = c - w / 2, c + w / 2
        dl, du = _dist_bounds(lo, hi)
        if min(dl) <= 0:
            continue
        plo, phi_ = omt.at_bounds(dl, du)
        p = [rng.uniform(lo[q], hi[q], size=(3000, 3)) for q in range(3)]
        # the box corners too, where the extremes of the distances sit
        f = omt.at_phi_np(p[0], p[1], p[2])
        assert plo <= f.min() and f.max() <= phi_
        # never looser than the envelope [-2 R, 11/8 R] at the smallest distances
        ru = 1.0 / (dl[0] * dl[1] * dl[2]) ** 3
        assert plo >= -2.0 * ru * (1 + 1e-14) and phi_ <= 1.375 * ru * (1 + 1e-14)
        checked += 1
    assert checked >= 20


def test_at_bounds_attained_for_point_boxes():
    # boxes shrunk to points: both ends equal phi of that triangle
    d = 1.7
    lo, hi = omt.at_bounds((d, d, d), (d, d, d))
    assert lo == pytest.approx(11.0 / (8.0 * d ** 9), rel=1e-14)
    assert hi == pytest.approx(11.0 / (8.0 * d ** 9), rel=1e-14)
    lo, hi = omt.at_bounds((1.0, 2.5, 1.5), (1.0, 2.5, 1.5))  # collinear 0, 1, 2.5
    assert lo == pytest.approx(-2.0 / (1.0 * 2.5 * 1.5) ** 3, rel=1e-14)
    assert hi == pytest.approx(lo, rel=1e-14)
    r = (3.0, 4.0, 5.0)  # right angle at node 1 (sides 12 = 3, 13 = 4, 23 = 5)
    lo, hi = omt.at_bounds(r, r)
    assert lo == pytest.approx(1.0 / (3.0 * 4.0 * 5.0) ** 3, rel=1e-14)
    assert hi == pytest.approx(lo, rel=1e-14)
    rng = workloads.rng(35)
    for _ in range(20):
        x = rng.normal(size=(3, 3))
        s = (np.linalg.norm(x[0] - x[1]), np.linalg.norm(x[0] - x[2]), np.linalg.norm(x[1] - x[2]))
        lo, hi = omt.at_bounds(s, s)
        f = oracle_direct.at_phi(x[0], x[1], x[2])
        assert lo == pytest.approx(f, rel=1e-9, abs=1e-12 * abs(f) + 1e-300)
        assert hi == pytest.approx(f, rel=1e-9, abs=1e-12 * abs(f) + 1e-300)


def test_at_bounds_tighten_as_the_boxes_shrink():
    # the span of the bound goes to zero with the box size (linearly), and
    # children's boxes never give a wider interval than their parent's
    rng = workloads.rng(36)
    c = rng.uniform(0, 8, size=(3, 3))
    prev = None
    for width in [2.0 ** -k for k in range(12)]:
        lo, hi = c - width / 2, c + width / 2
        plo, phi_ = omt.at_bounds(*_dist_bounds(lo, hi))
        if prev is not None:
            assert prev[0] <= plo and phi_ <= prev[1]
            if width <= 2.0 ** -4:
                assert (phi_ - plo) <= 0.6 * (prev[1] - prev[0])
        prev = (plo, phi_)
    f = oracle_direct.at_phi(c[0], c[1], c[2])
    assert prev[0] <= f <= prev[1] and (prev[1] - prev[0]) < 0.05 * abs(f)


def test_mc_try_meets_the_clt_bound():
    # One node triple of three separated leaves; every point that passes must
    # be within its error allowance with probability >= 1 - alpha (Theorem 4.1
    # applied per point, as Algorithm 4 uses it).  The allowance is set so
    # that points stop after about 100 samples, well above m_min, so that the
    # stop rule and not the sample floor decides.
    x = workloads.jittered_lattice(216, seed=13)
    t = okd.build_kdtree(x, 8)
    xs = x[t.perm]
    leaves = [v for v in range(t.n_nodes) if t.is_leaf(v)]
    p = (leaves[0], leaves[5], leaves[12])
    cnt = tuple(int(t.count[v]) for v in p)
    roles = omt.distinct_roles(p, cnt)
    r = [np.arange(t.begin[v], t.end[v]) for v in p]
    ii, jj, kk = omt.triple_index_arrays(omt.canonical_case(*p), *r)
    f = omt.at_phi_np(xs[ii], xs[jj], xs[kk])
    alpha = 0.1
    z = 1.6448536269514729  # two-sided normal quantile for alpha = 0.1
    exact, rel_sd = {}, []
    for node in p:
        for rank in range(int(t.begin[node]), int(t.end[node])):
            sel = (ii == rank) | (jj == rank) | (kk == rank)
            exact[rank] = f[sel].mean()
            rel_sd.append(f[sel].std() / abs(f[sel].mean()))
    # T_root = T_i and Phi^l = 0 make the allowance eps * |mu| per tuple
    eps = z * float(np.median(rel_sd)) / 10.0
    inside = total = 0
    for seed in range(100):
        for role in roles:
            ok, commits, _ = omt.mc_try(t, xs, p, [role], cnt, [0.0], eps, 0.0, role[1], z, seed,
                                        1024, 10)
            assert ok
            base, _, mu, _ = commits[0]
            for q, m in enumerate(mu):
                e = exact[base + q]
                total += 1
                inside += abs(m - e) <= eps * e
    frac = inside / total
    # binomial margin of 4 standard deviations below 1 - alpha
    assert frac >= 1 - alpha - 4 * math.sqrt(alpha * (1 - alpha) / total), frac


def test_two_sided_mode_exact_at_eps0_and_within_eps():
    # the two-sided statistic changes only which triples prune: eps = 0 is
    # still the exhaustive sum, and on separated clusters every point stays
    # within eps
    x = workloads.jittered_lattice(60, seed=4)
    res = omt.multitree(x, eps=0.0, alpha=0.0, leaf_size=4, bound="two_sided")
    np.testing.assert_allclose(res.phi, oracle_direct.phi(x), rtol=1e-12)
    x = blobs(24, [(0, 0, 0), (40, 0, 0), (0, 40, 0), (0, 0, 40), (40, 40, 40)], seed=11)
    eps = 0.05
    res = omt.multitree(x, eps=eps, alpha=0.0, leaf_size=4, bound="two_sided")
    rel = np.abs(res.phi - oracle_direct.phi(x)) / np.abs(oracle_direct.phi(x))
    assert res.stats["det_prunes"] > 0
    assert np.all(res.coverage == math.comb(x.shape[0] - 1, 2))
    assert rel.max() <= eps
    with pytest.raises(ValueError):
        omt.multitree(x, eps=eps, alpha=0.0, leaf_size=4, bound="magnitude")


def test_certified_reduces_to_the_paper_for_positive_bounds():
    # with every running lower bound positive (a non-negative potential) the
    # two-sided allowance is the paper's Phi^l(P) + T_i phi_lo, for the
    # deterministic interval and for a Monte Carlo interval alike
    rng = workloads.rng(41)
    for _ in range(200):
        lb = rng.uniform(0.1, 5.0, size=7)
        ub = lb + rng.uniform(0.0, 3.0, size=7)
        t = float(rng.integers(1, 1000))
        lo = rng.uniform(0.0, 1e-3)
        hi = lo + rng.uniform(0.0, 1e-3)
        stat = (lb.min(), (-ub).min(), np.maximum(lb, -ub).min())
        assert omt.certified("two_sided", stat, t, lo, hi) == omt.certified("signed", lb.min(), t, lo, hi)


def test_certified_is_a_lower_bound_on_the_new_magnitude():
    # brute force: after crediting t tuples with values in [lo, hi] to every
    # point of a node, max(LB', -UB') of every point is at least the allowance
    rng = workloads.rng(42)
    for _ in range(500):
        lb = rng.normal(size=9) * 3
        ub = lb + rng.uniform(0.0, 4.0, size=9)
        t = float(rng.integers(1, 50))
        lo = rng.normal() * 0.05
        hi = lo + rng.uniform(0.0, 0.1)
        stat = (lb.min(), (-ub).min(), np.maximum(lb, -ub).min())
        allow = omt.certified("two_sided", stat, t, lo, hi)
        for v in rng.uniform(lo, hi, size=(20, 9)):  # any credited values
            new_lb = lb + t * lo
            new_ub = ub + t * hi
            assert np.all(np.maximum(new_lb, -new_ub) >= allow - 1e-12)
            # and the exact running total, which lies between them
            tot = (lb + ub) / 2 + t * v
            assert np.all(np.abs(tot) >= allow - 1e-12) or allow <= 0
