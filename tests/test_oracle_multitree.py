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


def test_det_bounds_enclose_and_are_attained():
    # points drawn in three separated boxes stay inside [phi_lo, phi_lo + span]
    rng = workloads.rng(31)
    for _ in range(40):
        c = rng.uniform(0, 12, size=(3, 3))
        w = rng.uniform(0.05, 1.0, size=(3, 3))
        lo, hi = c - w / 2, c + w / 2
        d12 = okd.box_min_dist(lo[0], hi[0], lo[1], hi[1])
        d13 = okd.box_min_dist(lo[0], hi[0], lo[2], hi[2])
        d23 = okd.box_min_dist(lo[1], hi[1], lo[2], hi[2])
        if min(d12, d13, d23) <= 0:
            continue
        plo, span = omt.det_bounds(d12, d13, d23)
        p = [rng.uniform(lo[q], hi[q], size=(500, 3)) for q in range(3)]
        f = omt.at_phi_np(p[0], p[1], p[2])
        assert f.min() >= plo and f.max() <= plo + span
    # degenerate boxes: equilateral triangle attains the top, collinear the bottom
    s = math.sqrt(3.0) / 2.0
    tri = np.array([[0.0, 0, 0], [2.0, 0, 0], [1.0, 2 * s, 0]])
    plo, span = omt.det_bounds(2.0, 2.0, 2.0)
    assert omt.at_phi_np(tri[0], tri[1], tri[2]) == pytest.approx(plo + span, rel=1e-14)
    line = np.array([[0.0, 0, 0], [1.0, 0, 0], [2.5, 0, 0]])
    plo, _ = omt.det_bounds(1.0, 2.5, 1.5)
    assert omt.at_phi_np(line[0], line[1], line[2]) == pytest.approx(plo, rel=1e-14)


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


def test_magnitude_mode_exact_at_eps0_and_within_eps():
    # the magnitude reading changes only which triples prune: eps = 0 is still
    # the exhaustive sum, and on five separated clusters every point stays
    # within eps
    x = workloads.jittered_lattice(60, seed=4)
    res = omt.multitree(x, eps=0.0, alpha=0.0, leaf_size=4, bound="magnitude")
    np.testing.assert_allclose(res.phi, oracle_direct.phi(x), rtol=1e-12)
    x = blobs(24, [(0, 0, 0), (40, 0, 0), (0, 40, 0), (0, 0, 40), (40, 40, 40)], seed=11)
    eps = 0.05
    res = omt.multitree(x, eps=eps, alpha=0.0, leaf_size=4, bound="magnitude")
    rel = np.abs(res.phi - oracle_direct.phi(x)) / np.abs(oracle_direct.phi(x))
    assert res.stats["det_prunes"] > 0
    assert np.all(res.coverage == math.comb(x.shape[0] - 1, 2))
    assert rel.max() <= eps
    with pytest.raises(ValueError):
        omt.multitree(x, eps=eps, alpha=0.0, leaf_size=4, bound="other")
