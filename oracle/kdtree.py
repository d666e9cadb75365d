"""BuildKdTree (Algorithm 1) on the CPU - oracle side.

TEST INFRASTRUCTURE ONLY.

Follows Algorithm 1 and the text of Section 3: a node owning more points
than the leaf threshold is split along the widest dimension of its tight
bounding box; a node with at most ``leaf_size`` points is a leaf.  Points
are stored in depth-first order, so every node owns a contiguous range
[begin, end) of depth-first ranks (Section 3, the kd-tree figure).

Readings where the paper leaves a choice:
  * split value: the median by count - the left child takes the first
    floor(n/2) points in the order (coordinate along d, original index);
  * ties in the widest extent go to the lowest dimension;
  * the representative point c_P is the centroid (mean) of the node's points;
  * at expansion order p = 0 the far-field moment of a node is its count
    (Section 4).

Node numbering: the root is node 0 and nodes are numbered in pre-order
(depth-first, left before right), so a node's left child is node + 1.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class KdTree:
    perm: np.ndarray      # (N,) original index of the point at each depth-first rank
    begin: np.ndarray     # (M,) first rank owned by the node
    end: np.ndarray       # (M,) one past the last rank
    left: np.ndarray      # (M,) left child, -1 for a leaf
    right: np.ndarray     # (M,) right child, -1 for a leaf
    parent: np.ndarray    # (M,) parent, -1 for the root
    depth: np.ndarray     # (M,)
    lo: np.ndarray        # (M, 3) tight bounding box, lower corner
    hi: np.ndarray        # (M, 3) tight bounding box, upper corner
    centroid: np.ndarray  # (M, 3)
    leaf_size: int

    @property
    def count(self) -> np.ndarray:
        return self.end - self.begin

    def is_leaf(self, node: int) -> bool:
        return self.left[node] < 0

    @property
    def n_nodes(self) -> int:
        return int(self.begin.shape[0])


def build_kdtree(x: np.ndarray, leaf_size: int) -> KdTree:
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    if leaf_size < 1:
        raise ValueError("leaf_size must be >= 1")
    perm = np.arange(n, dtype=np.int64)
    nodes: list[dict] = []

    def rec(b: int, e: int, parent: int, depth: int) -> int:
        me = len(nodes)
        pts = x[perm[b:e]]
        lo = pts.min(axis=0) if e > b else np.zeros(3)
        hi = pts.max(axis=0) if e > b else np.zeros(3)
        cen = pts.mean(axis=0) if e > b else np.zeros(3)
        nodes.append(dict(begin=b, end=e, left=-1, right=-1, parent=parent, depth=depth,
                          lo=lo, hi=hi, centroid=cen))
        if e - b > leaf_size:
            ext = hi - lo
            d = int(np.argmax(ext))  # first maximum: ties go to the lowest dimension
            seg = perm[b:e]
            order = np.lexsort((seg, x[seg, d]))  # primary: coordinate, then original index
            perm[b:e] = seg[order]
            mid = b + (e - b) // 2
            nodes[me]["left"] = rec(b, mid, me, depth + 1)
            nodes[me]["right"] = rec(mid, e, me, depth + 1)
        return me

    rec(0, n, -1, 0)
    m = len(nodes)
    return KdTree(
        perm=perm,
        begin=np.array([v["begin"] for v in nodes], dtype=np.int64),
        end=np.array([v["end"] for v in nodes], dtype=np.int64),
        left=np.array([v["left"] for v in nodes], dtype=np.int64),
        right=np.array([v["right"] for v in nodes], dtype=np.int64),
        parent=np.array([v["parent"] for v in nodes], dtype=np.int64),
        depth=np.array([v["depth"] for v in nodes], dtype=np.int64),
        lo=np.array([v["lo"] for v in nodes]).reshape(m, 3),
        hi=np.array([v["hi"] for v in nodes]).reshape(m, 3),
        centroid=np.array([v["centroid"] for v in nodes]).reshape(m, 3),
        leaf_size=leaf_size,
    )


def box_min_dist(lo1, hi1, lo2, hi2) -> float:
    """d^l: smallest distance between two axis-aligned boxes (Section 3, distance-bound figure)."""
    gap = np.maximum(0.0, np.maximum(np.asarray(lo1) - hi2, np.asarray(lo2) - hi1))
    return float(np.sqrt(gap @ gap))


def box_max_dist(lo1, hi1, lo2, hi2) -> float:
    """d^u: largest distance between two axis-aligned boxes."""
    span = np.maximum(np.abs(np.asarray(hi2) - lo1), np.abs(np.asarray(hi1) - lo2))
    return float(np.sqrt(span @ span))
