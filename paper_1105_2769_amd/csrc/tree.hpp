// The kd-tree of BuildKdTree (Algorithm 1) as kept on the device.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "mb_internal.hpp"

namespace mb {

// Nodes are numbered in pre-order (depth first, left child = node + 1), and
// a node owns the depth-first ranks [begin, end) (Section 3).
struct TreeHost {
    int64_t n = 0;
    int leaf_size = 0;
    int n_nodes = 0;
    int max_depth = 0;
    std::vector<int32_t> begin, end, left, right, parent, depth;
    std::vector<std::vector<int32_t>> internal_at;  // internal nodes per depth
    std::vector<std::vector<int32_t>> nodes_at;     // all nodes per depth
};

struct DeviceTree {
    TreeHost h;
    int device = 0;
    // device arrays (owned)
    int32_t *perm = nullptr;       // original index of the point at each rank
    double *xs = nullptr;          // points in rank order, 3 per point
    int32_t *begin = nullptr, *end = nullptr, *left = nullptr, *right = nullptr,
            *parent = nullptr;
    int32_t *leaf_of = nullptr;    // leaf node of each rank
    int32_t *depth_nodes = nullptr;  // node ids grouped by depth (for level passes)
    std::vector<int> depth_off;      // offsets into depth_nodes, max_depth + 2 entries
    double *lo = nullptr, *hi = nullptr, *centroid = nullptr;  // 3 per node
    double build_ms = 0.0;
};

// Host topology from the counts alone: a node with more than leaf_size
// points is split into floor(n/2) + ceil(n/2).
TreeHost tree_topology(int64_t n, int leaf_size);

mb_status tree_build(const double *x, int64_t n, int leaf_size, hipStream_t s, DeviceTree **out);
void tree_free(DeviceTree *t);

// Factorized (matrix-product) evaluation over the points of a tree, in
// the tree's depth-first order; phi receives input order.
//   fmt: 0 = FP16, 1 = BF16; planes: 1..3.
mb_status factorized_eval(const DeviceTree *tr, int n, int fmt, int planes, double r_near,
                          double *phi, hipStream_t s, FactorStats *stats);

// Mean diagonal of the leaf bounding boxes (waits on s).
double tree_mean_leaf_diagonal(const DeviceTree *t, hipStream_t s);

}  // namespace mb
