// BuildKdTree (Algorithm 1) on gfx950.
//
// A node with more than leaf_size points is split along the widest
// dimension of its tight bounding box; the left child takes the first
// floor(n/2) points in the order (coordinate, original index), i.e. the
// split is the median by count (the paper's "two equal halves").  Because
// the split is by count, the node ranges depend on N alone and the host
// builds the topology; the device decides which points fall where.
//
// Device steps:
//   1. per dimension, the rank of every point in the order (coordinate,
//      index), from one stable radix sort of the coordinate keys (these
//      ranks are unique, so ordering a node by rank is ordering it by
//      (coordinate, index));
//   2. per depth: bounding box and widest dimension of each internal node,
//      then one radix sort of all ranks keyed (segment start, rank along the
//      segment's split dimension) - segments of finished leaves are keyed by
//      position and keep their order;
//   3. final bounding box and centroid of every node; points gathered in
//      rank (depth-first) order.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <cmath>
#include <functional>

#include "tree.hpp"

namespace mb {
namespace {

__device__ __forceinline__ unsigned long long coord_key(double d) {
    unsigned long long b = (unsigned long long)__double_as_longlong(d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ void coord_key_kernel(const double *__restrict__ x, int n, int d,
                                 unsigned long long *__restrict__ keys, int32_t *__restrict__ vals) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) {
        keys[p] = coord_key(x[3 * (int64_t)p + d]);
        vals[p] = p;
    }
}

__global__ void rank_scatter_kernel(const int32_t *__restrict__ sorted, int n,
                                    int32_t *__restrict__ rank) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) rank[sorted[r]] = r;
}

__global__ void iota_kernel(int32_t *__restrict__ a, int n, int32_t v0) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) a[r] = v0 + r;
}

__global__ void fill_i32_kernel(int32_t *__restrict__ a, int n, int32_t v) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) a[r] = v;
}

constexpr int kBT = 256;

// Bounding box (and, if want_dim, the widest dimension) of each listed node.
// With want_centroid, also the mean of its points.  One workgroup per node.
__global__ __launch_bounds__(kBT) void node_box_kernel(
    const int32_t *__restrict__ nodes, const int32_t *__restrict__ begin,
    const int32_t *__restrict__ end, const int32_t *__restrict__ perm,
    const double *__restrict__ x, double *__restrict__ lo, double *__restrict__ hi,
    double *__restrict__ centroid, int32_t *__restrict__ split_dim) {
    const int node = nodes[blockIdx.x];
    const int b = begin[node], e = end[node];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY},
           sm[3] = {0.0, 0.0, 0.0};
    for (int r = b + threadIdx.x; r < e; r += kBT) {
        const int64_t p = perm[r];
        for (int c = 0; c < 3; ++c) {
            const double v = x[3 * p + c];
            mn[c] = fmin(mn[c], v);
            mx[c] = fmax(mx[c], v);
            sm[c] += v;
        }
    }
    __shared__ double red[9][kBT];
    for (int c = 0; c < 3; ++c) {
        red[c][threadIdx.x] = mn[c];
        red[3 + c][threadIdx.x] = mx[c];
        red[6 + c][threadIdx.x] = sm[c];
    }
    __syncthreads();
    for (int w = kBT / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 3; ++c) {
                red[c][threadIdx.x] = fmin(red[c][threadIdx.x], red[c][threadIdx.x + w]);
                red[3 + c][threadIdx.x] = fmax(red[3 + c][threadIdx.x], red[3 + c][threadIdx.x + w]);
                red[6 + c][threadIdx.x] += red[6 + c][threadIdx.x + w];
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) {
            lo[3 * node + c] = red[c][0];
            hi[3 * node + c] = red[3 + c][0];
            if (centroid) centroid[3 * node + c] = red[6 + c][0] / (double)(e - b);
        }
        if (split_dim) {
            // widest extent, ties to the lowest dimension
            int d = 0;
            double w = red[3][0] - red[0][0];
            for (int c = 1; c < 3; ++c) {
                const double wc = red[3 + c][0] - red[c][0];
                if (wc > w) {
                    w = wc;
                    d = c;
                }
            }
            split_dim[node] = d;
        }
    }
}

// Sort keys for one depth: (segment start, rank along the split dimension)
// inside nodes being split at this depth, (segment start, position) elsewhere.
__global__ void seg_key_kernel(int n, int depth, const int32_t *__restrict__ owner,
                               const int32_t *__restrict__ node_depth,
                               const int32_t *__restrict__ left, const int32_t *__restrict__ begin,
                               const int32_t *__restrict__ split_dim,
                               const int32_t *__restrict__ rank, const int32_t *__restrict__ perm,
                               unsigned long long *__restrict__ keys) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int node = owner[r];
    const unsigned long long seg = (unsigned long long)(uint32_t)begin[node] << 32;
    if (node_depth[node] == depth && left[node] >= 0) {
        const int d = split_dim[node];
        keys[r] = seg | (uint32_t)rank[(int64_t)d * n + perm[r]];
    } else {
        keys[r] = seg | (uint32_t)r;
    }
}

// After the split at this depth, ranks move to the child that owns them.
__global__ void owner_update_kernel(int n, int depth, int32_t *__restrict__ owner,
                                    const int32_t *__restrict__ node_depth,
                                    const int32_t *__restrict__ left,
                                    const int32_t *__restrict__ right,
                                    const int32_t *__restrict__ begin) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int node = owner[r];
    if (node_depth[node] == depth && left[node] >= 0)
        owner[r] = r < begin[right[node]] ? left[node] : right[node];
}

__global__ void gather_points_kernel(const double *__restrict__ x, const int32_t *__restrict__ perm,
                                     int n, double *__restrict__ xs) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) {
        const int64_t p = perm[r];
        xs[3 * (int64_t)r + 0] = x[3 * p + 0];
        xs[3 * (int64_t)r + 1] = x[3 * p + 1];
        xs[3 * (int64_t)r + 2] = x[3 * p + 2];
    }
}

unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T>
mb_status dev_alloc(T **p, size_t count) {
    hipError_t e = hipMalloc((void **)p, sizeof(T) * (count ? count : 1));
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_fail(e, "hipMalloc (tree)");
    }
    return MB_OK;
}

}  // namespace

TreeHost tree_topology(int64_t n, int leaf_size) {
    TreeHost h;
    h.n = n;
    h.leaf_size = leaf_size;
    std::function<int(int64_t, int64_t, int, int)> rec = [&](int64_t b, int64_t e, int par,
                                                            int dep) -> int {
        const int me = (int)h.begin.size();
        h.begin.push_back((int32_t)b);
        h.end.push_back((int32_t)e);
        h.left.push_back(-1);
        h.right.push_back(-1);
        h.parent.push_back(par);
        h.depth.push_back(dep);
        h.max_depth = std::max(h.max_depth, dep);
        if (e - b > leaf_size) {
            const int64_t mid = b + (e - b) / 2;
            const int l = rec(b, mid, me, dep + 1);
            h.left[me] = l;
            const int r = rec(mid, e, me, dep + 1);
            h.right[me] = r;
        }
        return me;
    };
    rec(0, n, -1, 0);
    h.n_nodes = (int)h.begin.size();
    h.internal_at.assign(h.max_depth + 1, {});
    h.nodes_at.assign(h.max_depth + 1, {});
    for (int v = 0; v < h.n_nodes; ++v) {
        h.nodes_at[h.depth[v]].push_back(v);
        if (h.left[v] >= 0) h.internal_at[h.depth[v]].push_back(v);
    }
    return h;
}

void tree_free(DeviceTree *t) {
    if (!t) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(t->device);
    for (void *p : {(void *)t->perm, (void *)t->xs, (void *)t->begin, (void *)t->end,
                    (void *)t->left, (void *)t->right, (void *)t->parent, (void *)t->leaf_of,
                    (void *)t->depth_nodes, (void *)t->lo, (void *)t->hi, (void *)t->centroid})
        if (p) (void)hipFree(p);
    (void)hipSetDevice(prev);
    delete t;
}

mb_status tree_build(const double *x, int64_t n64, int leaf_size, hipStream_t s,
                     DeviceTree **out) {
    auto t0 = std::chrono::steady_clock::now();
    const int n = (int)n64;
    DeviceTree *t = new DeviceTree();
    t->h = tree_topology(n64, leaf_size);
    (void)hipGetDevice(&t->device);
    const TreeHost &h = t->h;
    const int M = h.n_nodes;
    mb_status st;
    auto fail_free = [&](mb_status e) {
        tree_free(t);
        return e;
    };
    if ((st = dev_alloc(&t->perm, n)) != MB_OK || (st = dev_alloc(&t->xs, 3 * (size_t)n)) != MB_OK ||
        (st = dev_alloc(&t->begin, M)) != MB_OK || (st = dev_alloc(&t->end, M)) != MB_OK ||
        (st = dev_alloc(&t->left, M)) != MB_OK || (st = dev_alloc(&t->right, M)) != MB_OK ||
        (st = dev_alloc(&t->parent, M)) != MB_OK || (st = dev_alloc(&t->leaf_of, n)) != MB_OK ||
        (st = dev_alloc(&t->depth_nodes, M)) != MB_OK || (st = dev_alloc(&t->lo, 3 * (size_t)M)) != MB_OK ||
        (st = dev_alloc(&t->hi, 3 * (size_t)M)) != MB_OK ||
        (st = dev_alloc(&t->centroid, 3 * (size_t)M)) != MB_OK)
        return fail_free(st);

    // topology upload (synchronous copies from host vectors)
    std::vector<int32_t> dn;
    t->depth_off.assign(h.max_depth + 2, 0);
    for (int d = 0; d <= h.max_depth; ++d) {
        t->depth_off[d] = (int)dn.size();
        dn.insert(dn.end(), h.nodes_at[d].begin(), h.nodes_at[d].end());
    }
    t->depth_off[h.max_depth + 1] = (int)dn.size();
    std::vector<int32_t> hdepth(h.depth.begin(), h.depth.end());
    auto up = [&](int32_t *dst, const std::vector<int32_t> &src) {
        return hipMemcpyAsync(dst, src.data(), sizeof(int32_t) * src.size(), hipMemcpyHostToDevice, s);
    };
    MB_HIP(up(t->begin, h.begin));
    MB_HIP(up(t->end, h.end));
    MB_HIP(up(t->left, h.left));
    MB_HIP(up(t->right, h.right));
    MB_HIP(up(t->parent, h.parent));
    MB_HIP(up(t->depth_nodes, dn));

    // scratch: depth of each node, split dims, owner, ranks, sort buffers
    Scratch s_depth, s_dim, s_owner, s_rank, s_keys, s_keys2, s_vals2, s_tmp, s_lists;
    if ((st = s_depth.alloc(sizeof(int32_t) * M, s)) != MB_OK ||
        (st = s_dim.alloc(sizeof(int32_t) * M, s)) != MB_OK ||
        (st = s_owner.alloc(sizeof(int32_t) * n, s)) != MB_OK ||
        (st = s_rank.alloc(sizeof(int32_t) * 3 * (size_t)n, s)) != MB_OK ||
        (st = s_keys.alloc(sizeof(unsigned long long) * n, s)) != MB_OK ||
        (st = s_keys2.alloc(sizeof(unsigned long long) * n, s)) != MB_OK ||
        (st = s_vals2.alloc(sizeof(int32_t) * n, s)) != MB_OK ||
        (st = s_lists.alloc(sizeof(int32_t) * M, s)) != MB_OK)
        return fail_free(st);
    MB_HIP(up(s_depth.as<int32_t>(), hdepth));
    unsigned long long *keys = s_keys.as<unsigned long long>();
    unsigned long long *keys2 = s_keys2.as<unsigned long long>();
    int32_t *vals2 = s_vals2.as<int32_t>();
    int32_t *rank = s_rank.as<int32_t>();

    size_t tmp_bytes = 0;
    MB_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, keys, keys2, t->perm, vals2, n, 0,
                                              64, s));
    if ((st = s_tmp.alloc(tmp_bytes, s)) != MB_OK) return fail_free(st);

    const unsigned nb = blocks_for(n, 256);
    // 1. ranks along each dimension (stable: ties keep index order)
    for (int d = 0; d < 3; ++d) {
        coord_key_kernel<<<nb, 256, 0, s>>>(x, n, d, keys, t->perm);
        MB_HIP(hipcub::DeviceRadixSort::SortPairs(s_tmp.ptr, tmp_bytes, keys, keys2, t->perm, vals2,
                                                  n, 0, 64, s));
        rank_scatter_kernel<<<nb, 256, 0, s>>>(vals2, n, rank + (size_t)d * n);
    }
    // 2. depth by depth
    iota_kernel<<<nb, 256, 0, s>>>(t->perm, n, 0);
    fill_i32_kernel<<<nb, 256, 0, s>>>(s_owner.as<int32_t>(), n, 0);
    int pos_bits = 1;
    while ((1ll << pos_bits) < (int64_t)n) ++pos_bits;
    for (int d = 0; d < h.max_depth; ++d) {
        const std::vector<int32_t> &lst = h.internal_at[d];
        if (lst.empty()) continue;
        MB_HIP(up(s_lists.as<int32_t>(), lst));
        node_box_kernel<<<(unsigned)lst.size(), kBT, 0, s>>>(s_lists.as<int32_t>(), t->begin, t->end,
                                                            t->perm, x, t->lo, t->hi, nullptr,
                                                            s_dim.as<int32_t>());
        seg_key_kernel<<<nb, 256, 0, s>>>(n, d, s_owner.as<int32_t>(), s_depth.as<int32_t>(),
                                          t->left, t->begin, s_dim.as<int32_t>(), rank, t->perm,
                                          keys);
        MB_HIP(hipcub::DeviceRadixSort::SortPairs(s_tmp.ptr, tmp_bytes, keys, keys2, t->perm, vals2,
                                                  n, 0, 32 + pos_bits, s));
        MB_HIP(hipMemcpyAsync(t->perm, vals2, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        owner_update_kernel<<<nb, 256, 0, s>>>(n, d, s_owner.as<int32_t>(), s_depth.as<int32_t>(),
                                               t->left, t->right, t->begin);
        // the list buffer is reused by the next depth: keep the upload ordered
        MB_HIP(hipStreamSynchronize(s));
    }
    // 3. final node statistics, rank-ordered points, leaf of each rank
    node_box_kernel<<<(unsigned)M, kBT, 0, s>>>(t->depth_nodes, t->begin, t->end, t->perm, x, t->lo,
                                                t->hi, t->centroid, nullptr);
    gather_points_kernel<<<nb, 256, 0, s>>>(x, t->perm, n, t->xs);
    MB_HIP(hipMemcpyAsync(t->leaf_of, s_owner.ptr, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    MB_HIP(hipGetLastError());
    MB_HIP(hipStreamSynchronize(s));
    t->build_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = t;
    return MB_OK;
}

double tree_mean_leaf_diagonal(const DeviceTree *t, hipStream_t s) {
    const int M = t->h.n_nodes;
    std::vector<double> lo(3 * (size_t)M), hi(3 * (size_t)M);
    if (hipMemcpyAsync(lo.data(), t->lo, sizeof(double) * 3 * M, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipMemcpyAsync(hi.data(), t->hi, sizeof(double) * 3 * M, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return 0.0;
    double sum = 0.0;
    int cnt = 0;
    for (int v = 0; v < M; ++v)
        if (t->h.left[v] < 0) {
            double d2 = 0.0;
            for (int c = 0; c < 3; ++c) d2 += (hi[3 * v + c] - lo[3 * v + c]) * (hi[3 * v + c] - lo[3 * v + c]);
            sum += std::sqrt(d2);
            ++cnt;
        }
    return cnt ? sum / cnt : 0.0;
}

}  // namespace mb
