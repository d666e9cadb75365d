// C ABI entry points (declared in include/mb.h): argument checks, the
// validation step and dispatch to the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mb_internal.hpp"
#include "multitree.hpp"
#include "tree.hpp"

namespace mb {

namespace {
thread_local std::string g_last_error;
}

mb_status fail(mb_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

void clear_error() { g_last_error.clear(); }

const char *last_error_cstr() { return g_last_error.c_str(); }

mb_status hip_fail(hipError_t e, const char *what) {
    std::string msg = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return fail(MB_ERR_OOM, msg);
    return fail(MB_ERR_DEVICE, msg);
}

size_t table_budget_bytes() {
    static const size_t v = [] {
        const char *e = std::getenv("MB_TABLE_BUDGET_MB");
        long mb = e ? std::atol(e) : 32768;
        if (mb < 1) mb = 1;
        return (size_t)mb << 20;
    }();
    return v;
}

void device_pool_setup() {
    static std::mutex mu;
    static bool done[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
    std::lock_guard<std::mutex> lock(mu);
    if (done[dev]) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    done[dev] = true;
}

mb_status check_points(const double *x, int64_t n, hipStream_t s, ValidateOut *v) {
    mb_status st = validate_points(x, n, s, v);
    if (st != MB_OK) return st;
    if (v->nonfinite) return fail(MB_ERR_INVALID, "non-finite coordinate");
    if (n >= 3) {
        double md2;
        static_assert(sizeof md2 == sizeof v->min_d2_bits, "bits");
        std::memcpy(&md2, &v->min_d2_bits, sizeof md2);
        if (!(md2 > 0.0)) return fail(MB_ERR_DEGENERATE, "two points coincide");
    }
    return MB_OK;
}

bool fp32c_suitable(const ValidateOut &v, int64_t n) {
    double md2;
    std::memcpy(&md2, &v.min_d2_bits, sizeof md2);
    double diag2 = 0.0;
    for (int c = 0; c < 3; ++c) diag2 += (v.hi[c] - v.lo[c]) * (v.hi[c] - v.lo[c]);
    if (diag2 > kFp32MaxRatio * kFp32MaxRatio * md2) return false;
    const double floor_ext = 1e-3 * std::sqrt(diag2);
    double vol = 1.0;
    for (int c = 0; c < 3; ++c) vol *= std::max(v.hi[c] - v.lo[c], floor_ext);
    const double spacing = std::cbrt(vol / (double)std::max<int64_t>(n, 1));
    return 16.0 * md2 >= spacing * spacing;  // closest pair >= spacing / 4
}

double unit_scale(double min_d2) {
    int e;
    std::frexp(std::sqrt(min_d2), &e);  // r = f * 2^e, f in [0.5, 1)
    return std::ldexp(1.0, 1 - e);
}

}  // namespace mb

using namespace mb;

extern "C" {

const char *mb_last_error(void) { return last_error_cstr(); }

int32_t mb_version(void) { return 100; }

mb_status mb_trim(void *stream, int64_t *released) {
    clear_error();
    if (released) *released = 0;
    MB_HIP(hipStreamSynchronize((hipStream_t)stream));
    int dev = 0;
    MB_HIP(hipGetDevice(&dev));
    hipMemPool_t pool;
    MB_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
    uint64_t before = 0, after = 0;
    MB_HIP(hipMemPoolGetAttribute(pool, hipMemPoolAttrReservedMemCurrent, &before));
    MB_HIP(hipMemPoolTrimTo(pool, 0));
    MB_HIP(hipMemPoolGetAttribute(pool, hipMemPoolAttrReservedMemCurrent, &after));
    if (released) *released = before > after ? (int64_t)(before - after) : 0;
    return MB_OK;
}

mb_status mb_validate(const double *x, int64_t n, double *min_d2, int32_t *finite, double *bbox,
                      void *stream) {
    clear_error();
    if (n < 0 || (n > 0 && !x) || !min_d2 || !finite) return fail(MB_ERR_INVALID, "bad argument");
    if (n >= ((int64_t)1 << 31)) return fail(MB_ERR_UNSUPPORTED, "n must be < 2^31");
    ValidateOut v{};
    mb_status st = validate_points(x, n, (hipStream_t)stream, &v);
    if (st != MB_OK) return st;
    std::memcpy(min_d2, &v.min_d2_bits, sizeof(double));
    *finite = v.nonfinite ? 0 : 1;
    if (bbox)
        for (int c = 0; c < 3; ++c) {
            bbox[c] = v.lo[c];
            bbox[3 + c] = v.hi[c];
        }
    return MB_OK;
}

mb_status mb_eval_direct(const double *x, int64_t n, int32_t prec, double *phi, void *stream) {
    clear_error();
    if (n < 0) return fail(MB_ERR_INVALID, "n < 0");
    if (n > 0 && (!x || !phi)) return fail(MB_ERR_INVALID, "null pointer");
    if (prec != MB_FP64 && prec != MB_FP32C) return fail(MB_ERR_INVALID, "unknown precision");
    if (n >= ((int64_t)1 << 31)) return fail(MB_ERR_UNSUPPORTED, "n must be < 2^31");
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return MB_OK;
    ValidateOut v{};
    mb_status st = check_points(x, n, s, &v);
    if (st != MB_OK) return st;
    if (n < 3) return zero_doubles(phi, n, s);
    double scale = 1.0, r_fix = 0.0;
    int p = prec;
    if (p == MB_FP32C) {
        double md2;
        std::memcpy(&md2, &v.min_d2_bits, sizeof md2);
        if (!fp32c_suitable(v, n)) {
            p = MB_FP64;  // too wide a range or too close a pair for binary32 tiles
        } else {
            scale = unit_scale(md2);
            r_fix = kNearFixFactor * std::sqrt(md2);
        }
    }
    return direct_launch(x, n, p, scale, phi, s, r_fix);
}

mb_status mb_eval_direct_deterministic(const double *x, int64_t n, double *phi,
                                       int64_t scratch_bytes, void *stream) {
    clear_error();
    if (n < 0) return fail(MB_ERR_INVALID, "n < 0");
    if (n > 0 && (!x || !phi)) return fail(MB_ERR_INVALID, "null pointer");
    if (n >= ((int64_t)1 << 31)) return fail(MB_ERR_UNSUPPORTED, "n must be < 2^31");
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return MB_OK;
    ValidateOut v{};
    mb_status st = check_points(x, n, s, &v);
    if (st != MB_OK) return st;
    const size_t budget = scratch_bytes > 0 ? (size_t)scratch_bytes : table_budget_bytes();
    return direct_launch_ordered(x, n, phi, budget, s);
}

mb_status mb_eval_direct_unchecked(const double *x, int64_t n, int32_t prec, double *phi,
                                   void *stream) {
    clear_error();
    if (n < 0) return fail(MB_ERR_INVALID, "n < 0");
    if (n > 0 && (!x || !phi)) return fail(MB_ERR_INVALID, "null pointer");
    if (prec != MB_FP64 && prec != MB_FP32C) return fail(MB_ERR_INVALID, "unknown precision");
    if (n >= ((int64_t)1 << 31)) return fail(MB_ERR_UNSUPPORTED, "n must be < 2^31");
    if (n == 0) return MB_OK;
    return direct_launch(x, n, prec, 1.0, phi, (hipStream_t)stream);
}

mb_status mb_eval_direct_noalloc(const double *x, int64_t n, int32_t prec, double *phi,
                                 void *stream) {
    clear_error();
    if (n < 0) return fail(MB_ERR_INVALID, "n < 0");
    if (n > 0 && (!x || !phi)) return fail(MB_ERR_INVALID, "null pointer");
    if (prec != MB_FP64 && prec != MB_FP32C) return fail(MB_ERR_INVALID, "unknown precision");
    if (n > kNoAllocMaxN) return fail(MB_ERR_UNSUPPORTED, "n above 1024 for mb_eval_direct_noalloc");
    if (n == 0) return MB_OK;
    return direct_launch_noalloc(x, n, prec, phi, (hipStream_t)stream);
}

mb_status mb_build_kdtree(const double *x, int64_t n, int32_t leaf_size, void *stream,
                          mb_tree *out) {
    clear_error();
    if (!out) return fail(MB_ERR_INVALID, "null output");
    *out = nullptr;
    if (n < 0 || (n > 0 && !x)) return fail(MB_ERR_INVALID, "bad points");
    if (leaf_size < 1) return fail(MB_ERR_INVALID, "leaf_size < 1");
    if (leaf_size > 32) return fail(MB_ERR_UNSUPPORTED, "leaf_size > 32");
    if (n >= ((int64_t)1 << 31)) return fail(MB_ERR_UNSUPPORTED, "n must be < 2^31");
    hipStream_t s = (hipStream_t)stream;
    ValidateOut v{};
    mb_status st = check_points(x, n, s, &v);
    if (st != MB_OK) return st;
    DeviceTree *t = nullptr;
    if ((st = tree_build(x, n, leaf_size, s, &t)) != MB_OK) return st;
    *out = reinterpret_cast<mb_tree>(t);
    return MB_OK;
}

mb_status mb_free_kdtree(mb_tree t) {
    tree_free(reinterpret_cast<DeviceTree *>(t));
    return MB_OK;
}

mb_status mb_kdtree_info(mb_tree tt, int64_t *n_points, int32_t *n_nodes, int32_t *max_depth,
                         double *build_ms) {
    clear_error();
    const DeviceTree *t = reinterpret_cast<const DeviceTree *>(tt);
    if (!t) return fail(MB_ERR_INVALID, "null tree");
    if (n_points) *n_points = t->h.n;
    if (n_nodes) *n_nodes = t->h.n_nodes;
    if (max_depth) *max_depth = t->h.max_depth;
    if (build_ms) *build_ms = t->build_ms;
    return MB_OK;
}

mb_status mb_kdtree_export(mb_tree tt, int32_t *perm, int32_t *ranges, int32_t *children,
                           double *bbox, double *centroid) {
    clear_error();
    const DeviceTree *t = reinterpret_cast<const DeviceTree *>(tt);
    if (!t) return fail(MB_ERR_INVALID, "null tree");
    const int M = t->h.n_nodes;
    if (perm && t->h.n > 0)
        MB_HIP(hipMemcpy(perm, t->perm, sizeof(int32_t) * t->h.n, hipMemcpyDeviceToHost));
    if (ranges)
        for (int v = 0; v < M; ++v) {
            ranges[2 * v] = t->h.begin[v];
            ranges[2 * v + 1] = t->h.end[v];
        }
    if (children)
        for (int v = 0; v < M; ++v) {
            children[2 * v] = t->h.left[v];
            children[2 * v + 1] = t->h.right[v];
        }
    if (bbox) {
        std::vector<double> lo(3 * (size_t)M), hi(3 * (size_t)M);
        MB_HIP(hipMemcpy(lo.data(), t->lo, sizeof(double) * 3 * M, hipMemcpyDeviceToHost));
        MB_HIP(hipMemcpy(hi.data(), t->hi, sizeof(double) * 3 * M, hipMemcpyDeviceToHost));
        for (int v = 0; v < M; ++v)
            for (int c = 0; c < 3; ++c) {
                bbox[6 * v + c] = lo[3 * v + c];
                bbox[6 * v + 3 + c] = hi[3 * v + c];
            }
    }
    if (centroid && M > 0)
        MB_HIP(hipMemcpy(centroid, t->centroid, sizeof(double) * 3 * M, hipMemcpyDeviceToHost));
    return MB_OK;
}

void mb_mt_params_default(mb_mt_params *p) {
    if (!p) return;
    p->eps_rel = 1e-2;
    p->tau_abs = 0.0;
    p->alpha = 0.05;
    p->m_limit = 128;
    p->m_min = 30;
    p->zeta = 128.0;
    p->seed = 0;
    p->base_prec = MB_FP32C;
    p->chunk = 1 << 20;  // fewer rounds: each round ends in a host wait for the stack size
    p->bound = MB_BOUND_SIGNED;
    p->order = 0;
}

mb_status mb_eval_multitree(const double *x, int64_t n, int32_t leaf_size,
                            const mb_mt_params *params, mb_tree tree, double *phi,
                            int64_t *coverage, mb_mt_stats *stats, void *stream) {
    clear_error();
    mb_mt_params p;
    if (params) p = *params; else mb_mt_params_default(&p);
    if (n < 0 || (n > 0 && (!x || !phi))) return fail(MB_ERR_INVALID, "bad points or output");
    if (!(p.eps_rel >= 0.0) || !(p.tau_abs >= 0.0) || !(p.alpha >= 0.0 && p.alpha < 1.0) ||
        p.m_limit < 2 || p.m_min < 2 || !(p.zeta >= 0.0) || p.chunk < 1 ||
        (p.bound != MB_BOUND_SIGNED && p.bound != MB_BOUND_TWO_SIDED) || p.order < 0 ||
        p.order > 2 ||
        (p.base_prec != MB_FP64 && p.base_prec != MB_FP32C))
        return fail(MB_ERR_INVALID, "bad traversal parameters");
    if (n >= ((int64_t)1 << 31)) return fail(MB_ERR_UNSUPPORTED, "n must be < 2^31");
    hipStream_t s = (hipStream_t)stream;
    if (stats) *stats = mb_mt_stats{};
    if (n == 0) return MB_OK;
    ValidateOut v{};
    mb_status st = check_points(x, n, s, &v);
    if (st != MB_OK) return st;
    DeviceTree *t = reinterpret_cast<DeviceTree *>(tree);
    DeviceTree *own = nullptr;
    if (t) {
        if (t->h.n != n) return fail(MB_ERR_INVALID, "tree built for a different point count");
        bool same = false;
        if ((st = tree_matches_points(t, x, n, s, &same)) != MB_OK) return st;
        if (!same) return fail(MB_ERR_INVALID, "tree built for other points");
    } else {
        if (leaf_size < 1) return fail(MB_ERR_INVALID, "leaf_size < 1");
        if (leaf_size > 32) return fail(MB_ERR_UNSUPPORTED, "leaf_size > 32");
        if ((st = tree_build(x, n, leaf_size, s, &own)) != MB_OK) return st;
        t = own;
    }
    MtParams mp;
    mp.eps = p.eps_rel;
    mp.tau = p.tau_abs;
    mp.alpha = p.alpha;
    mp.m_limit = p.m_limit;
    mp.m_min = p.m_min;
    mp.zeta = p.zeta;
    mp.seed = p.seed;
    mp.base_prec = p.base_prec;
    mp.chunk = p.chunk;
    mp.bound = p.bound;
    mp.order = p.order;
    {
        double md2;
        std::memcpy(&md2, &v.min_d2_bits, sizeof md2);
        mp.r_min = n >= 2 ? std::sqrt(md2) : 0.0;
    }
    // spread bands in units of the mean leaf-box diagonal
    mp.spread_unit = tree_mean_leaf_diagonal(t, s);
    MtStats ms;
    st = multitree_run(t, mp, phi, coverage, &ms, s);
    if (st == MB_OK && stats) {
        stats->visited = ms.visited;
        stats->det_prunes = ms.det_prunes;
        stats->mc_prunes = ms.mc_prunes;
        stats->mc_failed = ms.mc_failed;
        stats->base_cases = ms.base_cases;
        stats->base_triples = ms.base_triples;
        stats->mc_samples = ms.mc_samples;
        stats->max_stack = ms.max_stack;
        stats->rounds = ms.rounds;
        stats->build_ms = own ? own->build_ms : 0.0;
        stats->traverse_ms = ms.traverse_ms;
        stats->classify_ms = ms.classify_ms;
        stats->mc_ms = ms.mc_ms;
        stats->base_ms = ms.base_ms;
    }
    if (own) tree_free(own);
    return st;
}

mb_status mb_eval_factorized(const double *x, int64_t n, int32_t fmt, int32_t planes,
                             double r_near, double *phi, mb_factor_stats *stats, void *stream) {
    clear_error();
    if (n < 0 || (n > 0 && (!x || !phi))) return fail(MB_ERR_INVALID, "bad points or output");
    if (fmt != MB_FP16 && fmt != MB_BF16) return fail(MB_ERR_INVALID, "unknown operand format");
    if (planes < 1 || planes > 3) return fail(MB_ERR_INVALID, "planes must be 1..3");
    if (!(r_near >= 0.0) || !std::isfinite(r_near)) return fail(MB_ERR_INVALID, "bad r_near");
    if (n >= ((int64_t)1 << 31)) return fail(MB_ERR_UNSUPPORTED, "n must be < 2^31");
    if (stats) *stats = mb_factor_stats{};
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return MB_OK;
    ValidateOut v{};
    mb_status st = check_points(x, n, s, &v);
    if (st != MB_OK) return st;
    if (n < 3) return zero_doubles(phi, n, s);
    DeviceTree *t = nullptr;
    if ((st = tree_build(x, n, 32, s, &t)) != MB_OK) return st;
    FactorStats fs;
    st = factorized_eval(t, (int)n, fmt, planes, r_near, phi, s, &fs);
    tree_free(t);
    if (st == MB_OK && stats) {
        stats->pairmat_ms = fs.pairmat_ms;
        stats->gemm_ms = fs.gemm_ms;
        stats->near_ms = fs.near_ms;
        stats->near_pairs = fs.near_pairs;
        stats->gemm_flops = fs.gemm_flops;
    }
    return st;
}

mb_status mb_farfield_eval(const double *x, int64_t nx, const double *y, int64_t ny,
                           const double *z, int64_t nz, int32_t order, double *out, void *stream) {
    clear_error();
    if (nx < 0 || ny < 1 || nz < 1 || (nx > 0 && (!x || !out)) || !y || !z)
        return fail(MB_ERR_INVALID, "bad point sets or output");
    if (order < 0 || order > 2) return fail(MB_ERR_UNSUPPORTED, "order must be 0, 1 or 2");
    return farfield_eval(x, nx, y, ny, z, nz, order, out, (hipStream_t)stream);
}

double mb_normal_quantile(double alpha_half) { return normal_quantile_upper(alpha_half); }

int64_t mb_struct_size(const char *name) {
    if (!name) return -1;
    const std::string s(name);
    if (s == "mb_mt_params") return (int64_t)sizeof(mb_mt_params);
    if (s == "mb_mt_stats") return (int64_t)sizeof(mb_mt_stats);
    if (s == "mb_factor_stats") return (int64_t)sizeof(mb_factor_stats);
    if (s == "mb_server_stats") return (int64_t)sizeof(mb_server_stats);
    return -1;
}

}  // extern "C"
