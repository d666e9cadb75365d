// Host interface of the triple-tree traversal.
#pragma once

#include <cstdint>

#include "mb_internal.hpp"
#include "tree.hpp"

namespace mb {

struct MtParams {
    double eps = 0.0, tau = 0.0, alpha = 0.0;
    int m_limit = 128, m_min = 30;
    double zeta = 4.0;
    uint64_t seed = 0;
    int base_prec = MB_FP32C;
    int chunk = 65536;
    double r_min = 0.0;  // closest pair distance (a sound floor for box distances)
    // traversal order: triples are taken in bands of increasing spread (the
    // largest box distance within the triple): 0, unit, 2 unit, 4 unit, ...;
    // 0 disables the bands (one LIFO stack)
    double spread_unit = 0.0;
    int bound = MB_BOUND_SIGNED;  // or MB_BOUND_TWO_SIDED (running lower and upper bounds)
    int order = 0;  // 0: monopole estimate of a prune; 1, 2: far-field expansion at each point
};

struct MtStats {
    int64_t visited = 0, det_prunes = 0, mc_prunes = 0, mc_failed = 0, base_cases = 0,
            base_triples = 0, mc_samples = 0, max_stack = 0, rounds = 0;
    double traverse_ms = 0.0;
    double classify_ms = 0.0, mc_ms = 0.0, base_ms = 0.0;
};

// Whether tree t was built from the points x (N = n, same coordinates bit for
// bit in the tree's order).  Waits on s.
mb_status tree_matches_points(const DeviceTree *t, const double *x, int64_t n, hipStream_t s,
                              bool *same);

// z with P(Z > z) = alpha_half for a standard normal Z (0 if out of range).
double normal_quantile_upper(double alpha_half);

// Runs the traversal over a built tree; phi (device, input order) receives
// the estimate, coverage (device, nullable) the number of tuples credited
// to each point.
mb_status multitree_run(const DeviceTree *t, const MtParams &prm, double *phi, int64_t *coverage,
                        MtStats *stats, hipStream_t s);

}  // namespace mb
