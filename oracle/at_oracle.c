/*
 * CPU oracle for the per-particle Axilrod-Teller potential.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the GPU library.
 *
 * What it computes is the plain definition, in IEEE binary64:
 *
 *   phi(x_i, x_j, x_k) = (1 + 3 cos t_i cos t_j cos t_k) / (r_ij r_ik r_jk)^3
 *       (Section 1, the Axilrod-Teller potential; t_v is the interior angle of
 *        the triangle at vertex v, r_uv the Euclidean distance)
 *
 *   Phi(x_i) = sum over j < k, j != i, k != i of phi(x_i, x_j, x_k)
 *       (Section 1, the canonical multibody summation for n = 3: fix x, sum
 *        over the 2-subsets of X \ {x} in increasing index order)
 *
 * The cosines are formed from displacement dot products,
 * cos t_i = (x_j - x_i).(x_k - x_i) / (r_ij r_ik), and likewise at j and k.
 * Each particle's sum is compensated (Neumaier's improved Kahan summation),
 * so the oracle's own rounding error is far below the 1e-12 parity bar.
 * Particles are independent; OpenMP spreads them over host threads.
 */
#include <math.h>
#include <stdint.h>
#include <omp.h>

/* The Axilrod-Teller value of one triangle (Section 1). */
double oracle_at_phi(const double *xi, const double *xj, const double *xk)
{
    double dij[3], dik[3], djk[3];
    for (int d = 0; d < 3; ++d) {
        dij[d] = xj[d] - xi[d];
        dik[d] = xk[d] - xi[d];
        djk[d] = xk[d] - xj[d];
    }
    double rij = sqrt(dij[0] * dij[0] + dij[1] * dij[1] + dij[2] * dij[2]);
    double rik = sqrt(dik[0] * dik[0] + dik[1] * dik[1] + dik[2] * dik[2]);
    double rjk = sqrt(djk[0] * djk[0] + djk[1] * djk[1] + djk[2] * djk[2]);
    /* angle at i between (x_j - x_i) and (x_k - x_i) */
    double ci = (dij[0] * dik[0] + dij[1] * dik[1] + dij[2] * dik[2]) / (rij * rik);
    /* angle at j between (x_i - x_j) and (x_k - x_j) = (-dij) and djk */
    double cj = -(dij[0] * djk[0] + dij[1] * djk[1] + dij[2] * djk[2]) / (rij * rjk);
    /* angle at k between (x_i - x_k) and (x_j - x_k) = (-dik) and (-djk) */
    double ck = (dik[0] * djk[0] + dik[1] * djk[1] + dik[2] * djk[2]) / (rik * rjk);
    double r3 = rij * rik * rjk;
    r3 = r3 * r3 * r3;
    return (1.0 + 3.0 * ci * cj * ck) / r3;
}

/* Neumaier (1974) compensated accumulator. */
typedef struct {
    double s, c;
} oracle_acc;

static inline void acc_add(oracle_acc *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

/*
 * Phi(x_i) for each requested particle i = idx[s], s < m; out[s] receives it.
 * x is N x 3 row-major.  Returns 0, or -1 on a bad argument.
 */
int oracle_phi(const double *x, int64_t n, const int64_t *idx, int64_t m, double *out,
               int nthreads)
{
    if (n < 0 || m < 0)
        return -1;
    for (int64_t s = 0; s < m; ++s)
        if (idx[s] < 0 || idx[s] >= n)
            return -1;
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < m; ++s) {
        int64_t i = idx[s];
        oracle_acc acc = {0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            for (int64_t k = j + 1; k < n; ++k) {
                if (k == i)
                    continue;
                acc_add(&acc, oracle_at_phi(x + 3 * i, x + 3 * j, x + 3 * k));
            }
        }
        out[s] = acc.s + acc.c;
    }
    return 0;
}

/*
 * Total three-body energy E = sum over i < j < k of phi(x_i, x_j, x_k),
 * a separate loop used to pin sum_i Phi(x_i) = 3 E.
 */
int oracle_energy(const double *x, int64_t n, double *e_out, int nthreads)
{
    if (n < 0)
        return -1;
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
    double total_s = 0.0, total_c = 0.0;
#pragma omp parallel
    {
        oracle_acc acc = {0.0, 0.0};
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j)
                for (int64_t k = j + 1; k < n; ++k)
                    acc_add(&acc, oracle_at_phi(x + 3 * i, x + 3 * j, x + 3 * k));
#pragma omp critical
        {
            oracle_acc t = {total_s, total_c};
            acc_add(&t, acc.s);
            acc_add(&t, acc.c);
            total_s = t.s;
            total_c = t.c;
        }
    }
    *e_out = total_s + total_c;
    return 0;
}

/*
 * Phi(x_i) restricted to triangles whose three side lengths all satisfy the
 * predicate r >= r_cut (keep_far = 1) or that have at least one side with
 * r < r_cut (keep_far = 0).  The two restricted sums add up to Phi(x_i); they
 * are the far and near parts of the factorized form's split.
 */
int oracle_phi_split(const double *x, int64_t n, const int64_t *idx, int64_t m, double r_cut,
                     int keep_far, double *out, int nthreads)
{
    if (n < 0 || m < 0)
        return -1;
    for (int64_t s = 0; s < m; ++s)
        if (idx[s] < 0 || idx[s] >= n)
            return -1;
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < m; ++s) {
        int64_t i = idx[s];
        const double *xi = x + 3 * i;
        oracle_acc acc = {0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            const double *xj = x + 3 * j;
            for (int64_t k = j + 1; k < n; ++k) {
                if (k == i)
                    continue;
                const double *xk = x + 3 * k;
                double rij = sqrt((xj[0] - xi[0]) * (xj[0] - xi[0]) + (xj[1] - xi[1]) * (xj[1] - xi[1]) +
                                  (xj[2] - xi[2]) * (xj[2] - xi[2]));
                double rik = sqrt((xk[0] - xi[0]) * (xk[0] - xi[0]) + (xk[1] - xi[1]) * (xk[1] - xi[1]) +
                                  (xk[2] - xi[2]) * (xk[2] - xi[2]));
                double rjk = sqrt((xk[0] - xj[0]) * (xk[0] - xj[0]) + (xk[1] - xj[1]) * (xk[1] - xj[1]) +
                                  (xk[2] - xj[2]) * (xk[2] - xj[2]));
                int far = rij >= r_cut && rik >= r_cut && rjk >= r_cut;
                if (far == (keep_far != 0))
                    acc_add(&acc, oracle_at_phi(xi, xj, xk));
            }
        }
        out[s] = acc.s + acc.c;
    }
    return 0;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }
