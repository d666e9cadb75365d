/*
 * mb.h - C ABI of the MI355X (gfx950) library for the per-particle
 * Axilrod-Teller three-body potential.
 *
 * Problem (Section 1 of Lee, Ozakin & Gray, "Multibody Multipole Methods"):
 * given points X = {x_0, ..., x_{N-1}} in 3-D, compute for every x_i
 *
 *   Phi(x_i) = sum over j < k, j != i, k != i of phi(x_i, x_j, x_k),
 *   phi(x_i, x_j, x_k) = (1 + 3 cos t_i cos t_j cos t_k) / (r_ij r_ik r_jk)^3,
 *
 * where t_v is the triangle's interior angle at x_v and r_uv = |x_u - x_v|
 * (the Axilrod-Teller potential as printed, without a C9 prefactor).
 *
 * Conventions shared by every entry point:
 *   - x   : device pointer to N x 3 float64, row-major (x0, y0, z0, x1, ...),
 *           contiguous, owned by the caller, read-only for the library.
 *   - phi : device pointer to N float64, owned by the caller, written in the
 *           caller's input order.
 *   - stream : a hipStream_t passed as void* (NULL = the null stream).  All
 *           device work is enqueued on it.  A call that must report a status
 *           computed on the device (validation) waits for that stream.
 *   - The library never frees or retains caller pointers after returning.
 *   - Errors are status codes; mb_last_error() returns a message for the
 *     calling thread's last failed call.  No C++ exception crosses the ABI.
 *   - Point indices are 32-bit: N must be < 2^31.
 */
#ifndef MB_H
#define MB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MB_OK = 0,
    MB_ERR_INVALID = 1,     /* bad argument or non-finite coordinate            */
    MB_ERR_DEGENERATE = 2,  /* two coincident points: phi is undefined          */
    MB_ERR_OOM = 3,         /* device allocation failed or budget exceeded      */
    MB_ERR_DEVICE = 4,      /* a HIP call failed; see mb_last_error()           */
    MB_ERR_UNSUPPORTED = 5, /* request outside what the library implements      */
    MB_ERR_CANCELLED = 6    /* serving: request cancelled or timed out          */
} mb_status;

/* Arithmetic of the exhaustive (direct) sum and of the tree's base cases. */
typedef enum {
    MB_FP64 = 0,  /* binary64 throughout                                         */
    MB_FP32C = 1  /* pair terms formed in binary64, triple terms in binary32,
                     short binary32 partial sums folded into binary64            */
} mb_prec;

/* Message for the calling thread's last failed call ("" if none). */
const char *mb_last_error(void);

/* Library version as major * 10000 + minor * 100 + patch. */
int32_t mb_version(void);

/*
 * Return cached device memory to the device.  Every evaluation takes its
 * scratch (pair-term tables, work lists, unit rows) from the current
 * device's default memory pool by stream-ordered allocation, and the pool
 * keeps the freed blocks for later calls (its release threshold is set to
 * unlimited on first use), so repeated calls do not allocate again.
 * mb_trim waits for `stream` (the work of this library enqueued there,
 * frees included, has then run), then releases every block of that pool
 * that no allocation holds.  Memory held by live trees (mb_build_kdtree),
 * servers (mb_server_create) and the static array of
 * mb_eval_direct_noalloc is not touched.
 *   released : host pointer or NULL; receives the pool's reserved bytes
 *              before the trim minus those after it.
 * MB_ERR_DEVICE if a HIP call fails.
 */
mb_status mb_trim(void *stream, int64_t *released);

/*
 * Exhaustive Phi(x_i) for all N points (the naive O(N^3) algorithm that the
 * paper's Section 6 uses as its baseline; definition in Section 1).
 *
 *   prec : MB_FP64 or MB_FP32C.  MB_FP32C rescales the point set by a power
 *          of two so the closest pair is near unit distance (exact), and
 *          falls back to MB_FP64 when the ratio of the bounding-box
 *          diagonal to the closest-pair distance exceeds 2^16, or when the
 *          closest pair is shorter than a quarter of the mean spacing (cube
 *          root of bounding-box volume per point).  After the binary32 tiles
 *          it (1) re-adds in binary64 every triple whose three sides are
 *          shorter than 4 times the closest-pair distance (at most 64
 *          forward neighbours per point), the triples where the reuse of
 *          binary32 pair terms errs most, and (2) recomputes in binary64,
 *          point by point, the Phi of every point where |Phi| < 1/4 of the
 *          summed |phi| of those near triples (strong cancellation); if more
 *          than max(256, N/64) points qualify the whole sum is redone in
 *          binary64.  MB_FP32C therefore waits on `stream` at the end.
 *
 * Validation (device side, then a wait on `stream`): every coordinate must
 * be finite (else MB_ERR_INVALID); for N >= 3 no two points may coincide
 * (else MB_ERR_DEGENERATE).  N < 3 writes zeros (the empty sum) and returns
 * MB_OK.  n < 0, a NULL x or phi with n > 0, or an unknown prec return
 * MB_ERR_INVALID.  On any error phi is left unspecified.
 *
 * Device memory: a table of (i, j) pair terms, 12 bytes per pair in binary32
 * and 24 in binary64 over the blocks the work units touch (about N^2 / 2
 * pairs), built and consumed in stripes of at most MB_TABLE_BUDGET_MB
 * mebibytes (environment variable, default 32768); MB_ERR_OOM if it cannot
 * be allocated.
 */
mb_status mb_eval_direct(const double *x, int64_t n, int32_t prec, double *phi, void *stream);

/*
 * The binary64 exhaustive sum of mb_eval_direct (prec MB_FP64; Section 1's
 * definition) with every floating-point addition in an order fixed by N
 * alone: the same points give the same bits on every call, whatever the
 * scheduling of work on the GPU.  Within a work unit each wave keeps its
 * own partial sums and the waves are combined in wave order; each unit then
 * writes its sums to a row of device memory, and three passes add the rows
 * into Phi point by point in a fixed order.  The result differs from
 * mb_eval_direct's (whose FP64 atomics add in arrival order) only by
 * rounding, and the two differ bitwise from each other in general.
 *
 *   scratch_bytes : device-memory bound for one stripe of the evaluation
 *                   (pair-term table plus unit rows, 2 KiB per work unit of
 *                   64 x 64 x 128 slots); <= 0 means MB_TABLE_BUDGET_MB.
 *                   The J blocks are taken in stripes that fit it, at least
 *                   one block of 64 per stripe; stripes run in order.  A
 *                   one-block stripe still holds up to about N^2 / 32768
 *                   units (N^2 / 16 bytes of rows, 62.5 GB at N = 10^6),
 *                   which bounds this mode by device memory, not by
 *                   scratch_bytes.
 *
 * Validation, errors and the N < 3 case are those of mb_eval_direct; waits
 * on `stream` for the validation, then enqueues the sum.  MB_ERR_OOM if the
 * scratch cannot be allocated.
 */
mb_status mb_eval_direct_deterministic(const double *x, int64_t n, double *phi,
                                       int64_t scratch_bytes, void *stream);

/*
 * mb_eval_direct without the validation step and without any wait: the
 * evaluation is only enqueued on `stream`.  For callers that have already
 * validated the same points (mb_validate) and must not block, e.g. a timing
 * loop or a request pipeline.  Preconditions (unchecked on the device): all
 * coordinates finite, no two points coincide.  prec MB_FP32C here never
 * falls back, uses no rescaling and skips both binary64 repairs of
 * mb_eval_direct (binary32 tiles only).  Host-side argument errors are reported
 * as for mb_eval_direct.
 */
mb_status mb_eval_direct_unchecked(const double *x, int64_t n, int32_t prec, double *phi,
                                   void *stream);

/*
 * mb_eval_direct_unchecked for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same arguments, preconditions and result; it calls no
 * hipMalloc, hipFree or allocating routine.  Its scratch - the unit offsets
 * and the (i, j) pair-term table - lives in one library-owned device array
 * of 16 MiB + 256 bytes per GPU, allocated when the library is loaded and
 * held until the process ends, so N is limited to 1024
 * (MB_ERR_UNSUPPORTED above).  Every call on a GPU uses that GPU's array:
 * calls that overlap on one GPU (several streams or threads) race and give
 * wrong results.  Only enqueues work on `stream`.
 */
mb_status mb_eval_direct_noalloc(const double *x, int64_t n, int32_t prec, double *phi,
                                 void *stream);

/*
 * The minimum squared pair distance of the point set and whether every
 * coordinate is finite (the validation step of every evaluation, exposed
 * for callers that pick a precision themselves).
 *   min_d2 : host pointer, receives min over i < j of |x_i - x_j|^2
 *            (+inf for n < 2).
 *   finite : host pointer, receives 1 if all 3N coordinates are finite.
 *   bbox   : host pointer to 6 doubles or NULL; receives the bounding box
 *            (xmin, ymin, zmin, xmax, ymax, zmax), meaningful when finite.
 * Waits on `stream`.
 */
mb_status mb_validate(const double *x, int64_t n, double *min_d2, int32_t *finite, double *bbox,
                      void *stream);

/* ------------------------------------------------------------------------
 * kd-tree (BuildKdTree, Algorithm 1) and triple-tree traversal
 * (MTPotentialCanonical, Algorithm 2; approximation rules of Section 4)
 * ---------------------------------------------------------------------- */

/* Opaque device-resident kd-tree.  Immutable after build; may be shared by
 * calls on any stream of the device it was built on. */
typedef struct mb_tree_s *mb_tree;

/*
 * Build the kd-tree of the N points (Algorithm 1): a node holding more than
 * leaf_size points is split along the widest dimension of its tight
 * bounding box (ties to the lowest dimension) at the median by count: the
 * left child takes the floor(n/2) points first in the order (coordinate,
 * original index).  Points are kept in depth-first order; a node owns the
 * depth-first ranks [begin, end).  Nodes are numbered in pre-order (root 0,
 * left child = node + 1).
 *   leaf_size : 1 .. 32 (MB_ERR_UNSUPPORTED above 32, MB_ERR_INVALID below 1)
 *   out       : receives the tree; release with mb_free_kdtree.
 * Coordinates must be finite (MB_ERR_INVALID otherwise) and, for N >= 3, no
 * two points may coincide (MB_ERR_DEGENERATE).  Waits on stream.
 */
mb_status mb_build_kdtree(const double *x, int64_t n, int32_t leaf_size, void *stream,
                          mb_tree *out);

/* Release a tree (NULL is accepted). */
mb_status mb_free_kdtree(mb_tree t);

/* Sizes of a tree: points, nodes, depth of the deepest node, build time. */
mb_status mb_kdtree_info(mb_tree t, int64_t *n_points, int32_t *n_nodes, int32_t *max_depth,
                         double *build_ms);

/*
 * Copy a tree to host arrays (each pointer may be NULL):
 *   perm     [N]     original index of the point at each depth-first rank
 *   ranges   [2M]    begin, end of node v at 2v, 2v+1
 *   children [2M]    left, right of node v (-1, -1 for a leaf)
 *   bbox     [6M]    lower corner then upper corner of node v at 6v
 *   centroid [3M]    mean of node v's points
 */
mb_status mb_kdtree_export(mb_tree t, int32_t *perm, int32_t *ranges, int32_t *children,
                           double *bbox, double *centroid);

/* Parameters of the traversal (error criteria of Definitions 2.1-2.3). */
typedef struct {
    double eps_rel;    /* epsilon: relative error bound (Definition 2.2), >= 0         */
    double tau_abs;    /* tau: absolute error bound (Definition 2.1), >= 0             */
    double alpha;      /* 1 - alpha: probability level (Definition 2.3), 0 <= alpha < 1;
                          0 disables Monte Carlo (deterministic guarantee only)        */
    int32_t m_limit;   /* samples per point before Monte Carlo gives up (Algorithm 4)  */
    int32_t m_min;     /* samples required before the normal approximation is used    */
    double zeta;       /* Monte Carlo is tried only if zeta * m_limit <= min_i T_i     */
    uint64_t seed;     /* seed of the counter-based sampler                            */
    int32_t base_prec; /* arithmetic of the exhaustive base cases: MB_FP64 or MB_FP32C */
    int32_t chunk;     /* node triples processed per round of the device stack         */
    int32_t bound;     /* MB_BOUND_SIGNED or MB_BOUND_TWO_SIDED (below)                */
    int32_t order;     /* expansion order p of a deterministic prune's estimate, 0..2:
                          0 = the monopole |P_j| |P_k| phi(c1, c2, c3) of Section 4;
                          1, 2 = the truncated three-body far-field expansion of
                          Section 3.2 at each point of a node due to the other two
                          (mb_farfield_eval), for node triples where every two
                          nodes have radii summing to at most half their centroid
                          distance (elsewhere the monopole).  The prune test is
                          the same for every p.                                     */
} mb_mt_params;

/*
 * What the node statistics of the prune rules hold.  Both accumulate, per
 * point, what has been credited to it so far: exact base-case values, and
 * for pruned node triples the ends of the interval that bounds them
 * (T_i phi_lo .. T_i phi_hi for a deterministic prune, T_i (mu -+ z sigma_mu)
 * for a Monte Carlo one).
 *   MB_BOUND_SIGNED: the paper's running lower bound Phi^l (Section 4.1, the
 *     deterministic-prune equation, and the relative termination rule of
 *     Algorithm 4).  It presumes potentials >= 0: for a point whose Phi is
 *     negative it stays negative, and no node triple holding that point is
 *     pruned.
 *   MB_BOUND_TWO_SIDED: a running upper bound is kept beside it, and the
 *     allowance is a lower bound on max(lower, -upper), i.e. on |Phi| (the
 *     relative bound of Definition 2.2) from whichever side has settled.
 *     For potentials >= 0 it is the same rule as MB_BOUND_SIGNED.
 * For the sign-indefinite Axilrod-Teller potential neither running sum is a
 * bound on the final Phi (triples not yet credited may have either sign), so
 * the eps guarantee is empirical in both modes: measured as the fraction of
 * points within eps.
 */
enum { MB_BOUND_SIGNED = 0, MB_BOUND_TWO_SIDED = 1 };

/* Defaults: eps 1e-2, tau 0, alpha 0.05, m_limit 128, m_min 30, zeta 128 (one
 * Monte Carlo sample - a counter-based draw, an index map, gathers and a
 * binary64 phi - costs tens of the binary32 tile terms of a base case, so
 * sampling pays only where it replaces far more tuples than the paper's
 * small zeta suggests; measured on the 65536-point mixture: 7.2 s at
 * zeta 4, 3.8 s at 128, 4.2 s without Monte Carlo),
 * seed 0, base_prec MB_FP32C, chunk 1048576, bound MB_BOUND_SIGNED, order 0. */
void mb_mt_params_default(mb_mt_params *p);

typedef struct {
    int64_t visited;      /* node triples examined                                   */
    int64_t det_prunes;   /* triples summarized by the deterministic bound           */
    int64_t mc_prunes;    /* triples summarized by Monte Carlo                       */
    int64_t mc_failed;    /* Monte Carlo attempts that did not meet the bound        */
    int64_t base_cases;   /* leaf triples summed exhaustively                        */
    int64_t base_triples; /* particle triples in those base cases                    */
    int64_t mc_samples;   /* phi evaluations drawn by Monte Carlo                    */
    int64_t max_stack;    /* largest device stack (node triples)                     */
    int64_t rounds;       /* rounds of the device stack                              */
    double build_ms;      /* tree build (0 if a tree was passed in)                  */
    double traverse_ms;   /* traversal incl. top-down pass                           */
    double classify_ms;   /* device time classifying node triples (and far-field
                             estimates of prunes)                                    */
    double mc_ms;         /* device time of Monte Carlo tests                        */
    double base_ms;       /* device time of base cases (sort, units, tiles)         */
} mb_mt_stats;

/*
 * Approximate Phi(x) for all points by the triple-tree traversal
 * (Algorithm 2 with CanSummarize / Summarize of Section 4 and Algorithms
 * 3-5), aiming at |Phi~ - Phi| <= eps |Phi| + tau per point in the sense of
 * Definition 2.3 (with alpha = 0, Theorem 5.1's deterministic form).  The
 * deterministic prune bounds phi over every triangle whose sides lie between
 * the smallest and largest distances d^l, d^u of the three node boxes
 * (phi = R g, R = (r_12 r_13 r_23)^-3 over its range, g = 1 + 3 cos cos cos
 * from exact ranges of the cosines, clipped to [-2, 11/8]); every d^l is
 * raised to the closest-pair distance of the points.  Because the
 * Axilrod-Teller potential is sign-indefinite, the running statistics are
 * not bounds on the final Phi and the guarantee is checked empirically (see
 * the bound modes above).
 *   tree     : a tree built by mb_build_kdtree from these same points (the
 *              coordinates are compared bit for bit on the device), or NULL
 *              to build one internally with leaf_size.
 *   params   : host pointer (NULL = defaults).
 *   phi      : device, N doubles, input order.
 *   coverage : device, N int64 or NULL; receives the number of particle
 *              triples credited to each point (C(N-1, 2) when the traversal
 *              partitions the tuples exactly, which it does by construction).
 *   stats    : host, nullable.
 * Validation as for mb_eval_direct.  eps < 0, tau < 0, alpha outside [0,1),
 * m_limit < 2, m_min < 2, zeta < 0, or a tree built for other points ->
 * MB_ERR_INVALID.  Waits on stream (the host drives the device stack).
 */
mb_status mb_eval_multitree(const double *x, int64_t n, int32_t leaf_size,
                            const mb_mt_params *params, mb_tree tree, double *phi,
                            int64_t *coverage, mb_mt_stats *stats, void *stream);

/* ------------------------------------------------------------------------
 * Factorized form (matrix products on MFMA)
 * ---------------------------------------------------------------------- */

typedef enum { MB_FP16 = 0, MB_BF16 = 1 } mb_half;

typedef struct {
    double pairmat_ms;  /* building the pair-matrix planes                          */
    double gemm_ms;     /* the five products with their epilogues                   */
    double near_ms;     /* exact near-field triples and the final combination       */
    int64_t near_pairs; /* pairs closer than r_near                                  */
    double gemm_flops;  /* MFMA flops issued (10 N_pad^3 per plane product)         */
} mb_factor_stats;

/*
 * Phi(x) for all points through the product form of the potential.  The
 * law of cosines writes the Axilrod-Teller phi (Section 1) as ten products
 * of pairwise powers r_ij^e1 r_ik^e2 r_jk^e3 - the product-of-pairwise form
 * the paper's method requires - so Phi_i = 1/2 sum_t c_t (A_t C_t B_t^T)_ii
 * with pair matrices of r^e (e in -5, -3, -1, +1) with zero diagonals; this
 * form is an extension, not in the paper.  Triples with a side shorter than
 * r_near are excluded from the matrices and summed exactly in binary64.
 *   fmt    : MB_FP16 or MB_BF16 operands of the matrix products.
 *   planes : 1..3 - each matrix entry is held as a sum of `planes` numbers of
 *            the format (a per-64x64-tile power of two keeps all in range);
 *            products of planes are kept while their level is < planes.
 *            Accumulation is binary32 inside 64-wide chunks and over groups
 *            of up to 8 chunks at one reference scale, binary64 across groups.
 *   r_near : >= 0, in the units of x.
 *   stats  : host, nullable.
 * Device memory: 4 * planes * Np^2 * 2 bytes, Np = N rounded up to 128
 * (MB_ERR_OOM if it cannot be allocated).  Validation as mb_eval_direct.
 * Waits on stream.
 */
mb_status mb_eval_factorized(const double *x, int64_t n, int32_t fmt, int32_t planes,
                             double r_near, double *phi, mb_factor_stats *stats, void *stream);

/*
 * The three-body far-field expansion of order p (Section 3.2, its truncated
 * form) at nx target points due to two source sets: for each target x,
 *   sum over |a| + |b| <= p of C_ab(x) M_a(Y) M_b(Z),
 * the degree-p Taylor polynomial of phi(x, cY + u, cZ + v) in the source
 * displacements (u, v), summed over y in Y and z in Z, with cY, cZ the
 * centroids and M the moments about them (p = 0: |Y| |Z| phi(x, cY, cZ);
 * the first-order moments about a centroid vanish, so p = 1 equals p = 0).
 *   x : device, nx x 3 (nx >= 0);  y : device, ny x 3 (ny >= 1);
 *   z : device, nz x 3 (nz >= 1);  out : device, nx doubles.
 *   order : 0, 1 or 2 (MB_ERR_UNSUPPORTED otherwise).
 * The expansion converges when the sets are small against their distances
 * to each other and to x; no check is made.  Enqueue only.
 */
mb_status mb_farfield_eval(const double *x, int64_t nx, const double *y, int64_t ny,
                           const double *z, int64_t nz, int32_t order, double *out, void *stream);

/*
 * z such that P(Z > z) = alpha_half for a standard normal Z: the quantile
 * z_{alpha/2} of the Monte Carlo stop rule is mb_normal_quantile(alpha / 2).
 * Host only; returns 0 for alpha_half outside (0, 0.5).
 */
double mb_normal_quantile(double alpha_half);

/*
 * Serving (an extension: the paper evaluates one point set at a time).  A
 * server owns a host thread that batches exhaustive Phi evaluations of many
 * point sets of different N as they arrive:
 *   - admission: requests are admitted in arrival order while a slot is free
 *     and their device footprint fits the HBM budget; the footprint of a
 *     request of N points is 24 N + 16 N bytes (points, Phi, near-field
 *     magnitudes) plus a region for its (i, j) pair-term table (about N^2
 *     numbers: a and w of each pair) large enough for either the binary32
 *     or the binary64 table, each part rounded up to 256 B; the request holds all of it
 *     until it is released, whichever table validation selects;
 *   - continuous batching: the work units (block triples) of all admitted
 *     requests are drained together by one persistent kernel whose
 *     workgroups take (request, unit) items from a ring in coherent pinned
 *     host memory, which the server thread writes directly, in slices of a
 *     bounded number of units, requests with the fewest units left first
 *     (MB_SERVE_TRACE in the environment: a progress line every 2 s on
 *     stderr).  The kernel is launched cooperatively (all its
 *     workgroups resident at once, on a hardware queue no other stream
 *     shares), stays resident while work arrives and exits after all its
 *     workgroups have been idle for 20 ms at once (it is launched again
 *     when work arrives); it leaves 32 CUs free for the staging and
 *     finishing kernels of requests;
 *   - completion: when a request's last unit has run, its Phi is copied back
 *     and the request counts as done (latency = done - submit, host clock).
 * Results are those of mb_eval_direct with the same precision, up to the
 * order of binary64 additions.
 */
typedef struct {
    int64_t submitted, completed, failed; /* failed: finished with an error     */
    int64_t fp64_fallbacks;                /* binary32 requests run in binary64  */
    int64_t slices, units;                 /* slices published, work units run   */
    int64_t mixed_slices;                  /* slices holding units of >= 2 requests */
    int64_t points_fp64;                   /* points recomputed in binary64 after binary32 */
    int64_t peak_reserved;                 /* bytes of the budget held at most   */
    int32_t peak_active;                   /* admitted requests at most          */
    int32_t drain_launches;                /* launches of the persistent drain kernel */
    double triples;                        /* sum of C(N, 3) of completed ones   */
    double busy_ms;                        /* wall time with units outstanding on the device */
    double stage_ms, finalize_ms;          /* host time staging / finishing requests */
    int64_t cancelled;                     /* cancelled or timed out (also in failed) */
} mb_server_stats;

/*
 * Create a server.  hbm_budget_bytes > 0 bounds the device memory held by
 * admitted requests; 1 <= max_slots <= 4096 bounds how many are admitted at
 * once.  stream: the compute stream (NULL: the server creates its own); a
 * second, server-owned stream stages requests.  Uses the current device.
 * *srv receives an opaque handle.
 */
mb_status mb_server_create(int64_t hbm_budget_bytes, int32_t max_slots, void *stream, void **srv);

/*
 * Queue one request.  host_x: host pointer to N x 3 float64, row-major; it is
 * copied before the call returns.  prec: MB_FP64 or MB_FP32C (which falls
 * back to binary64 as mb_eval_direct does).  *req_id receives the id.
 * Errors at submission: MB_ERR_INVALID (bad argument or non-finite
 * coordinate), MB_ERR_OOM (the footprint exceeds the whole budget), and
 * MB_ERR_DEVICE once the server has stopped after a device error.  N < 3
 * completes at once with Phi = 0.  Coincident points are found on the device:
 * the request then finishes with MB_ERR_DEGENERATE.
 */
mb_status mb_server_submit(void *srv, const double *host_x, int64_t n, int32_t prec,
                           int64_t *req_id);

/*
 * Non-blocking status of a request.  *done = 1 once it has finished.  If it
 * finished with an error, that status is returned (with *done = 1).  If
 * host_phi is non-NULL and the request succeeded, its N results are copied
 * there (caller's input order) and the server drops its copy: a second fetch
 * is MB_ERR_INVALID.  Unknown id: MB_ERR_INVALID.
 */
mb_status mb_server_poll(void *srv, int64_t req_id, double *host_phi, int32_t *done);

/*
 * Block until request req_id (or, for req_id < 0, every request submitted so
 * far) has finished, or timeout_ms milliseconds have passed (timeout_ms < 0:
 * no limit).  *done (nullable) tells which.
 */
mb_status mb_server_wait(void *srv, int64_t req_id, int32_t timeout_ms, int32_t *done);

/* Seconds from submission to completion of a finished request. */
mb_status mb_server_latency(void *srv, int64_t req_id, double *seconds);

/*
 * Stop a request.  One that has not finished ends with MB_ERR_CANCELLED
 * (poll and wait report it like any other error): a queued request leaves
 * the queue; one being staged is dropped when its staging work has landed;
 * a running one hands out no more work units, and its device memory and
 * slot return once the units already published have run.  A request whose
 * last unit has run (its result is being copied back) completes normally.
 * The server's thread carries the cancellation out shortly after the call.
 * MB_OK for any known id, finished or not; unknown id: MB_ERR_INVALID.
 */
mb_status mb_server_cancel(void *srv, int64_t req_id);

/*
 * Time limit for requests submitted after the call: a request not finished
 * timeout_ms milliseconds after its submission is cancelled as by
 * mb_server_cancel (MB_ERR_CANCELLED, message "timed out after ... ms").
 * timeout_ms <= 0: no limit (the default).
 */
mb_status mb_server_set_timeout(void *srv, int32_t timeout_ms);

/* Counters of the server so far (host struct). */
mb_status mb_server_stats_get(void *srv, mb_server_stats *out);

/* Units per slice (>= 1, at most 65536); the default is 8 per workgroup of
 * the drain kernel.  At most two slices' worth of units are outstanding on
 * the device at a time.  Takes effect at the next slice. */
mb_status mb_server_set_slice_units(void *srv, int64_t units);

/* Finish every request already submitted, then free the server. */
mb_status mb_server_destroy(void *srv);

/*
 * sizeof of a struct of this header by name ("mb_mt_params", "mb_mt_stats",
 * "mb_factor_stats", "mb_server_stats"), so that bindings can check their
 * layouts; -1 for an unknown name.  Host only.
 */
int64_t mb_struct_size(const char *name);

#ifdef __cplusplus
}
#endif

#endif /* MB_H */
