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
    MB_ERR_UNSUPPORTED = 5  /* request outside what this build implements       */
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
 * Exhaustive Phi(x_i) for all N points (the naive O(N^3) algorithm that the
 * paper's Section 6 uses as its baseline; definition in Section 1).
 *
 *   prec : MB_FP64 or MB_FP32C.  MB_FP32C rescales the point set by a power
 *          of two so the closest pair is near unit distance (exact), and
 *          falls back to MB_FP64 when the ratio of the largest to the
 *          smallest pair distance exceeds 2^16.
 *
 * Validation (device side, then a wait on `stream`): every coordinate must
 * be finite (else MB_ERR_INVALID); for N >= 3 no two points may coincide
 * (else MB_ERR_DEGENERATE).  N < 3 writes zeros (the empty sum) and returns
 * MB_OK.  n < 0, a NULL x or phi with n > 0, or an unknown prec return
 * MB_ERR_INVALID.  On any error phi is left unspecified.
 */
mb_status mb_eval_direct(const double *x, int64_t n, int32_t prec, double *phi, void *stream);

/*
 * mb_eval_direct without the validation step and without any wait: the
 * evaluation is only enqueued on `stream`.  For callers that have already
 * validated the same points (mb_validate) and must not block, e.g. a timing
 * loop or a request pipeline.  Preconditions (unchecked on the device): all
 * coordinates finite, no two points coincide.  prec MB_FP32C here never
 * falls back and uses no rescaling.  Host-side argument errors are reported
 * as for mb_eval_direct.
 */
mb_status mb_eval_direct_unchecked(const double *x, int64_t n, int32_t prec, double *phi,
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

#ifdef __cplusplus
}
#endif

#endif /* MB_H */
