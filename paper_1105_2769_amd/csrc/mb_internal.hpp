// Host-side helpers shared by the library's translation units: error state,
// HIP error mapping and stream-ordered scratch allocation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/mb.h"

namespace mb {

// Record a message for mb_last_error() and return the status.
mb_status fail(mb_status st, const std::string &msg);
void clear_error();
const char *last_error_cstr();

// Map a HIP error to MB_ERR_DEVICE (or MB_ERR_OOM for allocation failures).
mb_status hip_fail(hipError_t e, const char *what);

#define MB_HIP(call)                                                 \
    do {                                                             \
        hipError_t mb_e_ = (call);                                   \
        if (mb_e_ != hipSuccess) return ::mb::hip_fail(mb_e_, #call); \
    } while (0)

// Keep freed stream-ordered memory in the current device's pool instead of
// returning it to the driver at every synchronization (once per device).
void device_pool_setup();

// Stream-ordered device scratch that frees itself on scope exit.
struct Scratch {
    void *ptr = nullptr;
    hipStream_t stream = nullptr;
    Scratch() = default;
    Scratch(const Scratch &) = delete;
    Scratch &operator=(const Scratch &) = delete;
    ~Scratch() {
        if (ptr) (void)hipFreeAsync(ptr, stream);
    }
    mb_status alloc(size_t bytes, hipStream_t s) {
        stream = s;
        device_pool_setup();
        hipError_t e = hipMallocAsync(&ptr, bytes ? bytes : 1, s);
        if (e != hipSuccess) {
            ptr = nullptr;
            return hip_fail(e, "hipMallocAsync");
        }
        return MB_OK;
    }
    template <typename T>
    T *as() const {
        return static_cast<T *>(ptr);
    }
};

// Result of the validation pass (device layout mirrors this struct).
struct ValidateOut {
    unsigned long long min_d2_bits;  // bit pattern of min |xi-xj|^2 (non-negative double)
    int32_t nonfinite;               // nonzero if any coordinate is NaN or Inf
    int32_t pad;
    unsigned long long lo_key[3];    // order-preserving keys of the bounding box
    unsigned long long hi_key[3];
    // filled on the host after the copy back
    double lo[3];
    double hi[3];
};

// Enqueue validation and wait for it.  n >= 0.
mb_status validate_points(const double *x, int64_t n, hipStream_t s, ValidateOut *out);

// The same without the wait: the result lands in *out (host) when the stream
// reaches the copy; dev is device scratch of sizeof(ValidateOut).  Call
// validate_decode on it afterwards.
mb_status validate_enqueue(const double *x, int64_t n, hipStream_t s, ValidateOut *dev,
                           ValidateOut *out);
void validate_decode(ValidateOut *out, int64_t n);

// Enqueue phi[0:n] = 0.
mb_status zero_doubles(double *p, int64_t n, hipStream_t s);

// Upper bound on the bytes of the (i, j) pair-term table the exhaustive sum
// keeps per launch stripe (MB_TABLE_BUDGET_MB overrides, default 32 GiB: one
// stripe up to N = 46000 in binary32, 32768 in binary64).
size_t table_budget_bytes();

// Direct (exhaustive) evaluation, no validation; phi is zeroed and
// accumulated.  `scale` is a power of two applied to all coordinate
// differences (the result is rescaled exactly).  For binary32 tiles, r_fix > 0
// also runs the near-field refinement below.
// `recomputed` (nullable) receives how many points point_fp64_finish redid.
mb_status direct_launch(const double *x, int64_t n, int prec, double scale, double *phi,
                        hipStream_t s, double r_fix = 0.0, int64_t *recomputed = nullptr);

// The binary64 exhaustive sum with every addition in a fixed order
// (mb_eval_direct_deterministic); phi is zeroed first.  Scratch per stripe
// of J blocks (pair table and unit rows) stays within `budget` bytes where
// one J block allows.
mb_status direct_launch_ordered(const double *x, int64_t n, double *phi, size_t budget,
                                hipStream_t s);

// The exhaustive sum as mb_eval_direct_unchecked, with its scratch in the
// library's static device array (no allocation); n <= kNoAllocMaxN.
constexpr int64_t kNoAllocMaxN = 1024;
mb_status direct_launch_noalloc(const double *x, int64_t n, int prec, double *phi, hipStream_t s);

// Near-field refinement of a binary32 tile sum already in (or going to)
// phi: every triple with all sides < r_fix (input units), at most 64
// forward neighbours per point, is moved from its binary32 tile value to
// binary64.  mag[0:n] receives, per point, the sum of |phi| over those
// triples.  Enqueue only.
mb_status near_refine_launch(const double *x, int64_t n, double scale, double r_fix, double *phi,
                             double *mag, hipStream_t s);

// After a refined binary32 sum: points with |Phi| < kPointFixRatio * mag
// (where cancellation can lift the binary32 error above 1e-6 of |Phi|) get
// Phi recomputed point by point in binary64, at most point_fix_cap(n) of
// them.  Enqueue only; *count_host receives the number of such points once
// the stream reaches it (more than the cap: the caller must redo the whole
// sum, point_fp64_redo_all).
int64_t point_fix_cap(int64_t n);
mb_status point_fp64_enqueue(const double *x, int64_t n, const double *mag, double *phi,
                             hipStream_t s, int32_t *count_host);
mb_status point_fp64_redo_all(const double *x, int64_t n, double *phi, hipStream_t s);

// Radius of the near-field refinement, in multiples of the closest-pair
// distance.
constexpr double kNearFixFactor = 4.0;
constexpr double kPointFixRatio = 0.25;
constexpr int64_t kPointFixMin = 256;
constexpr int64_t kPointFixShare = 64;

// Ratio limit between the bounding-box diagonal and the closest pair above
// which the binary32 path hands over to binary64.
constexpr double kFp32MaxRatio = 65536.0;

// validate_points plus the status it implies: MB_ERR_INVALID for a
// non-finite coordinate, MB_ERR_DEGENERATE for coincident points (n >= 3).
mb_status check_points(const double *x, int64_t n, hipStream_t s, ValidateOut *v);

// Power of two that maps the closest-pair distance sqrt(min_d2) into [1, 2).
double unit_scale(double min_d2);

// Whether binary32 tiles suit a validated point set: the bounding-box
// diagonal is within kFp32MaxRatio of the closest pair, and the closest pair
// is at least a quarter of the mean spacing (cube root of box volume per
// point).  A pair much closer than the spacing makes thin triangles whose
// binary32 law-of-cosines terms lose about log2(spacing / pair) bits.
bool fp32c_suitable(const ValidateOut &v, int64_t n);

// The far-field expansion of order `order` (0..2) at nx target points x due
// to the source sets y (ny points) and z (nz), about their centroids; out
// receives one value per target.  Enqueue only.
mb_status farfield_eval(const double *x, int64_t nx, const double *y, int64_t ny, const double *z,
                        int64_t nz, int order, double *out, hipStream_t s);

struct FactorStats {
    double pairmat_ms = 0.0, gemm_ms = 0.0, near_ms = 0.0;
    int64_t near_pairs = 0;
    double gemm_flops = 0.0;
};

}  // namespace mb
