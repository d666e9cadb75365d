// C ABI entry points (declared in include/mb.h): argument checks, the
// validation step and dispatch to the kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "mb_internal.hpp"

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
        long mb = e ? std::atol(e) : 2048;
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

// Ratio limit between the bounding-box diagonal and the closest pair above
// which the binary32 path hands over to binary64.
constexpr double kFp32MaxRatio = 65536.0;

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

// Power of two that maps the closest-pair distance into [1, 2).
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
    double scale = 1.0;
    int p = prec;
    if (p == MB_FP32C) {
        double md2;
        std::memcpy(&md2, &v.min_d2_bits, sizeof md2);
        double diag2 = 0.0;
        for (int c = 0; c < 3; ++c) diag2 += (v.hi[c] - v.lo[c]) * (v.hi[c] - v.lo[c]);
        if (diag2 > kFp32MaxRatio * kFp32MaxRatio * md2)
            p = MB_FP64;  // dynamic range too wide for binary32 pair terms
        else
            scale = unit_scale(md2);
    }
    return direct_launch(x, n, p, scale, phi, s);
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

}  // extern "C"
