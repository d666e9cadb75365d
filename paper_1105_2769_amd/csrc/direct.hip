// Exhaustive per-particle Axilrod-Teller sum on gfx950 (the naive algorithm
// of Section 6, definition in Section 1), plus input validation.  The tile
// code and its work decomposition are in direct_tile.hpp.
#include "direct_tile.hpp"
#include "mb_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace mb {
namespace {

template <typename T>
__global__ __launch_bounds__(kThreads, 1) void direct_kernel(
    const double *__restrict__ x, int n, int na, int nb, int nt,
    const int64_t *__restrict__ unit_off, int64_t u_begin, int64_t u_end, int b0,
    const T *__restrict__ utab, double scale, double out_scale, double *__restrict__ phi) {
    constexpr int IB = DirectLds<T>::IB;
    __shared__ DirectLds<T> s;
    for (int64_t u = u_begin + blockIdx.x; u < u_end; u += gridDim.x) {
        int a, b, t;
        decode_unit(u, unit_off, nb, nt, a, b, t);
        direct_unit<T>(s, x, n, a, b, t, utab + ((int64_t)(b - b0) * na + a) * (IB * kB * 3),
                       scale, out_scale, phi);
    }
}

// Prefix offsets of the unit list, units of J block b: units_a(b) * (nt - b / 4).
__global__ void unit_offsets_kernel(int nb, int nt, int ib, int na, int64_t *__restrict__ off) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t acc = 0;
    off[0] = 0;
    for (int b = 0; b < nb; ++b) {
        acc += (int64_t)units_a(b, ib, na) * (nt - (b >> 2));
        off[b + 1] = acc;
    }
}

__global__ void zero_kernel(double *__restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// Order-preserving map of a double to an unsigned key (for atomic min/max).
__device__ __forceinline__ unsigned long long order_key(double d) {
    unsigned long long b = (unsigned long long)__double_as_longlong(d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ void validate_init_kernel(ValidateOut *out) {
    out->min_d2_bits = 0x7FF0000000000000ull;  // +inf
    out->nonfinite = 0;
    out->pad = 0;
    for (int d = 0; d < 3; ++d) {
        out->lo_key[d] = ~0ull;
        out->hi_key[d] = 0ull;
    }
}

constexpr int kVT = 256;

// One workgroup compares the points of tile bi with those of tile bj >= bi.
__global__ __launch_bounds__(kVT) void validate_kernel(const double *__restrict__ x, int n,
                                                       ValidateOut *out) {
    const int bi = blockIdx.y, bj = blockIdx.x;
    if (bj < bi) return;
    __shared__ double xj[3][kVT];
    const int tid = threadIdx.x;
    const int j = bj * kVT + tid;
    xj[0][tid] = j < n ? x[3 * (int64_t)j + 0] : 0.0;
    xj[1][tid] = j < n ? x[3 * (int64_t)j + 1] : 0.0;
    xj[2][tid] = j < n ? x[3 * (int64_t)j + 2] : 0.0;
    __syncthreads();
    const int i = bi * kVT + tid;
    double mn = __longlong_as_double(0x7FF0000000000000ll);
    if (i < n) {
        const double x0 = x[3 * (int64_t)i], x1 = x[3 * (int64_t)i + 1], x2 = x[3 * (int64_t)i + 2];
        const int cend = min(kVT, n - bj * kVT);
        for (int c = 0; c < cend; ++c) {
            const int jj = bj * kVT + c;
            if (jj <= i) continue;
            const double d0 = xj[0][c] - x0, d1 = xj[1][c] - x1, d2 = xj[2][c] - x2;
            mn = fmin(mn, fma(d0, d0, fma(d1, d1, d2 * d2)));
        }
        if (bi == bj) {
            if (!(isfinite(x0) && isfinite(x1) && isfinite(x2))) atomicOr(&out->nonfinite, 1);
            atomicMin(&out->lo_key[0], order_key(x0));
            atomicMin(&out->lo_key[1], order_key(x1));
            atomicMin(&out->lo_key[2], order_key(x2));
            atomicMax(&out->hi_key[0], order_key(x0));
            atomicMax(&out->hi_key[1], order_key(x1));
            atomicMax(&out->hi_key[2], order_key(x2));
        }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) mn = fmin(mn, __shfl_xor(mn, m));
    if ((tid & 63) == 0 && mn >= 0.0)
        atomicMin(&out->min_d2_bits, (unsigned long long)__double_as_longlong(mn));
}

double key_to_double(unsigned long long k) {
    unsigned long long b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
    double d;
    std::memcpy(&d, &b, sizeof d);
    return d;
}

template <typename T>
mb_status direct_launch_t(const double *x, int64_t n, double scale, double *phi, hipStream_t s) {
    constexpr int IB = DirectLds<T>::IB;
    const int na = (int)((n + IB - 1) / IB);
    const int nb = (int)((n + kB - 1) / kB);
    const int nt = (int)((n + kKT - 1) / kKT);
    std::vector<int64_t> off(nb + 1, 0);
    for (int b = 0; b < nb; ++b)
        off[b + 1] = off[b] + (int64_t)units_a(b, IB, na) * (nt - (b >> 2));
    mb_status st;
    Scratch unit_tab;
    if ((st = unit_tab.alloc(sizeof(int64_t) * (nb + 1), s)) != MB_OK) return st;
    unit_offsets_kernel<<<1, 1, 0, s>>>(nb, nt, IB, na, unit_tab.as<int64_t>());
    MB_HIP(hipGetLastError());

    // the (i, j) table is built for a stripe of J blocks at a time
    const size_t per_b = (size_t)na * IB * kB * 3 * sizeof(T);
    int stripe = (int)std::max<size_t>(1, table_budget_bytes() / per_b);
    stripe = std::min(stripe, nb);
    Scratch pair_tab;
    if ((st = pair_tab.alloc(per_b * stripe, s)) != MB_OK) return st;

    const double s2 = scale * scale;
    const double out_scale = s2 * s2 * s2 * s2 * scale;  // scale^9, exact for a power of two
    for (int b0 = 0; b0 < nb; b0 += stripe) {
        const int b1 = std::min(nb, b0 + stripe);
        const int64_t u0 = off[b0], u1 = off[b1];
        pair_table_kernel<T><<<dim3((unsigned)na, (unsigned)(b1 - b0)), 256, 0, s>>>(
            x, (int)n, na, b0, scale, pair_tab.as<T>());
        const unsigned grid = (unsigned)std::min<int64_t>(u1 - u0, (int64_t)1 << 30);
        direct_kernel<T><<<grid, kThreads, 0, s>>>(x, (int)n, na, nb, nt, unit_tab.as<int64_t>(),
                                                   u0, u1, b0, pair_tab.as<T>(), scale,
                                                   out_scale, phi);
        MB_HIP(hipGetLastError());
    }
    return MB_OK;
}

}  // namespace

mb_status zero_doubles(double *p, int64_t n, hipStream_t s) {
    if (n <= 0) return MB_OK;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    zero_kernel<<<(unsigned)blocks, 256, 0, s>>>(p, n);
    MB_HIP(hipGetLastError());
    return MB_OK;
}

mb_status validate_points(const double *x, int64_t n, hipStream_t s, ValidateOut *out) {
    Scratch buf;
    mb_status st = buf.alloc(sizeof(ValidateOut), s);
    if (st != MB_OK) return st;
    ValidateOut *d = buf.as<ValidateOut>();
    validate_init_kernel<<<1, 1, 0, s>>>(d);
    MB_HIP(hipGetLastError());
    if (n > 0) {
        const int64_t nt = (n + kVT - 1) / kVT;
        if (nt > 65535) return fail(MB_ERR_UNSUPPORTED, "validate: n too large for the tile grid");
        validate_kernel<<<dim3((unsigned)nt, (unsigned)nt), kVT, 0, s>>>(x, (int)n, d);
        MB_HIP(hipGetLastError());
    }
    MB_HIP(hipMemcpyAsync(out, d, sizeof(ValidateOut), hipMemcpyDeviceToHost, s));
    MB_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < 3; ++c) {
        out->lo[c] = n > 0 ? key_to_double(out->lo_key[c]) : 0.0;
        out->hi[c] = n > 0 ? key_to_double(out->hi_key[c]) : 0.0;
    }
    return MB_OK;
}

mb_status direct_launch(const double *x, int64_t n, int prec, double scale, double *phi,
                        hipStream_t s) {
    mb_status st = zero_doubles(phi, n, s);
    if (st != MB_OK) return st;
    if (n < 3) return MB_OK;
    return prec == MB_FP64 ? direct_launch_t<double>(x, n, scale, phi, s)
                           : direct_launch_t<float>(x, n, scale, phi, s);
}

}  // namespace mb
