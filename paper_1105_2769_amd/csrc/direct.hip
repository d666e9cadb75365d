// Exhaustive per-particle Axilrod-Teller sum on gfx950 (the naive algorithm
// of Section 6, definition in Section 1), plus input validation.
//
// Work decomposition.  Points are cut into blocks of 64 (I and J roles) and
// tiles of 128 (K role).  A work unit is (I, J, K) with I <= J and the K tile
// reaching past J; together the units cover every unordered triple i < j < k
// exactly once, the global-index masks i < j, j < k, i < k inside a unit
// removing the rest.  One 512-thread workgroup (8 wave64s) runs one unit:
//
//   * lane l of every wave owns the two points k = K0 + l and K0 + 64 + l;
//   * wave w owns the eight points i = I0 + 8w .. I0 + 8w + 7 and keeps the
//     pair terms (i, k) of its 16 (i, k) combinations in registers;
//   * j runs over the J block in chunks of 16: the workgroup stages the
//     pair terms (i, j) (same for all lanes: LDS broadcast reads) and
//     (j, k) (one per lane) of the chunk in LDS.
//
// Inner step for one triple, with (a, qa, wa) the (i, j) terms, (g, qg, wg)
// the (i, k) terms and (b, qb, ob = 3/8 / b) the (j, k) terms:
//
//   phi = qb * psi,   psi = qa qg + ob (wa wg) (a + g - b)(b^2 - (a - g)^2)
//
// Per-particle sums: Phi_k += qb * sum_i psi (register), Phi_i += qb * psi
// (register array), Phi_j += sum over lanes and waves of qb * sum_i psi
// (LDS atomics into a per-(j, k) slot, reduced once per chunk).  The three
// sums are pushed to Phi with FP64 atomics once per unit.
#include "at_device.hpp"
#include "mb_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace mb {
namespace {

constexpr int kB = 64;           // points per I and J block
constexpr int kKT = 128;         // points per K tile (two per lane)
constexpr int kNW = 8;           // waves per workgroup
constexpr int kIPW = kB / kNW;   // i points per wave
constexpr int kJC = 16;          // j points per LDS chunk
constexpr int kThreads = kNW * 64;
constexpr int kXS = kB + kB + kKT;

template <typename T>
struct DirectLds {
    double xs[3][kXS];            // coordinates of the I block, J block and K tile
    T ua[kJC][kB], uq[kJC][kB], uw[kJC][kB];      // (i, j) terms of the chunk
    T cb[kJC][kKT], cq[kJC][kKT], co[kJC][kKT];   // (j, k) terms of the chunk
    double pj[kJC][kKT];          // Phi_j partials per (j, k), summed over waves
    double pjacc[kB];             // Phi_j of the unit
    double kacc[kKT];             // Phi_k of the unit
};

__device__ __forceinline__ void decode_unit(int64_t u, const int64_t *__restrict__ off, int nb,
                                            int nt, int &a, int &b, int &t) {
    int lo = 0, hi = nb;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= u) lo = mid; else hi = mid;
    }
    b = lo;
    int64_t rem = u - off[b];
    int tc = nt - (b >> 1);
    a = (int)(rem / tc);
    t = (b >> 1) + (int)(rem % tc);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

template <typename T>
__global__ __launch_bounds__(kThreads, 1) void direct_kernel(
    const double *__restrict__ x, int n, int nb, int nt, const int64_t *__restrict__ unit_off,
    int64_t n_units, double scale, double out_scale, double *__restrict__ phi) {
    __shared__ DirectLds<T> s;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    for (int64_t u = blockIdx.x; u < n_units; u += gridDim.x) {
        int a, b, t;
        decode_unit(u, unit_off, nb, nt, a, b, t);
        const int I0 = a * kB, J0 = b * kB, K0 = t * kKT;

        __syncthreads();  // the previous unit is done with the LDS
        if (tid < kXS) {
            int p = tid < kB ? I0 + tid : (tid < 2 * kB ? J0 + tid - kB : K0 + tid - 2 * kB);
            bool ok = p < n;
            s.xs[0][tid] = ok ? x[3 * (int64_t)p + 0] * scale : 0.0;
            s.xs[1][tid] = ok ? x[3 * (int64_t)p + 1] * scale : 0.0;
            s.xs[2][tid] = ok ? x[3 * (int64_t)p + 2] * scale : 0.0;
        }
        if (tid < kKT) s.kacc[tid] = 0.0;
        __syncthreads();

        // (i, k) pair terms of this wave, kept in registers for the whole unit
        T ag[kIPW][2], aq[kIPW][2], aw[kIPW][2];
        T acc_i[kIPW];
        double acc_i64[kIPW];
#pragma unroll
        for (int ii = 0; ii < kIPW; ++ii) {
            const int il = wave * kIPW + ii;
            const int i = I0 + il;
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const int kl = lane + 64 * kk;
                const int k = K0 + kl;
                double pa, pq, pw, pia;
                pair_terms(s.xs[0][2 * kB + kl] - s.xs[0][il], s.xs[1][2 * kB + kl] - s.xs[1][il],
                           s.xs[2][2 * kB + kl] - s.xs[2][il], (i < k) && (k < n), pa, pq, pw, pia);
                ag[ii][kk] = (T)pa;
                aq[ii][kk] = (T)pq;
                aw[ii][kk] = (T)pw;
            }
            acc_i[ii] = T(0);
            acc_i64[ii] = 0.0;
        }
        double acck0 = 0.0, acck1 = 0.0;

        for (int jc = 0; jc < kB / kJC; ++jc) {
            __syncthreads();  // previous chunk's readers are done
            for (int e = tid; e < kJC * kB; e += kThreads) {
                const int jj = e / kB, il = e % kB;
                const int jl = jc * kJC + jj;
                const int i = I0 + il, j = J0 + jl;
                double pa, pq, pw, pia;
                pair_terms(s.xs[0][kB + jl] - s.xs[0][il], s.xs[1][kB + jl] - s.xs[1][il],
                           s.xs[2][kB + jl] - s.xs[2][il], (i < j) && (j < n), pa, pq, pw, pia);
                s.ua[jj][il] = (T)pa;
                s.uq[jj][il] = (T)pq;
                s.uw[jj][il] = (T)pw;
            }
            for (int e = tid; e < kJC * kKT; e += kThreads) {
                const int jj = e / kKT, kl = e % kKT;
                const int jl = jc * kJC + jj;
                const int j = J0 + jl, k = K0 + kl;
                double pa, pq, pw, pia;
                pair_terms(s.xs[0][2 * kB + kl] - s.xs[0][kB + jl],
                           s.xs[1][2 * kB + kl] - s.xs[1][kB + jl],
                           s.xs[2][2 * kB + kl] - s.xs[2][kB + jl], (j < k) && (k < n), pa, pq, pw,
                           pia);
                s.cb[jj][kl] = (T)pa;
                s.cq[jj][kl] = (T)pq;
                s.co[jj][kl] = (T)(0.375 * pia);
                s.pj[jj][kl] = 0.0;
            }
            __syncthreads();

            for (int jj = 0; jj < kJC; ++jj) {
                const T b1 = s.cb[jj][lane], q1 = s.cq[jj][lane], o1 = s.co[jj][lane];
                const T b2 = s.cb[jj][lane + 64], q2 = s.cq[jj][lane + 64], o2 = s.co[jj][lane + 64];
                const T bb1 = b1 * b1, bb2 = b2 * b2;
                T s1 = T(0), s2 = T(0);
#pragma unroll
                for (int ii = 0; ii < kIPW; ++ii) {
                    const int il = wave * kIPW + ii;
                    const T al = s.ua[jj][il], qa = s.uq[jj][il], wa = s.uw[jj][il];
                    {
                        const T g = ag[ii][0];
                        const T d = al - g;
                        const T tt = (al + g) - b1;
                        const T m = fma(-d, d, bb1);
                        const T P = tt * m;
                        const T X = qa * aq[ii][0];
                        const T Y = (wa * aw[ii][0]) * P;
                        const T psi = fma(o1, Y, X);
                        s1 += psi;
                        acc_i[ii] = fma(q1, psi, acc_i[ii]);
                    }
                    {
                        const T g = ag[ii][1];
                        const T d = al - g;
                        const T tt = (al + g) - b2;
                        const T m = fma(-d, d, bb2);
                        const T P = tt * m;
                        const T X = qa * aq[ii][1];
                        const T Y = (wa * aw[ii][1]) * P;
                        const T psi = fma(o2, Y, X);
                        s2 += psi;
                        acc_i[ii] = fma(q2, psi, acc_i[ii]);
                    }
                }
                const T p1 = q1 * s1, p2 = q2 * s2;
                acck0 += (double)p1;
                acck1 += (double)p2;
                atomicAdd(&s.pj[jj][lane], (double)p1);
                atomicAdd(&s.pj[jj][lane + 64], (double)p2);
            }
            // fold the short binary32 partial sums into binary64
#pragma unroll
            for (int ii = 0; ii < kIPW; ++ii) {
                acc_i64[ii] += (double)acc_i[ii];
                acc_i[ii] = T(0);
            }
            __syncthreads();
            {
                // Phi_j of the chunk: sum the (j, k) slots over k
                const int row = tid >> 5, c = tid & 31;
                double v = s.pj[row][c] + s.pj[row][c + 32] + s.pj[row][c + 64] + s.pj[row][c + 96];
#pragma unroll
                for (int m = 16; m >= 1; m >>= 1) v += __shfl_xor(v, m);
                if (c == 0) s.pjacc[jc * kJC + row] = v;
            }
        }

#pragma unroll
        for (int ii = 0; ii < kIPW; ++ii) {
            const double v = wave_sum(acc_i64[ii]);
            const int i = I0 + wave * kIPW + ii;
            if (lane == 0 && i < n) atomicAdd(&phi[i], v * out_scale);
        }
        atomicAdd(&s.kacc[lane], acck0);
        atomicAdd(&s.kacc[lane + 64], acck1);
        __syncthreads();
        if (tid < kKT) {
            const int k = K0 + tid;
            if (k < n) atomicAdd(&phi[k], s.kacc[tid] * out_scale);
        } else if (tid < kKT + kB) {
            const int j = J0 + tid - kKT;
            if (j < n) atomicAdd(&phi[j], s.pjacc[tid - kKT] * out_scale);
        }
    }
}

// Prefix offsets of the unit list: units with J block b number (b + 1) * (nt - b / 2).
__global__ void unit_offsets_kernel(int nb, int nt, int64_t *__restrict__ off) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t acc = 0;
    off[0] = 0;
    for (int b = 0; b < nb; ++b) {
        acc += (int64_t)(b + 1) * (nt - (b >> 1));
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
    const int nb = (int)((n + kB - 1) / kB);
    const int nt = (int)((n + kKT - 1) / kKT);
    int64_t n_units = 0;
    for (int b = 0; b < nb; ++b) n_units += (int64_t)(b + 1) * (nt - (b >> 1));
    Scratch tab;
    if ((st = tab.alloc(sizeof(int64_t) * (nb + 1), s)) != MB_OK) return st;
    unit_offsets_kernel<<<1, 1, 0, s>>>(nb, nt, tab.as<int64_t>());
    MB_HIP(hipGetLastError());
    const unsigned grid = (unsigned)std::min<int64_t>(n_units, (int64_t)1 << 30);
    const double s2 = scale * scale;
    const double out_scale = s2 * s2 * s2 * s2 * scale;  // scale^9, exact for a power of two
    if (prec == MB_FP64)
        direct_kernel<double><<<grid, kThreads, 0, s>>>(x, (int)n, nb, nt, tab.as<int64_t>(),
                                                        n_units, scale, out_scale, phi);
    else
        direct_kernel<float><<<grid, kThreads, 0, s>>>(x, (int)n, nb, nt, tab.as<int64_t>(),
                                                       n_units, scale, out_scale, phi);
    MB_HIP(hipGetLastError());
    return MB_OK;
}

}  // namespace mb
