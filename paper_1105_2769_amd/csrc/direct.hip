// Exhaustive per-particle Axilrod-Teller sum on gfx950 (the naive algorithm
// of Section 6, definition in Section 1), plus input validation.  The tile
// code and its work decomposition are in direct_tile.hpp.
#include "direct_tile.hpp"
#include "mb_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

namespace mb {
namespace {

template <typename T>
__global__ __launch_bounds__(DirectLds<T>::TPB, DirectShape<T>::MINB) void direct_kernel(
    const double *__restrict__ x, int n, int na, int nb, int nt,
    const int64_t *__restrict__ unit_off, int64_t u_begin, int64_t u_end, int b0,
    const T *__restrict__ utab, double scale, double out_scale, double *__restrict__ phi) {
    constexpr int IB = DirectLds<T>::IB;
    __shared__ DirectLds<T> s;
    for (int64_t u = u_begin + blockIdx.x; u < u_end; u += gridDim.x) {
        int a, b, t;
        decode_unit(u, unit_off, nb, nt, DirectLds<T>::KR, a, b, t);
        direct_unit<T>(s, x, n, a, b, t, utab + ((int64_t)(b - b0) * na + a) * (IB * kB * kPairVals),
                       scale, out_scale, phi);
    }
}

// The exhaustive sum's units in the fixed-order mode: unit u writes its row
// of IB + JB + KT sums (tile_unit) to rows[(u - u_begin) * W].
template <typename T>
__global__ __launch_bounds__(DirectLds<T>::TPB, DirectShape<T>::MINB) void direct_rows_kernel(
    const double *__restrict__ x, int n, int na, int nb, int nt,
    const int64_t *__restrict__ unit_off, int64_t u_begin, int64_t u_end, int b0,
    const T *__restrict__ utab, double *__restrict__ rows) {
    constexpr int IB = DirectLds<T>::IB;
    constexpr int W = IB + kB + DirectLds<T>::KT;
    __shared__ DirectLds<T> s;
    __shared__ double pjl[DirectShape<T>::NW * DirectShape<T>::JC * 64];
    for (int64_t u = u_begin + blockIdx.x; u < u_end; u += gridDim.x) {
        int a, b, t;
        decode_unit(u, unit_off, nb, nt, DirectLds<T>::KR, a, b, t);
        direct_unit<T, const T *, true>(
            s, x, n, a, b, t, utab + ((int64_t)(b - b0) * na + a) * (IB * kB * kPairVals), 1.0,
            1.0, rows + (u - u_begin) * W, pjl);
    }
}

// Sums of the unit rows of J blocks [b0, b1) (units [off[b0], off[b1]),
// row r = u - off[b0]) into phi, one launch per role of a point: as i, as j,
// as k.  A workgroup owns one block of points and adds, for each point, the
// rows that hold it in a fixed order split into kRT / columns interleaved
// streams; the streams are added in stream order and the total is added to
// phi.  Launches on one stream run in order, so every point's result is the
// same sequence of additions on every call.
constexpr int kRT = 256;  // threads of the row-sum kernels

// As i: block a, rows of units (a, b, t) in order of b, then t.
template <int IB, int KR, int W>
__global__ __launch_bounds__(kRT) void rows_i_kernel(const double *__restrict__ rows,
                                                     const int64_t *__restrict__ off, int n, int na,
                                                     int nt, int b0, int b1,
                                                     double *__restrict__ phi) {
    constexpr int S = kRT / IB;
    static_assert(kRT % IB == 0, "whole streams");
    __shared__ double part[S][IB];
    const int a = blockIdx.x, c = threadIdx.x % IB, st = threadIdx.x / IB;
    const int64_t r_first = off[b0];
    double acc = 0.0;
    for (int b = b0; b < b1; ++b) {
        if (a >= units_a(b, IB, na)) continue;
        const int tc = nt - b / KR;
        const int64_t base = off[b] - r_first + (int64_t)a * tc;
#pragma unroll 4
        for (int q = st; q < tc; q += S) acc += rows[(base + q) * W + c];
    }
    part[st][c] = acc;
    __syncthreads();
    if (st == 0) {
        double v = part[0][c];
#pragma unroll
        for (int k = 1; k < S; ++k) v += part[k][c];
        const int64_t i = (int64_t)a * IB + c;
        if (i < n) phi[i] += v;
    }
}

// As j: J block b0 + blockIdx.x, its units in unit order.
template <int IB, int JB, int W>
__global__ __launch_bounds__(kRT) void rows_j_kernel(const double *__restrict__ rows,
                                                     const int64_t *__restrict__ off, int n, int b0,
                                                     double *__restrict__ phi) {
    constexpr int S = kRT / JB;
    static_assert(kRT % JB == 0, "whole streams");
    __shared__ double part[S][JB];
    const int b = b0 + blockIdx.x, c = threadIdx.x % JB, st = threadIdx.x / JB;
    const int64_t r_first = off[b0];
    const int64_t r0 = off[b] - r_first, r1 = off[b + 1] - r_first;
    double acc = 0.0;
#pragma unroll 4
    for (int64_t r = r0 + st; r < r1; r += S) acc += rows[r * W + IB + c];
    part[st][c] = acc;
    __syncthreads();
    if (st == 0) {
        double v = part[0][c];
#pragma unroll
        for (int k = 1; k < S; ++k) v += part[k][c];
        const int64_t j = (int64_t)b * JB + c;
        if (j < n) phi[j] += v;
    }
}

// As k: K tile t, rows of units (a, b, t) in order of b, then a.
template <int IB, int JB, int KT, int KR, int W>
__global__ __launch_bounds__(kRT) void rows_k_kernel(const double *__restrict__ rows,
                                                     const int64_t *__restrict__ off, int n, int na,
                                                     int nt, int b0, int b1,
                                                     double *__restrict__ phi) {
    constexpr int S = kRT / KT;
    static_assert(kRT % KT == 0, "whole streams");
    __shared__ double part[S][KT];
    const int t = blockIdx.x, c = threadIdx.x % KT, st = threadIdx.x / KT;
    const int64_t r_first = off[b0];
    const int b_end = min(b1, KR * (t + 1));  // k > j needs b / KR <= t
    double acc = 0.0;
    for (int b = b0; b < b_end; ++b) {
        const int tb = b / KR, tc = nt - tb;
        const int n_a = units_a(b, IB, na);
        const int64_t base = off[b] - r_first + (t - tb);
#pragma unroll 4
        for (int a = st; a < n_a; a += S) acc += rows[(base + (int64_t)a * tc) * W + IB + JB + c];
    }
    part[st][c] = acc;
    __syncthreads();
    if (st == 0) {
        double v = part[0][c];
#pragma unroll
        for (int k = 1; k < S; ++k) v += part[k][c];
        const int64_t kk = (int64_t)t * KT + c;
        if (kk < n) phi[kk] += v;
    }
}

// Near-field refinement of the binary32 tiles.  Each pair term is rounded to
// binary32 once and reused by every triple through that pair, so its
// rounding error does not average out over those triples; through the
// difference of two squared sides in the law of cosines it is largest for
// the compact triangles of near neighbours, which also carry the largest
// phi.  For every triple whose three sides are shorter than r_c the
// refinement adds phi in binary64 minus the binary32 value the tiles
// computed for it (same pair terms, same operations: tile_psi), so those
// triples end up in binary64.  The identity holds for any subset of
// triples, each taken at most once, so the neighbour cap below only limits
// how much is refined.
constexpr int kNearMax = 64;  // forward neighbours kept per point
constexpr int kPointGroup = 8;     // flagged points per workgroup of point_group_kernel
constexpr int kPointGroupMin = 4;  // more flagged points than this go to point_group_kernel
constexpr int kPointKChunk = 2048;  // k points per workgroup of the point-wise kernels

// Forward neighbours v > u with |x_v - x_u| < r_c, in index order, at most
// kNearMax per point.
// One wave per point u: the lanes test 64 consecutive candidates v at a
// time, in index order, and a ballot appends the hits in that order.
__global__ __launch_bounds__(256) void near_list_kernel(const double *__restrict__ x, int n,
                                                        double rc2, int32_t *__restrict__ cnt,
                                                        int32_t *__restrict__ nbr) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int u = (int)(g >> 6), lane = (int)(g & 63);
    if (u >= n) return;  // whole waves: u is uniform in a wave
    const double x0 = x[3 * (int64_t)u], x1 = x[3 * (int64_t)u + 1], x2 = x[3 * (int64_t)u + 2];
    int c = 0;
    for (int v0 = u + 1; v0 < n && c < kNearMax; v0 += 64) {
        const int v = v0 + lane;
        bool hit = false;
        if (v < n) {
            const double dx = x[3 * (int64_t)v] - x0, dy = x[3 * (int64_t)v + 1] - x1,
                         dz = x[3 * (int64_t)v + 2] - x2;
            hit = fma(dx, dx, fma(dy, dy, dz * dz)) < rc2;
        }
        const unsigned long long mask = __ballot(hit);
        if (hit) {
            const int pos = c + __popcll(mask & ((1ull << lane) - 1ull));
            if (pos < kNearMax) nbr[(int64_t)u * kNearMax + pos] = v;
        }
        c += __popcll(mask);
    }
    if (lane == 0) cnt[u] = min(c, kNearMax);
}

// Every triple u < v < w with v, w in u's list and |x_w - x_v| < r_c (so each
// triple once, from its smallest index).  One wave per point u, lane l the
// l-th forward neighbour v of u: the lane
// takes the pairs (v, w) with w a later neighbour in u's list.  (One thread
// per point ran every pair of the list in sequence, which set the kernel's
// duration for the small sets of a serving request.)
__global__ __launch_bounds__(256) void near_fix_kernel(const double *__restrict__ x, int n,
                                                       double scale, double out_scale, double rc2,
                                                       const int32_t *__restrict__ cnt,
                                                       const int32_t *__restrict__ nbr,
                                                       double *__restrict__ phi,
                                                       double *__restrict__ mag) {
    static_assert(kNearMax == 64, "one lane per neighbour slot");
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int u = (int)(g >> 6), p = (int)(g & 63);
    if (u >= n) return;  // whole waves: u is uniform in a wave
    const int c = cnt[u];
    const int32_t *list = nbr + (int64_t)u * kNearMax;
    double xu[3];
    for (int d = 0; d < 3; ++d) xu[d] = x[3 * (int64_t)u + d] * scale;
    double acc_u = 0.0, mag_u = 0.0;
    for (int q = p + 1; q < c; ++q) {
        int v = list[p], w = list[q];
        if (v > w) {
            const int tmp = v;
            v = w;
            w = tmp;
        }
        double xv[3], xw[3], r2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double dv = x[3 * (int64_t)w + d] - x[3 * (int64_t)v + d];
            r2 = fma(dv, dv, r2);
            xv[d] = x[3 * (int64_t)v + d] * scale;
            xw[d] = x[3 * (int64_t)w + d] * scale;
        }
        if (r2 >= rc2) continue;
        // pair terms as the tiles form them: (i, j) = (u, v), (i, k) = (u, w),
        // (j, k) = (v, w), each from the difference of scaled coordinates
        double a1, q1, w1, i1, a2, q2, w2, i2, a3, q3, w3, i3;
        pair_terms(xv[0] - xu[0], xv[1] - xu[1], xv[2] - xu[2], true, a1, q1, w1, i1);
        pair_terms(xw[0] - xu[0], xw[1] - xu[1], xw[2] - xu[2], true, a2, q2, w2, i2);
        pair_terms(xw[0] - xv[0], xw[1] - xv[1], xw[2] - xv[2], true, a3, q3, w3, i3);
        const double f64 = phi_from_pairs<double>(a1, q1, w1, a2, q2, w2, a3, q3, w3);
        const float cb = (float)a3;
        const float psi = tile_psi<float>((float)a1, (float)a2, (float)w2, cb, cb * cb,
                                          (float)(0.375 * i3));
        const double f32 = (double)(float)q3 * (double)(float)w1 * (double)psi;
        const double dlt = (f64 - f32) * out_scale;
        const double m = fabs(f64) * out_scale;
        acc_u += dlt;
        mag_u += m;
        atomicAdd(&phi[v], dlt);
        atomicAdd(&phi[w], dlt);
        atomicAdd(&mag[v], m);
        atomicAdd(&mag[w], m);
    }
    acc_u = wave_sum(acc_u);
    mag_u = wave_sum(mag_u);
    if (p == 0) {
        atomicAdd(&phi[u], acc_u);
        atomicAdd(&mag[u], mag_u);
    }
}

// Points whose binary32 result may miss the relative bar: |Phi| small next
// to the magnitude of their near-field terms (the binary32 error of a point
// stays below about 1.2e-7 of that magnitude on the workloads measured).
__global__ void flag_kernel(const double *__restrict__ phi, const double *__restrict__ mag, int n,
                            double ratio, int32_t *__restrict__ list, int32_t *__restrict__ count,
                            int cap) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    if (fabs(phi[p]) < ratio * mag[p]) {
        const int slot = atomicAdd(count, 1);
        if (slot < cap) list[slot] = p;
    }
}

// Phi of listed points in binary64, one workgroup per (tile of 256 j, point,
// chunk of kPointKChunk k): thread j sums phi(p, j, k) over the chunk's
// k > j (k != p), with the (p, k) pair terms staged in LDS per tile of k.
// The k chunks spread the triangle j < k over many workgroups.
__global__ __launch_bounds__(256) void point_fp64_kernel(const double *__restrict__ x, int n,
                                                         const int32_t *__restrict__ list,
                                                         const int32_t *__restrict__ count,
                                                         double *__restrict__ out) {
    const int f = blockIdx.y;
    // grid sized for the cap; the list may be shorter, and longer lists go to
    // point_group_kernel
    if (f >= *count || *count > kPointGroupMin) return;
    const int p = list[f];
    const int j0 = blockIdx.x * 256;
    const int j = j0 + threadIdx.x;
    // k chunk z of kPointKChunk points; only k > j contribute
    const int kbeg = max(j0, (int)blockIdx.z * kPointKChunk);
    const int kend = min(n, ((int)blockIdx.z + 1) * kPointKChunk);
    if (kbeg >= kend) return;
    __shared__ double xk[3][256], ak[256], qk[256], wk[256];
    const double xp0 = x[3 * (int64_t)p], xp1 = x[3 * (int64_t)p + 1], xp2 = x[3 * (int64_t)p + 2];
    const bool jok = j < n && j != p;
    double xj0 = 0.0, xj1 = 0.0, xj2 = 0.0, a1 = 1.0, q1 = 0.0, w1 = 0.0, i1;
    if (jok) {
        xj0 = x[3 * (int64_t)j];
        xj1 = x[3 * (int64_t)j + 1];
        xj2 = x[3 * (int64_t)j + 2];
        pair_terms(xj0 - xp0, xj1 - xp1, xj2 - xp2, true, a1, q1, w1, i1);
    }
    double acc = 0.0;
    for (int k0 = kbeg; k0 < kend; k0 += 256) {
        __syncthreads();
        {
            const int k = k0 + threadIdx.x;
            const bool kok = k < kend && k != p;
            double d0 = 0.0, d1 = 0.0, d2 = 0.0;
            if (k < kend) {
                d0 = x[3 * (int64_t)k];
                d1 = x[3 * (int64_t)k + 1];
                d2 = x[3 * (int64_t)k + 2];
            }
            xk[0][threadIdx.x] = d0;
            xk[1][threadIdx.x] = d1;
            xk[2][threadIdx.x] = d2;
            double a, q, w, ia;
            pair_terms(d0 - xp0, d1 - xp1, d2 - xp2, kok, a, q, w, ia);
            ak[threadIdx.x] = a;
            qk[threadIdx.x] = q;
            wk[threadIdx.x] = w;
        }
        __syncthreads();
        if (jok) {
            const int lim = min(256, kend - k0);
            for (int t = 0; t < lim; ++t) {
                const int k = k0 + t;
                if (k <= j || qk[t] == 0.0) continue;
                double a3, q3, w3, i3;
                pair_terms(xk[0][t] - xj0, xk[1][t] - xj1, xk[2][t] - xj2, true, a3, q3, w3, i3);
                acc += phi_from_pairs<double>(a1, q1, w1, ak[t], qk[t], wk[t], a3, q3, w3);
            }
        }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m);
    if ((threadIdx.x & 63) == 0) atomicAdd(&out[f], acc);
}

// The same sums for kPointGroup flagged points at a time, used when more
// than kPointGroupMin points are flagged: the (j, k) pair terms, which do not
// depend on the point, are formed once per (j, k) and serve the whole group.
// Workgroup (x, y, z): j in tile x, points kPointGroup y .. kPointGroup y + 7,
// k in chunk z.
__global__ __launch_bounds__(256) void point_group_kernel(const double *__restrict__ x, int n,
                                                          const int32_t *__restrict__ list,
                                                          const int32_t *__restrict__ count,
                                                          double *__restrict__ out) {
    constexpr int G = kPointGroup;
    const int cnt = *count;
    const int f0 = blockIdx.y * G;
    if (cnt <= kPointGroupMin || f0 >= cnt) return;
    const int j0 = blockIdx.x * 256;
    const int j = j0 + threadIdx.x;
    const int kbeg = max(j0, (int)blockIdx.z * kPointKChunk);
    const int kend = min(n, ((int)blockIdx.z + 1) * kPointKChunk);
    if (kbeg >= kend) return;
    __shared__ double xk[3][256];
    __shared__ double ak[G][256], qk[G][256], wk[G][256];
    __shared__ double xp[3][G];
    __shared__ int pidx[G];
    if (threadIdx.x < G) {
        const int f = f0 + threadIdx.x;
        const int p = f < cnt ? list[f] : -1;  // -1: an empty slot of the group
        pidx[threadIdx.x] = p;
        for (int c = 0; c < 3; ++c) xp[c][threadIdx.x] = p >= 0 ? x[3 * (int64_t)p + c] : 0.0;
    }
    __syncthreads();
    double xj0 = 0.0, xj1 = 0.0, xj2 = 0.0;
    if (j < n) {
        xj0 = x[3 * (int64_t)j];
        xj1 = x[3 * (int64_t)j + 1];
        xj2 = x[3 * (int64_t)j + 2];
    }
    // (p, j) terms of the group's points; masked (zero) for j = p, j >= n and
    // empty slots
    double a1[G], q1[G], w1[G], acc[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        double i1;
        pair_terms(xj0 - xp[0][g], xj1 - xp[1][g], xj2 - xp[2][g],
                   j < n && pidx[g] >= 0 && j != pidx[g], a1[g], q1[g], w1[g], i1);
        acc[g] = 0.0;
    }
    for (int k0 = kbeg; k0 < kend; k0 += 256) {
        __syncthreads();
        {
            const int k = k0 + threadIdx.x;
            double d0 = 0.0, d1 = 0.0, d2 = 0.0;
            if (k < kend) {
                d0 = x[3 * (int64_t)k];
                d1 = x[3 * (int64_t)k + 1];
                d2 = x[3 * (int64_t)k + 2];
            }
            xk[0][threadIdx.x] = d0;
            xk[1][threadIdx.x] = d1;
            xk[2][threadIdx.x] = d2;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                double a, q, w, ia;
                pair_terms(d0 - xp[0][g], d1 - xp[1][g], d2 - xp[2][g],
                           k < kend && pidx[g] >= 0 && k != pidx[g], a, q, w, ia);
                ak[g][threadIdx.x] = a;
                qk[g][threadIdx.x] = q;
                wk[g][threadIdx.x] = w;
            }
        }
        __syncthreads();
        if (j < n) {
            const int lim = min(256, kend - k0);
            for (int t = 0; t < lim; ++t) {
                if (k0 + t <= j) continue;
                double a3, q3, w3, i3;
                pair_terms(xk[0][t] - xj0, xk[1][t] - xj1, xk[2][t] - xj2, true, a3, q3, w3, i3);
#pragma unroll
                for (int g = 0; g < G; ++g)
                    acc[g] += phi_from_pairs<double>(a1[g], q1[g], w1[g], ak[g][t], qk[g][t],
                                                     wk[g][t], a3, q3, w3);
            }
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        double v = acc[g];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
        if ((threadIdx.x & 63) == 0 && f0 + g < cnt) atomicAdd(&out[f0 + g], v);
    }
}

__global__ void zero_i32_kernel(int32_t *p) { *p = 0; }

__global__ void scatter_points_kernel(const int32_t *__restrict__ list, const int32_t *count,
                                      int cap, const double *__restrict__ vals,
                                      double *__restrict__ phi) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < min(*count, cap)) phi[list[f]] = vals[f];
}

// Prefix offsets of the unit list, units of J block b: units_a(b) * (nt - b / kr).
__global__ void unit_offsets_kernel(int nb, int nt, int kr, int ib, int na,
                                    int64_t *__restrict__ off) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t acc = 0;
    off[0] = 0;
    for (int b = 0; b < nb; ++b) {
        acc += (int64_t)units_a(b, ib, na) * (nt - b / kr);
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

// Units of the exhaustive sum of N points with tile type T, and the bytes
// of its (i, j) table over J blocks [0, nb).
template <typename T>
int64_t direct_units(int64_t n) {
    constexpr int IB = DirectLds<T>::IB, KR = DirectLds<T>::KR, KT = DirectLds<T>::KT;
    const int na = (int)((n + IB - 1) / IB), nb = (int)((n + kB - 1) / kB);
    const int nt = (int)((n + KT - 1) / KT);
    int64_t u = 0;
    for (int b = 0; b < nb; ++b) u += (int64_t)units_a(b, IB, na) * (nt - b / KR);
    return u;
}

template <typename T>
constexpr size_t direct_table_bytes(int64_t n) {
    return (size_t)((n + DirectLds<T>::IB - 1) / DirectLds<T>::IB) *
           (size_t)((n + kB - 1) / kB) * DirectLds<T>::IB * kB * kPairVals * sizeof(T);
}

// The exhaustive sum with its unit offsets and (i, j) table in caller-given
// device memory (`offsets`: nb + 1 int64, `table`: the whole table), one
// stripe; phi must already be zero.
template <typename T>
mb_status direct_launch_into(const double *x, int64_t n, double scale, double *phi,
                             int64_t *offsets, T *table, hipStream_t s) {
    constexpr int IB = DirectLds<T>::IB, KR = DirectLds<T>::KR, KT = DirectLds<T>::KT;
    const int na = (int)((n + IB - 1) / IB), nb = (int)((n + kB - 1) / kB);
    const int nt = (int)((n + KT - 1) / KT);
    unit_offsets_kernel<<<1, 1, 0, s>>>(nb, nt, KR, IB, na, offsets);
    pair_table_kernel<T><<<dim3((unsigned)na, (unsigned)nb), 256, 0, s>>>(x, (int)n, na, 0, scale,
                                                                          table);
    const double s2 = scale * scale;
    const double out_scale = s2 * s2 * s2 * s2 * scale;
    const int64_t units = direct_units<T>(n);
    direct_kernel<T><<<(unsigned)std::min<int64_t>(units, (int64_t)1 << 30), DirectLds<T>::TPB, 0,
                       s>>>(x, (int)n, na, nb, nt, offsets, 0, units, 0, table, scale, out_scale,
                            phi);
    MB_HIP(hipGetLastError());
    return MB_OK;
}

template <typename T>
mb_status direct_launch_t(const double *x, int64_t n, double scale, double *phi, hipStream_t s) {
    constexpr int IB = DirectLds<T>::IB;
    const int na = (int)((n + IB - 1) / IB);
    const int nb = (int)((n + kB - 1) / kB);
    constexpr int KR = DirectLds<T>::KR, KT = DirectLds<T>::KT;
    const int nt = (int)((n + KT - 1) / KT);
    std::vector<int64_t> off(nb + 1, 0);
    for (int b = 0; b < nb; ++b)
        off[b + 1] = off[b] + (int64_t)units_a(b, IB, na) * (nt - b / KR);
    mb_status st;
    Scratch unit_tab;
    if ((st = unit_tab.alloc(sizeof(int64_t) * (nb + 1), s)) != MB_OK) return st;

    // the (i, j) table is built for a stripe of J blocks at a time
    const size_t per_b = (size_t)na * IB * kB * kPairVals * sizeof(T);
    int stripe = (int)std::max<size_t>(1, table_budget_bytes() / per_b);
    stripe = std::min(stripe, nb);
    Scratch pair_tab;
    if ((st = pair_tab.alloc(per_b * stripe, s)) != MB_OK) return st;
    if (stripe == nb)
        return direct_launch_into<T>(x, n, scale, phi, unit_tab.as<int64_t>(), pair_tab.as<T>(), s);

    unit_offsets_kernel<<<1, 1, 0, s>>>(nb, nt, KR, IB, na, unit_tab.as<int64_t>());
    MB_HIP(hipGetLastError());
    const double s2 = scale * scale;
    const double out_scale = s2 * s2 * s2 * s2 * scale;  // scale^9, exact for a power of two
    for (int b0 = 0; b0 < nb; b0 += stripe) {
        const int b1 = std::min(nb, b0 + stripe);
        const int64_t u0 = off[b0], u1 = off[b1];
        pair_table_kernel<T><<<dim3((unsigned)na, (unsigned)(b1 - b0)), 256, 0, s>>>(
            x, (int)n, na, b0, scale, pair_tab.as<T>());
        const unsigned grid = (unsigned)std::min<int64_t>(u1 - u0, (int64_t)1 << 30);
        direct_kernel<T><<<grid, DirectLds<T>::TPB, 0, s>>>(x, (int)n, na, nb, nt, unit_tab.as<int64_t>(),
                                                   u0, u1, b0, pair_tab.as<T>(), scale,
                                                   out_scale, phi);
        MB_HIP(hipGetLastError());
    }
    return MB_OK;
}

// Device memory of mb_eval_direct_noalloc: the unit offsets (first 256
// bytes) and the (i, j) table of either tile type for N <= kNoAllocMaxN.
// In host code `scratch` only names the array; its device address on the
// current GPU comes from hipGetSymbolAddress (noalloc_scratch below).
constexpr size_t kNoAllocOffsets = 256;
constexpr size_t kNoAllocBytes =
    kNoAllocOffsets + (direct_table_bytes<double>(kNoAllocMaxN) > direct_table_bytes<float>(kNoAllocMaxN)
                           ? direct_table_bytes<double>(kNoAllocMaxN)
                           : direct_table_bytes<float>(kNoAllocMaxN));
static_assert(((kNoAllocMaxN + kB - 1) / kB + 1) * 8 <= kNoAllocOffsets, "offsets fit");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Address of `scratch` on the current device, looked up once per device.
mb_status noalloc_scratch(unsigned char **out) {
    static std::mutex mu;
    static unsigned char *ptr[64] = {};
    int dev = 0;
    MB_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(MB_ERR_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> g(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = ptr[dev];
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

mb_status validate_enqueue(const double *x, int64_t n, hipStream_t s, ValidateOut *dev,
                           ValidateOut *out) {
    validate_init_kernel<<<1, 1, 0, s>>>(dev);
    MB_HIP(hipGetLastError());
    if (n > 0) {
        const int64_t nt = (n + kVT - 1) / kVT;
        if (nt > 65535) return fail(MB_ERR_UNSUPPORTED, "validate: n too large for the tile grid");
        validate_kernel<<<dim3((unsigned)nt, (unsigned)nt), kVT, 0, s>>>(x, (int)n, dev);
        MB_HIP(hipGetLastError());
    }
    MB_HIP(hipMemcpyAsync(out, dev, sizeof(ValidateOut), hipMemcpyDeviceToHost, s));
    return MB_OK;
}

void validate_decode(ValidateOut *out, int64_t n) {
    for (int c = 0; c < 3; ++c) {
        out->lo[c] = n > 0 ? key_to_double(out->lo_key[c]) : 0.0;
        out->hi[c] = n > 0 ? key_to_double(out->hi_key[c]) : 0.0;
    }
}

mb_status validate_points(const double *x, int64_t n, hipStream_t s, ValidateOut *out) {
    Scratch buf;
    mb_status st = buf.alloc(sizeof(ValidateOut), s);
    if (st != MB_OK) return st;
    if ((st = validate_enqueue(x, n, s, buf.as<ValidateOut>(), out)) != MB_OK) return st;
    MB_HIP(hipStreamSynchronize(s));
    validate_decode(out, n);
    return MB_OK;
}

mb_status near_refine_launch(const double *x, int64_t n, double scale, double r_fix, double *phi,
                             double *mag, hipStream_t s) {
    if (n < 3 || !(r_fix > 0.0)) return MB_OK;
    Scratch lists;
    mb_status st = lists.alloc(sizeof(int32_t) * (size_t)n * (kNearMax + 1), s);
    if (st != MB_OK) return st;
    int32_t *cnt = lists.as<int32_t>();
    int32_t *nbr = cnt + n;
    const unsigned wave_blocks = (unsigned)((n * (int64_t)kNearMax + 255) / 256);  // a wave per point
    const double rc2 = r_fix * r_fix;
    const double s2 = scale * scale;
    const double out_scale = s2 * s2 * s2 * s2 * scale;
    if ((st = zero_doubles(mag, n, s)) != MB_OK) return st;
    near_list_kernel<<<wave_blocks, 256, 0, s>>>(x, (int)n, rc2, cnt, nbr);
    near_fix_kernel<<<wave_blocks, 256, 0, s>>>(x, (int)n, scale, out_scale, rc2, cnt, nbr, phi,
                                                 mag);
    MB_HIP(hipGetLastError());
    return MB_OK;
}

int64_t point_fix_cap(int64_t n) {
    return std::min<int64_t>(65535, std::max<int64_t>(kPointFixMin, n / kPointFixShare));
}

mb_status point_fp64_enqueue(const double *x, int64_t n, const double *mag, double *phi,
                             hipStream_t s, int32_t *count_host) {
    *count_host = 0;
    if (n < 3) return MB_OK;
    const int cap = (int)point_fix_cap(n);
    Scratch buf;
    mb_status st = buf.alloc(sizeof(int32_t) * (cap + 1) + sizeof(double) * cap + 64, s);
    if (st != MB_OK) return st;
    int32_t *count = buf.as<int32_t>();
    int32_t *list = count + 1;
    double *vals = reinterpret_cast<double *>(
        (reinterpret_cast<uintptr_t>(list + cap) + 15) & ~(uintptr_t)15);
    zero_i32_kernel<<<1, 1, 0, s>>>(count);
    if ((st = zero_doubles(vals, cap, s)) != MB_OK) return st;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    flag_kernel<<<blocks, 256, 0, s>>>(phi, mag, (int)n, kPointFixRatio, list, count, cap);
    // one of the two kernels does the work, depending on the device-side count
    const unsigned kchunks = (unsigned)((n + kPointKChunk - 1) / kPointKChunk);
    point_fp64_kernel<<<dim3(blocks, (unsigned)cap, kchunks), 256, 0, s>>>(x, (int)n, list, count,
                                                                          vals);
    point_group_kernel<<<dim3(blocks, (unsigned)((cap + kPointGroup - 1) / kPointGroup), kchunks),
                         256, 0, s>>>(x, (int)n, list, count, vals);
    scatter_points_kernel<<<(unsigned)((cap + 255) / 256), 256, 0, s>>>(list, count, cap, vals, phi);
    MB_HIP(hipGetLastError());
    MB_HIP(hipMemcpyAsync(count_host, count, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    return MB_OK;
}

mb_status point_fp64_redo_all(const double *x, int64_t n, double *phi, hipStream_t s) {
    mb_status st = zero_doubles(phi, n, s);
    if (st != MB_OK) return st;
    return direct_launch_t<double>(x, n, 1.0, phi, s);
}

mb_status direct_launch_noalloc(const double *x, int64_t n, int prec, double *phi, hipStream_t s) {
    if (n > kNoAllocMaxN) return fail(MB_ERR_UNSUPPORTED, "n above the no-allocation maximum");
    unsigned char *base = nullptr;
    mb_status st = noalloc_scratch(&base);
    if (st != MB_OK) return st;
    if ((st = zero_doubles(phi, n, s)) != MB_OK) return st;
    if (n < 3) return MB_OK;
    int64_t *off = reinterpret_cast<int64_t *>(base);
    if (prec == MB_FP64)
        return direct_launch_into<double>(x, n, 1.0, phi, off,
                                          reinterpret_cast<double *>(base + kNoAllocOffsets), s);
    return direct_launch_into<float>(x, n, 1.0, phi, off,
                                     reinterpret_cast<float *>(base + kNoAllocOffsets), s);
}

mb_status direct_launch(const double *x, int64_t n, int prec, double scale, double *phi,
                        hipStream_t s, double r_fix, int64_t *recomputed) {
    if (recomputed) *recomputed = 0;
    mb_status st = zero_doubles(phi, n, s);
    if (st != MB_OK) return st;
    if (n < 3) return MB_OK;
    if (prec == MB_FP64) return direct_launch_t<double>(x, n, scale, phi, s);
    if ((st = direct_launch_t<float>(x, n, scale, phi, s)) != MB_OK) return st;
    if (!(r_fix > 0.0)) return MB_OK;
    Scratch mag;
    if ((st = mag.alloc(sizeof(double) * (size_t)n, s)) != MB_OK) return st;
    if ((st = near_refine_launch(x, n, scale, r_fix, phi, mag.as<double>(), s)) != MB_OK) return st;
    int32_t flagged = 0;
    if ((st = point_fp64_enqueue(x, n, mag.as<double>(), phi, s, &flagged)) != MB_OK) return st;
    MB_HIP(hipStreamSynchronize(s));
    if (recomputed) *recomputed = flagged;
    if (flagged <= point_fix_cap(n)) return MB_OK;
    // too many strongly cancelling points for point-wise repair
    if (recomputed) *recomputed = n;
    return point_fp64_redo_all(x, n, phi, s);
}

// The binary64 exhaustive sum in the fixed-order mode: per stripe of J
// blocks, the units write their rows, then the three row-sum kernels add
// them into phi (zeroed here).  A stripe holds as many J blocks as keep its
// (i, j) table plus its rows within `budget` bytes, at least one.
mb_status direct_launch_ordered(const double *x, int64_t n, double *phi, size_t budget,
                                hipStream_t s) {
    using T = double;
    constexpr int IB = DirectLds<T>::IB, KR = DirectLds<T>::KR, KT = DirectLds<T>::KT;
    constexpr int W = IB + kB + KT;
    mb_status st = zero_doubles(phi, n, s);
    if (st != MB_OK || n < 3) return st;
    const int na = (int)((n + IB - 1) / IB), nb = (int)((n + kB - 1) / kB);
    const int nt = (int)((n + KT - 1) / KT);
    std::vector<int64_t> off(nb + 1, 0);
    for (int b = 0; b < nb; ++b)
        off[b + 1] = off[b] + (int64_t)units_a(b, IB, na) * (nt - b / KR);
    const size_t per_b = (size_t)na * IB * kB * kPairVals * sizeof(T);
    const size_t row_bytes = (size_t)W * sizeof(double);
    std::vector<int> cut{0};
    size_t tab_max = 0, rows_max = 0;
    for (int b0 = 0; b0 < nb;) {
        auto need = [&](int e) { return per_b * (e - b0) + (size_t)(off[e] - off[b0]) * row_bytes; };
        int b1 = b0 + 1;
        while (b1 < nb && need(b1 + 1) <= budget) ++b1;
        tab_max = std::max(tab_max, per_b * (b1 - b0));
        rows_max = std::max(rows_max, (size_t)(off[b1] - off[b0]));
        cut.push_back(b1);
        b0 = b1;
    }
    Scratch unit_tab, pair_tab, rows;
    if ((st = unit_tab.alloc(sizeof(int64_t) * (nb + 1), s)) != MB_OK) return st;
    if ((st = pair_tab.alloc(tab_max, s)) != MB_OK) return st;
    if ((st = rows.alloc(rows_max * row_bytes, s)) != MB_OK) return st;
    const int64_t *doff = unit_tab.as<int64_t>();
    unit_offsets_kernel<<<1, 1, 0, s>>>(nb, nt, KR, IB, na, unit_tab.as<int64_t>());
    MB_HIP(hipGetLastError());
    for (size_t c = 0; c + 1 < cut.size(); ++c) {
        const int b0 = cut[c], b1 = cut[c + 1];
        const int64_t u0 = off[b0], u1 = off[b1];
        pair_table_kernel<T><<<dim3((unsigned)na, (unsigned)(b1 - b0)), 256, 0, s>>>(
            x, (int)n, na, b0, 1.0, pair_tab.as<T>());
        const unsigned grid = (unsigned)std::min<int64_t>(u1 - u0, (int64_t)1 << 30);
        direct_rows_kernel<T><<<grid, DirectLds<T>::TPB, 0, s>>>(
            x, (int)n, na, nb, nt, doff, u0, u1, b0, pair_tab.as<T>(), rows.as<double>());
        rows_i_kernel<IB, KR, W><<<(unsigned)na, kRT, 0, s>>>(rows.as<double>(), doff, (int)n, na,
                                                              nt, b0, b1, phi);
        rows_j_kernel<IB, kB, W><<<(unsigned)(b1 - b0), kRT, 0, s>>>(rows.as<double>(), doff,
                                                                     (int)n, b0, phi);
        rows_k_kernel<IB, kB, KT, KR, W><<<(unsigned)nt, kRT, 0, s>>>(rows.as<double>(), doff,
                                                                      (int)n, na, nt, b0, b1, phi);
        MB_HIP(hipGetLastError());
    }
    return MB_OK;
}

}  // namespace mb
