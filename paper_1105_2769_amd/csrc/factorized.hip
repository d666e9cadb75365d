// Factorized (matrix-product) form of the per-particle Axilrod-Teller sum on
// gfx950 MFMA.
//
// The law of cosines turns phi into ten products of pairwise powers
// r_ij^e1 r_ik^e2 r_jk^e3 - functions of the product form the paper's method
// is built for (Section 1) - so with M_e[u,v] = r_uv^e (zero diagonal)
//
//   Phi_i = 1/2 sum_t c_t sum_j M_e1[i,j] (M_e2 M_e3)[i,j]
//
// and, merging the pairs of monomials that differ by j <-> k, six sums
// built on five products:
//
//   T1 = rows of M-3 (.) (M-3 M-3)   c = 1/4
//   T2 = rows of M+1 (.) (M-5 M-5)   c = -3/4
//   T3 = rows of M-5 (.) (M-5 M+1)   c = -3/8
//   T4 = cols of M-1 (.) (M-5 M-3)   c = 3/4
//   T5 = rows of M-1 (.) (M-5 M-3)   c = 3/4
//   T6 = rows of M-3 (.) (M-5 M-1)   c = 3/4
//
// The products run on MFMA in FP16 or BF16.  Each M entry is split into up to
// three planes (hi, mid, lo; plane p carries 2^(B p) times its remainder, B
// the format's mantissa bits), with one power-of-two exponent per 64 x 64
// tile, so that the planes hold full-precision numbers whatever the range of
// r^e.  Products of planes are accumulated in FP32 within a 64-wide K chunk,
// grouped by level p_a + p_b < planes, then scaled and summed in FP64.  The
// elementwise weights of the epilogue are formed in FP64 from coordinates.
//
// Triples with a side shorter than r_near are excluded from the matrices
// (their entries are zero) and summed exactly in FP64 by a separate kernel:
// those are the thin triangles where the monomial expansion cancels.
// Points are first put in kd-tree order so that tiles are compact in space.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "at_device.hpp"
#include "mb_internal.hpp"
#include "tree.hpp"

namespace mb {
namespace {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kTS = 64;    // scale tile and K chunk
constexpr int kGT = 128;   // output tile of a workgroup
constexpr int kLdsRow = kTS + 8;  // padded LDS row (halves)
constexpr int kGemmWaves = 8;     // waves per GEMM workgroup (two per SIMD)

// exponents of the four pair matrices, in storage order
constexpr int kExp[4] = {-5, 1, -3, -1};

template <typename H> struct HalfFmt;
template <> struct HalfFmt<_Float16> {
    static constexpr int kBits = 11;
    __device__ static _Float16 from(double v) { return (_Float16)(float)v; }
    __device__ static double to(_Float16 h) { return (double)(float)h; }
};
template <> struct HalfFmt<__bf16> {
    static constexpr int kBits = 8;
    __device__ static __bf16 from(double v) { return (__bf16)(float)v; }
    __device__ static double to(__bf16 h) { return (double)(float)h; }
};

__device__ __forceinline__ double rpow(double r, double ir, int e) {
    const double ir2 = ir * ir;
    switch (e) {
        case -5: return ir * ir2 * ir2;
        case -3: return ir * ir2;
        case -1: return ir;
        default: return r;
    }
}

// C-1: pair matrices as planes with per-tile exponents.  One workgroup per
// 64 x 64 tile (ti, tk) of all four matrices.
template <typename H, int P>
__global__ __launch_bounds__(256) void pairmat_kernel(const double *__restrict__ xs, int n, int np,
                                                      double rn2, H *__restrict__ planes,
                                                      int *__restrict__ texp) {
    const int ti = blockIdx.y, tk = blockIdx.x, tid = threadIdx.x;
    const int nt = np / kTS;
    __shared__ double xi[3][kTS], xk[3][kTS];
    __shared__ double red[4][256];
    __shared__ int sexp[4];
    if (tid < kTS) {
        const int i = ti * kTS + tid;
        for (int c = 0; c < 3; ++c) xi[c][tid] = i < n ? xs[3 * (int64_t)i + c] : 0.0;
    } else if (tid < 2 * kTS) {
        const int k = tk * kTS + tid - kTS;
        for (int c = 0; c < 3; ++c) xk[c][tid - kTS] = k < n ? xs[3 * (int64_t)k + c] : 0.0;
    }
    __syncthreads();
    double v[16][4];
    double mx[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = tid + 256 * q;
        const int a = e / kTS, b = e % kTS;
        const int i = ti * kTS + a, k = tk * kTS + b;
        const double dx = xk[0][b] - xi[0][a], dy = xk[1][b] - xi[1][a], dz = xk[2][b] - xi[2][a];
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        const double r = sqrt(r2);
        const bool ok = i < n && k < n && i != k && r2 >= rn2;
        const double ir = 1.0 / r;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            v[q][m] = ok ? rpow(r, ir, kExp[m]) : 0.0;
            mx[m] = fmax(mx[m], v[q][m]);
        }
    }
    for (int m = 0; m < 4; ++m) red[m][tid] = mx[m];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (tid < w)
            for (int m = 0; m < 4; ++m) red[m][tid] = fmax(red[m][tid], red[m][tid + w]);
        __syncthreads();
    }
    if (tid < 4) {
        int ex = 0;
        if (red[tid][0] > 0.0) frexp(red[tid][0], &ex);  // max = f 2^ex, f in [0.5, 1)
        sexp[tid] = ex;
        texp[((int64_t)tid * nt + ti) * nt + tk] = ex;
    }
    __syncthreads();
    const int B = HalfFmt<H>::kBits;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = tid + 256 * q;
        const int a = e / kTS, b = e % kTS;
        const int64_t row = ti * kTS + a, col = tk * kTS + b;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            double rem = ldexp(v[q][m], -sexp[m]);  // in [0, 1)
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const H h = HalfFmt<H>::from(rem);
                planes[(((int64_t)m * P + p) * np + row) * np + col] = h;
                rem = (rem - HalfFmt<H>::to(h)) * (double)(1 << B);
            }
        }
    }
}

template <typename H>
__device__ __forceinline__ floatx16 mfma(const H *a, const H *b, floatx16 c);
template <>
__device__ __forceinline__ floatx16 mfma<_Float16>(const _Float16 *a, const _Float16 *b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(*(const half8_t *)a, *(const half8_t *)b, c, 0,
                                                  0, 0);
}
template <>
__device__ __forceinline__ floatx16 mfma<__bf16>(const __bf16 *a, const __bf16 *b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(*(const bf16x8_t *)a, *(const bf16x8_t *)b, c, 0,
                                                   0, 0);
}

// C-2: one product M_ma M_mb (M_mb symmetric, so B[k][j] = M_mb[j][k]) with
// the fused epilogue: rows of w (.) product into trow, and if tcol is set,
// columns into tcol, where w = r^we (masked like the matrices).
template <typename H, int P>
__global__ __launch_bounds__(64 * kGemmWaves) void gemm_kernel(const H *__restrict__ planes,
                                                   const int *__restrict__ texp,
                                                   const double *__restrict__ xs, int n, int np,
                                                   int ma, int mb, int we, double rn2,
                                                   double *__restrict__ trow,
                                                   double *__restrict__ tcol) {
    constexpr int kBufs = P <= 2 ? 2 : 1;  // LDS buffers (two with register prefetch)
    __shared__ H As[kBufs][P][kGT][kLdsRow], Bs[kBufs][P][kGT][kLdsRow];
    __shared__ double xr[3][kGT], xc[3][kGT];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // waves as a 2 x (kGemmWaves / 2) grid over the 128 x 128 tile: wave
    // (wr, wc) owns rows 64 wr.. and kWC columns from kWC wc, as 2 x kCB
    // blocks of 32 x 32
    constexpr int kThreads = 64 * kGemmWaves;
    constexpr int kWC = kGT / (kGemmWaves / 2);
    constexpr int kCB = kWC / 32;
    const int wr = wave / (kGemmWaves / 2), wc = wave % (kGemmWaves / 2);
    // Launch order.  Workgroups are dealt to the 8 XCDs in turn (workgroup w
    // to XCD w mod 8), and each XCD has its own L2.  When the tile count is
    // a multiple of 8, XCD x takes the x-th eighth of a grouped order (4 tile
    // rows per column sweep): the 32 workgroups an XCD runs at once cover 4
    // rows x 8 columns, so per K chunk its L2 fetches 12 tiles instead of
    // one per workgroup.  Otherwise the grouped order is used directly.
    constexpr int kGroup = 4;
    const int n_i = gridDim.y, n_j = gridDim.x;
    const int n_wg = n_i * n_j;
    int wg = blockIdx.y * n_j + blockIdx.x;
    if (n_wg % 8 == 0) wg = (wg % 8) * (n_wg / 8) + wg / 8;
    const int g_first = (wg / (kGroup * n_j)) * kGroup;
    const int g_rows = min(n_i - g_first, kGroup);
    const int g_local = wg - g_first * n_j;
    const int I0 = (g_first + g_local % g_rows) * kGT, J0 = (g_local / g_rows) * kGT;
    const int nt = np / kTS;
    const int B = HalfFmt<H>::kBits;

    double acc64[2][kCB][16];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < kCB; ++cb)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc64[rb][cb][r] = 0.0;

    // binary32 partial sums over groups of chunks (see the fold below)
    constexpr int kFoldChunks = 8;
    float acc32[2][kCB][16];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < kCB; ++cb)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc32[rb][cb][r] = 0.0f;
    int group = 0, ex_ref = 0;

    const H *pa = planes + (int64_t)ma * P * np * np;
    const H *pb = planes + (int64_t)mb * P * np * np;
    // The A rows I0.. and B rows J0.. of a K chunk, all planes: kPieces
    // 16-byte pieces per thread and operand.  With one or two planes the
    // next chunk's pieces are loaded into registers while this chunk's
    // products run and stored to the other LDS buffer after them; three
    // planes have no registers or LDS to spare and load each chunk into the
    // one buffer before its products.
    constexpr int kPieces = kGT * (kTS / 8) / kThreads;
    static_assert(kPieces * kThreads == kGT * (kTS / 8), "whole pieces per thread");
    constexpr bool kPrefetch = P <= 2;
    constexpr int PR = kPrefetch ? P : 1;
    u32x4 nextA[PR][kPieces], nextB[PR][kPieces];
    // (written out rather than as a lambda: a captured array would be kept in
    // scratch memory instead of registers)
    if constexpr (kPrefetch) {
        // two LDS buffers: chunk kc is read from buffer kc & 1 while chunk
        // kc + 1 is stored into the other one, one barrier per chunk
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int q = 0; q < kPieces; ++q) {
                const int e = tid + kThreads * q;
                const int row = e / (kTS / 8), c8 = (e % (kTS / 8)) * 8;
                *(u32x4 *)&As[0][p][row][c8] =
                    *(const u32x4 *)&pa[((int64_t)p * np + I0 + row) * np + c8];
                *(u32x4 *)&Bs[0][p][row][c8] =
                    *(const u32x4 *)&pb[((int64_t)p * np + J0 + row) * np + c8];
            }
        if (nt > 1) {
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int q = 0; q < kPieces; ++q) {
                    const int e = tid + kThreads * q;
                    const int row = e / (kTS / 8), c8 = (e % (kTS / 8)) * 8;
                    nextA[p][q] = *(const u32x4 *)&pa[((int64_t)p * np + I0 + row) * np + kTS + c8];
                    nextB[p][q] = *(const u32x4 *)&pb[((int64_t)p * np + J0 + row) * np + kTS + c8];
                }
        }
        __syncthreads();
    }
    for (int kc = 0; kc < nt; ++kc) {
        const int cur = kPrefetch ? (kc & 1) : 0;
        if constexpr (!kPrefetch) {
            __syncthreads();  // the previous chunk's products are done with the LDS
            const int K0 = kc * kTS;
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int q = 0; q < kPieces; ++q) {
                    const int e = tid + kThreads * q;
                    const int row = e / (kTS / 8), c8 = (e % (kTS / 8)) * 8;
                    *(u32x4 *)&As[0][p][row][c8] =
                        *(const u32x4 *)&pa[((int64_t)p * np + I0 + row) * np + K0 + c8];
                    *(u32x4 *)&Bs[0][p][row][c8] =
                        *(const u32x4 *)&pb[((int64_t)p * np + J0 + row) * np + K0 + c8];
                }
            __syncthreads();
        }
        floatx16 acc[P][2][kCB];
#pragma unroll
        for (int L = 0; L < P; ++L)
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < kCB; ++cb)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[L][rb][cb][r] = 0.0f;
#pragma unroll
        for (int kk = 0; kk < kTS / 16; ++kk) {
            const int kcol = kk * 16 + 8 * (lane >> 5);
#pragma unroll
            for (int qa = 0; qa < P; ++qa)
#pragma unroll
                for (int qb = 0; qa + qb < P; ++qb)
#pragma unroll
                    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                        for (int cb = 0; cb < kCB; ++cb)
                            acc[qa + qb][rb][cb] =
                                mfma<H>(&As[cur][qa][64 * wr + 32 * rb + (lane & 31)][kcol],
                                        &Bs[cur][qb][kWC * wc + 32 * cb + (lane & 31)][kcol],
                                        acc[qa + qb][rb][cb]);
        }
        // Scale of this wave's block (inside one 64 x 64 scale tile) for this
        // chunk (wave-uniform).  Chunk sums are added in binary32 relative to
        // the scale 2^ex_ref of the first chunk of a group; a group ends after
        // kFoldChunks chunks or when a scale leaves [ex_ref - 24, ex_ref + 24],
        // and its sum is then added to the binary64 accumulator.  Chunk sums
        // are non-negative up to the small lower-plane corrections, so a
        // group adds at most kFoldChunks roundings of 2^-24 relative.
        const int ex = texp[((int64_t)ma * nt + (I0 / kTS + wr)) * nt + kc] +
                       texp[((int64_t)mb * nt + (J0 + kWC * wc) / kTS) * nt + kc];
        if (group == kFoldChunks || ex > ex_ref + 24 || ex < ex_ref - 24) {
            const double sc = ldexp(1.0, ex_ref);
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < kCB; ++cb)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        acc64[rb][cb][r] = fma((double)acc32[rb][cb][r], sc, acc64[rb][cb][r]);
                        acc32[rb][cb][r] = 0.0f;
                    }
            group = 0;
        }
        if (group == 0) ex_ref = ex;
        ++group;
        const float rs = ldexpf(1.0f, ex - ex_ref);  // a power of two in [2^-24, 2^24]
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < kCB; ++cb)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    float v = acc[P - 1][rb][cb][r];
#pragma unroll
                    for (int L = P - 2; L >= 0; --L) v = fmaf(v, 1.0f / (float)(1 << B), acc[L][rb][cb][r]);
                    acc32[rb][cb][r] = fmaf(v, rs, acc32[rb][cb][r]);
                }
        if constexpr (kPrefetch) {
            if (kc + 1 < nt) {
                // chunk kc + 1 into the other buffer (last read in chunk kc - 1,
                // before the previous barrier), then fetch chunk kc + 2
#pragma unroll
                for (int p = 0; p < P; ++p)
#pragma unroll
                    for (int q = 0; q < kPieces; ++q) {
                        const int e = tid + kThreads * q;
                        const int row = e / (kTS / 8), c8 = (e % (kTS / 8)) * 8;
                        *(u32x4 *)&As[cur ^ 1][p][row][c8] = nextA[p][q];
                        *(u32x4 *)&Bs[cur ^ 1][p][row][c8] = nextB[p][q];
                    }
                if (kc + 2 < nt) {
                    const int K2 = (kc + 2) * kTS;
#pragma unroll
                    for (int p = 0; p < P; ++p)
#pragma unroll
                        for (int q = 0; q < kPieces; ++q) {
                            const int e = tid + kThreads * q;
                            const int row = e / (kTS / 8), c8 = (e % (kTS / 8)) * 8;
                            nextA[p][q] = *(const u32x4 *)&pa[((int64_t)p * np + I0 + row) * np +
                                                              K2 + c8];
                            nextB[p][q] = *(const u32x4 *)&pb[((int64_t)p * np + J0 + row) * np +
                                                              K2 + c8];
                        }
                }
            }
            __syncthreads();
        }
    }
    {
        const double sc = ldexp(1.0, ex_ref);
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < kCB; ++cb)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    acc64[rb][cb][r] = fma((double)acc32[rb][cb][r], sc, acc64[rb][cb][r]);
    }
    // epilogue: weights from coordinates
    __syncthreads();
    if (tid < kGT) {
        const int i = I0 + tid;
        for (int c = 0; c < 3; ++c) xr[c][tid] = i < n ? xs[3 * (int64_t)i + c] : 0.0;
    } else if (tid < 2 * kGT) {
        const int j = J0 + tid - kGT;
        for (int c = 0; c < 3; ++c) xc[c][tid - kGT] = j < n ? xs[3 * (int64_t)j + c] : 0.0;
    }
    __syncthreads();
    double colsum[kCB];
#pragma unroll
    for (int cb = 0; cb < kCB; ++cb) colsum[cb] = 0.0;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < kCB; ++cb) {
            const int jl = kWC * wc + 32 * cb + (lane & 31);
            const int j = J0 + jl;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int il = 64 * wr + 32 * rb + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int i = I0 + il;
                const double dx = xc[0][jl] - xr[0][il], dy = xc[1][jl] - xr[1][il],
                             dz = xc[2][jl] - xr[2][il];
                const double rr2 = fma(dx, dx, fma(dy, dy, dz * dz));
                const double rr = sqrt(rr2);
                const bool ok = i < n && j < n && i != j && rr2 >= rn2;
                const double w = ok ? rpow(rr, 1.0 / rr, we) * acc64[rb][cb][r] : 0.0;
                colsum[cb] += w;
                // row sum over the 32 lanes that hold this row
                double v = w;
#pragma unroll
                for (int m = 16; m >= 1; m >>= 1) v += __shfl_xor(v, m);
                if ((lane & 31) == 0 && i < n) atomicAdd(&trow[i], v);
            }
        }
    if (tcol) {
#pragma unroll
        for (int cb = 0; cb < kCB; ++cb) {
            const double v = colsum[cb] + __shfl_xor(colsum[cb], 32);
            const int j = J0 + kWC * wc + 32 * cb + (lane & 31);
            if (lane < 32 && j < n) atomicAdd(&tcol[j], v);
        }
    }
}

// C-3a: pairs closer than r_near (u < v), appended to a list.
__global__ void near_pairs_kernel(const double *__restrict__ xs, int n, double rn2,
                                  int2 *__restrict__ out, unsigned long long *__restrict__ count,
                                  unsigned long long cap) {
    const int u = blockIdx.y * blockDim.x + threadIdx.x;
    const int v0 = blockIdx.x * 256;
    __shared__ double xv[3][256];
    const int v = v0 + threadIdx.x;
    for (int c = 0; c < 3; ++c) xv[c][threadIdx.x] = v < n ? xs[3 * (int64_t)v + c] : 0.0;
    __syncthreads();
    if (u >= n || v0 + 255 <= u) return;
    const double x0 = xs[3 * (int64_t)u], x1 = xs[3 * (int64_t)u + 1], x2 = xs[3 * (int64_t)u + 2];
    for (int q = 0; q < 256; ++q) {
        const int vv = v0 + q;
        if (vv <= u || vv >= n) continue;
        const double dx = xv[0][q] - x0, dy = xv[1][q] - x1, dz = xv[2][q] - x2;
        if (fma(dx, dx, fma(dy, dy, dz * dz)) < rn2) {
            const unsigned long long s = atomicAdd(count, 1ull);
            if (s < cap) out[s] = make_int2(u, vv);
        }
    }
}

__device__ __forceinline__ bool pair_less(int a0, int a1, int b0, int b1) {
    return a0 < b0 || (a0 == b0 && a1 < b1);
}

// C-3b: every triple with at least one side shorter than r_near, exactly in
// FP64, counted once: by the smallest (lexicographic) of its short pairs.
// A workgroup takes 256 third points w and a range of short pairs.
__global__ __launch_bounds__(256) void near_triples_kernel(
    const double *__restrict__ xs, int n, double rn2, const int2 *__restrict__ pairs,
    long long n_pairs, long long pairs_per_block, double *__restrict__ phi) {
    const int w = blockIdx.x * 256 + threadIdx.x;
    const long long p0 = (long long)blockIdx.y * pairs_per_block;
    const long long p1 = min(n_pairs, p0 + pairs_per_block);
    __shared__ double pair_sum[256];
    const int lane = threadIdx.x & 63;
    const bool wok = w < n;
    double xw[3] = {0.0, 0.0, 0.0};
    if (wok)
        for (int c = 0; c < 3; ++c) xw[c] = xs[3 * (int64_t)w + c];
    double accw = 0.0;
    for (long long pbase = p0; pbase < p1; pbase += 256) {
        __syncthreads();
        pair_sum[threadIdx.x] = 0.0;
        __syncthreads();
        const int cnt = (int)min(256ll, p1 - pbase);
        for (int q = 0; q < cnt; ++q) {
            const int2 pr = pairs[pbase + q];
            const int u = pr.x, v = pr.y;
            double f = 0.0;
            if (wok && w != u && w != v) {
                const double *xu = xs + 3 * (int64_t)u, *xv = xs + 3 * (int64_t)v;
                const double duw[3] = {xw[0] - xu[0], xw[1] - xu[1], xw[2] - xu[2]};
                const double dvw[3] = {xw[0] - xv[0], xw[1] - xv[1], xw[2] - xv[2]};
                const double ruw2 = fma(duw[0], duw[0], fma(duw[1], duw[1], duw[2] * duw[2]));
                const double rvw2 = fma(dvw[0], dvw[0], fma(dvw[1], dvw[1], dvw[2] * dvw[2]));
                // is (u, v) the smallest short pair of the triple?
                bool canon = true;
                if (ruw2 < rn2 && pair_less(min(u, w), max(u, w), u, v)) canon = false;
                if (rvw2 < rn2 && pair_less(min(v, w), max(v, w), u, v)) canon = false;
                if (canon) {
                    double a, qa, wa, ia, b, qb, wb, ib, c, qc, wc_, ic;
                    pair_terms(xv[0] - xu[0], xv[1] - xu[1], xv[2] - xu[2], true, a, qa, wa, ia);
                    pair_terms(duw[0], duw[1], duw[2], true, b, qb, wb, ib);
                    pair_terms(dvw[0], dvw[1], dvw[2], true, c, qc, wc_, ic);
                    f = phi_from_pairs<double>(a, qa, wa, b, qb, wb, c, qc, wc_);
                }
            }
            accw += f;
            double s = f;
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
            if (lane == 0) atomicAdd(&pair_sum[q], s);
        }
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            const int2 pr = pairs[pbase + threadIdx.x];
            const double s = pair_sum[threadIdx.x];
            if (s != 0.0) {
                atomicAdd(&phi[pr.x], s);
                atomicAdd(&phi[pr.y], s);
            }
        }
    }
    if (wok && accw != 0.0) atomicAdd(&phi[w], accw);
}

// Combine: Phi = 1/2 sum_t c_t T_t + near, back to input order.
__global__ void factor_combine_kernel(int n, const int32_t *__restrict__ perm,
                                      const double *__restrict__ t, const double *__restrict__ near,
                                      double *__restrict__ phi) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const double s = 0.25 * t[0 * (int64_t)n + r] - 0.75 * t[1 * (int64_t)n + r] -
                     0.375 * t[2 * (int64_t)n + r] +
                     0.75 * (t[3 * (int64_t)n + r] + t[4 * (int64_t)n + r] + t[5 * (int64_t)n + r]);
    phi[perm[r]] = 0.5 * s + near[r];
}

template <typename H, int P>
mb_status factorized_run(const DeviceTree *tr, int n, double r_near, double *phi, hipStream_t s,
                         FactorStats *stats) {
    const int np = (n + kGT - 1) / kGT * kGT;
    const int nt = np / kTS;
    mb_status st;
    Scratch s_planes, s_exp, s_t, s_near, s_pairs, s_cnt;
    const size_t plane_elems = (size_t)4 * P * np * np;
    if ((st = s_planes.alloc(sizeof(H) * plane_elems, s)) != MB_OK) return st;
    if ((st = s_exp.alloc(sizeof(int) * 4 * (size_t)nt * nt, s)) != MB_OK) return st;
    if ((st = s_t.alloc(sizeof(double) * 6 * (size_t)n, s)) != MB_OK) return st;
    if ((st = s_near.alloc(sizeof(double) * n, s)) != MB_OK) return st;
    if ((st = s_cnt.alloc(sizeof(unsigned long long), s)) != MB_OK) return st;
    double *t = s_t.as<double>();
    zero_doubles(t, 6 * (int64_t)n, s);
    zero_doubles(s_near.as<double>(), n, s);

    // one squared threshold for every near / far decision: a pair is near
    // iff its squared distance (formed the same way in every kernel) is < rn2
    const double rn2 = r_near * r_near;
    hipEvent_t e0, e1, e2, e3;
    MB_HIP(hipEventCreate(&e0));
    MB_HIP(hipEventCreate(&e1));
    MB_HIP(hipEventCreate(&e2));
    MB_HIP(hipEventCreate(&e3));
    MB_HIP(hipEventRecord(e0, s));
    pairmat_kernel<H, P><<<dim3(nt, nt), 256, 0, s>>>(tr->xs, n, np, rn2, s_planes.as<H>(),
                                                      s_exp.as<int>());
    MB_HIP(hipEventRecord(e1, s));
    const dim3 g(np / kGT, np / kGT);
    // (A matrix, B matrix, weight exponent, row target, column target); storage order -5, +1, -3, -1
    gemm_kernel<H, P><<<g, 64 * kGemmWaves, 0, s>>>(s_planes.as<H>(), s_exp.as<int>(), tr->xs, n, np, 2, 2, -3,
                                        rn2, t + 0 * (int64_t)n, nullptr);
    gemm_kernel<H, P><<<g, 64 * kGemmWaves, 0, s>>>(s_planes.as<H>(), s_exp.as<int>(), tr->xs, n, np, 0, 0, 1,
                                        rn2, t + 1 * (int64_t)n, nullptr);
    gemm_kernel<H, P><<<g, 64 * kGemmWaves, 0, s>>>(s_planes.as<H>(), s_exp.as<int>(), tr->xs, n, np, 0, 1, -5,
                                        rn2, t + 2 * (int64_t)n, nullptr);
    gemm_kernel<H, P><<<g, 64 * kGemmWaves, 0, s>>>(s_planes.as<H>(), s_exp.as<int>(), tr->xs, n, np, 0, 2, -1,
                                        rn2, t + 4 * (int64_t)n, t + 3 * (int64_t)n);
    gemm_kernel<H, P><<<g, 64 * kGemmWaves, 0, s>>>(s_planes.as<H>(), s_exp.as<int>(), tr->xs, n, np, 0, 3, -3,
                                        rn2, t + 5 * (int64_t)n, nullptr);
    MB_HIP(hipGetLastError());
    MB_HIP(hipEventRecord(e2, s));
    // near field: count, then list, then triples
    unsigned long long cnt = 0;
    MB_HIP(hipMemsetAsync(s_cnt.ptr, 0, sizeof cnt, s));
    const dim3 pg((n + 255) / 256, (n + 255) / 256);
    near_pairs_kernel<<<pg, 256, 0, s>>>(tr->xs, n, rn2, nullptr, s_cnt.as<unsigned long long>(), 0);
    MB_HIP(hipMemcpyAsync(&cnt, s_cnt.ptr, sizeof cnt, hipMemcpyDeviceToHost, s));
    MB_HIP(hipStreamSynchronize(s));
    if (cnt > 0) {
        if ((st = s_pairs.alloc(sizeof(int2) * cnt, s)) != MB_OK) return st;
        MB_HIP(hipMemsetAsync(s_cnt.ptr, 0, sizeof cnt, s));
        near_pairs_kernel<<<pg, 256, 0, s>>>(tr->xs, n, rn2, s_pairs.as<int2>(),
                                             s_cnt.as<unsigned long long>(), cnt);
        const long long per = 4096;
        const dim3 tg((n + 255) / 256, (unsigned)((cnt + per - 1) / per));
        near_triples_kernel<<<tg, 256, 0, s>>>(tr->xs, n, rn2, s_pairs.as<int2>(), (long long)cnt,
                                               per, s_near.as<double>());
    }
    MB_HIP(hipGetLastError());
    factor_combine_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, tr->perm, t, s_near.as<double>(), phi);
    MB_HIP(hipEventRecord(e3, s));
    MB_HIP(hipEventSynchronize(e3));
    float m01 = 0, m12 = 0, m23 = 0;
    MB_HIP(hipEventElapsedTime(&m01, e0, e1));
    MB_HIP(hipEventElapsedTime(&m12, e1, e2));
    MB_HIP(hipEventElapsedTime(&m23, e2, e3));
    for (hipEvent_t e : {e0, e1, e2, e3}) (void)hipEventDestroy(e);
    if (stats) {
        stats->pairmat_ms = m01;
        stats->gemm_ms = m12;
        stats->near_ms = m23;
        stats->near_pairs = (int64_t)cnt;
        stats->gemm_flops = 10.0 * (double)np * np * np * (P * (P + 1) / 2);
    }
    return MB_OK;
}

}  // namespace

mb_status factorized_eval(const DeviceTree *tr, int n, int fmt, int planes, double r_near,
                          double *phi, hipStream_t s, FactorStats *stats) {
    if (fmt == 0) {
        if (planes == 1) return factorized_run<_Float16, 1>(tr, n, r_near, phi, s, stats);
        if (planes == 2) return factorized_run<_Float16, 2>(tr, n, r_near, phi, s, stats);
        return factorized_run<_Float16, 3>(tr, n, r_near, phi, s, stats);
    }
    if (planes == 1) return factorized_run<__bf16, 1>(tr, n, r_near, phi, s, stats);
    if (planes == 2) return factorized_run<__bf16, 2>(tr, n, r_near, phi, s, stats);
    return factorized_run<__bf16, 3>(tr, n, r_near, phi, s, stats);
}

}  // namespace mb
