// Tile code of the exhaustive per-particle Axilrod-Teller sum (the naive
// algorithm of Section 6, definition in Section 1), shared by the one-shot
// kernel and the serving kernel.
//
// Work decomposition.  A work unit is a block triple (I, J, K): an I block of
// NW * IPW points, a J block of 64 and a K tile of 64 * KR.  Units are
// enumerated so that together they hold every unordered triple i < j < k
// exactly once; inside a unit the global-index masks i < j < k < n drop the
// rest.  One workgroup of NW wave64s runs one unit:
//
//   * lane l owns the KR points k = K0 + l + 64 m, m = 0..KR-1;
//   * wave w owns IPW points i and keeps the (i, k) pair terms of its
//     KR * IPW combinations in registers for the whole unit;
//   * the (i, j) pair terms do not depend on the lane.  A table kernel writes
//     them to HBM per (I, J) block pair, and the triple kernel reads them
//     with scalar loads into SGPRs, issued one j ahead of their use;
//   * the (j, k) terms (one per lane) are staged in LDS per chunk of 16 j
//     and also read one j ahead into registers.
//
// Inner step for one triple, with (a, wa) the (i, j) terms, (g, wg) the
// (i, k) terms and (b, qb, ob = 3/8 / b) the (j, k) terms.  Since
// q_x = x w_x, phi = qa qb qg + 3/8 wa wb wg P factors as
//
//   phi = qb wa psi,   psi = wg (a g + ob (a + g - b)(b^2 - (a - g)^2))
//
// (8 VALU operations), and the sums take the two remaining factors at once:
// Phi_k += qb * sum_i wa psi (register), Phi_i += wa * sum_k qb psi
// (register array, the wa product once per (i, j)) and Phi_j += sum over
// lanes, waves of sum_k qb * sum_i wa psi (one LDS atomic per lane and j
// into a per-(j, lane) slot, reduced once per chunk): about 10.3 operations
// per triple.  The register partials of Phi_i and Phi_k live in the tile
// type for one chunk of 16 j and are folded into binary64 after it; unit
// sums go to Phi with FP64 atomics.
#pragma once

#include "at_device.hpp"

namespace mb {
namespace {

constexpr int kB = 64;              // points per J block
constexpr int kPairVals = 2;        // numbers per pair of the (i, j) table: a, w
#ifndef MB_FOLD_J
#define MB_FOLD_J 16                // j steps per binary32 partial of Phi_i
#endif

// Tile shape per arithmetic type: i points per wave, waves per workgroup,
// k points per lane, j points per LDS chunk; kLdsBB: b^2 of the (j, k)
// terms is staged in LDS with them (else squared at every j step).
template <typename T> struct DirectShape;
#ifndef MB_IPW64
#define MB_IPW64 8
#endif
#ifndef MB_NW64
#define MB_NW64 8
#endif
#ifndef MB_KR64
#define MB_KR64 2
#endif
#ifndef MB_IPW32
#define MB_IPW32 8
#endif
#ifndef MB_NW32
#define MB_NW32 8
#endif
#ifndef MB_KR32
#define MB_KR32 4
#endif
#ifndef MB_JC64
#define MB_JC64 16
#endif
#ifndef MB_JC32
#define MB_JC32 16
#endif
#ifndef MB_BB64
#define MB_BB64 1
#endif
#ifndef MB_BB32
#define MB_BB32 1
#endif
#ifndef MB_MINB64
#define MB_MINB64 1
#endif
#ifndef MB_MINB32
#define MB_MINB32 1
#endif
template <> struct DirectShape<double> {
    static constexpr int IPW = MB_IPW64;
    static constexpr int NW = MB_NW64;
    static constexpr int KR = MB_KR64;
    static constexpr int JC = MB_JC64;
    static constexpr bool kPair32 = false;  // (i, k) and (j, k) terms from pair_terms (binary64)
    static constexpr bool kLdsBB = MB_BB64;
    static constexpr int MINB = MB_MINB64;  // workgroups per CU the registers must allow
};
template <> struct DirectShape<float> {
    static constexpr int IPW = MB_IPW32;
    static constexpr int NW = MB_NW32;
    static constexpr int KR = MB_KR32;
    static constexpr int JC = MB_JC32;
    static constexpr bool kPair32 = false;
    static constexpr bool kLdsBB = MB_BB32;
    static constexpr int MINB = MB_MINB32;
};

// LDS of one work unit.  Shape gives i points per wave, waves and k points
// per lane (DirectShape<T> for the exhaustive sum); JB is the J block.
template <typename T, int JB = kB, typename Shape = DirectShape<T>>
struct DirectLds {
    static constexpr int kJC = Shape::JC;
    static_assert(JB % kJC == 0 && kJC % 2 == 0, "the J block is a whole number of chunks");
    static constexpr int TPB = Shape::NW * 64;  // threads per workgroup
    static constexpr int IB = Shape::NW * Shape::IPW;
    static constexpr int KR = Shape::KR;
    static constexpr int KT = 64 * KR;                   // points per K tile
    static constexpr int XS = IB + JB + KT;
    // the fixed-order mode's per-wave Phi_k sums fit in the space they share
    static constexpr bool kOrderedFits = Shape::NW * 8 <= kJC * (int)sizeof(T);
    static constexpr int kOW = kOrderedFits ? Shape::NW : 1;
    double xs[3][XS];                              // coordinates of the I, J blocks and K tile
    union {
        T cb[kJC][KT];                             // (j, k) terms of the chunk
        double kw[kOW][KT];                        // fixed order: Phi_k per wave, after the chunks
    };
    T cq[kJC][KT], co[kJC][KT];
    T cbb[Shape::kLdsBB ? kJC : 1][KT];            // their b^2 (kLdsBB)
    double pj[kJC][64];                            // Phi_j partials per (j, lane), all waves
    double pjacc[JB];                              // Phi_j of the unit
    double kacc[KT];                               // Phi_k of the unit
};

// Where the points of a unit's slots come from: slot p of the unit (I block
// [0, IB), J block [IB, IB + JB), K tile [IB + JB, XS)) holds the point of
// index rank(p) in the coordinate array, or none if rank(p) < 0; ri, rj, rk
// give the same by offset inside the I block, J block and K tile.  A pair
// (u, v) of slots counts iff both hold points and rank(u) < rank(v): every
// triple of a unit is then taken once, in the order i < j < k.
//
// BlockIndex: the exhaustive sum's blocks of consecutive input indices
// (I block a, J block b, K tile t).
template <int IB, int JB, int KT>
struct BlockIndex {
    int n, I0, J0, K0;
    __device__ __forceinline__ BlockIndex(int n_, int a, int b, int t)
        : n(n_), I0(a * IB), J0(b * JB), K0(t * KT) {}
    __device__ __forceinline__ int rank(int p) const {
        const int g = p < IB ? I0 + p : (p < IB + JB ? J0 + p - IB : K0 + p - IB - JB);
        return g < n ? g : -1;
    }
    __device__ __forceinline__ int ri(int il) const { return I0 + il < n ? I0 + il : -1; }
    __device__ __forceinline__ int rj(int jl) const { return J0 + jl < n ? J0 + jl : -1; }
    __device__ __forceinline__ int rk(int kl) const { return K0 + kl < n ? K0 + kl : -1; }
};

// Units of J block b: a in [0, na_b) times t in [b / kr, nt), where a K tile
// holds kr J blocks (k > j >= 64 b puts k in tile b / kr or later).
__host__ __device__ __forceinline__ int units_a(int b, int ib, int na) {
    return min(na, (64 * b + 62) / ib + 1);
}

__device__ __forceinline__ void decode_unit(int64_t u, const int64_t *__restrict__ off, int nb,
                                            int nt, int kr, int &a, int &b, int &t) {
    int lo = 0, hi = nb;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= u) lo = mid; else hi = mid;
    }
    b = lo;
    const int64_t rem = u - off[b];
    const int tc = nt - b / kr;
    a = (int)(rem / tc);
    t = b / kr + (int)(rem % tc);
}

// s_waitcnt lgkmcnt(0) (vmcnt and expcnt left at their maxima), with
// scheduling barriers so no memory operation moves across it.
__device__ __forceinline__ void lgkm_wait_all() {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_sched_barrier(0);
}

__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// One entry of an (i, j) table: a = |d|^2 and w = a^(-5/2) in binary64,
// rounded to T; a masked pair gets a = 1, w = 0, so the triples through it
// vanish.
template <typename T>
__device__ __forceinline__ void table_entry(double dx, double dy, double dz, bool valid, T *out) {
    double pa, pq, pw, pia;
    pair_terms(dx, dy, dz, valid, pa, pq, pw, pia);
    out[0] = (T)pa;
    out[1] = (T)pw;
}

// (i, j) pair-term table for J blocks b0 <= b < b0 + gridDim.y: block (a, b)
// holds (a_ij, w_ij) at [jl][il][kPairVals] for i = IB a + il, j = 64 b + jl,
// masked unless i < j < n.
template <typename T>
__global__ __launch_bounds__(256) void pair_table_kernel(const double *__restrict__ x, int n,
                                                         int na, int b0, double scale,
                                                         T *__restrict__ tab) {
    constexpr int IB = DirectLds<T>::IB;
    const int a = blockIdx.x, b = b0 + blockIdx.y;
    if (a >= units_a(b, IB, na)) return;
    __shared__ double xa[3][IB], xb[3][kB];
    const int tid = threadIdx.x;
    if (tid < IB) {
        const int i = a * IB + tid;
        for (int c = 0; c < 3; ++c) xa[c][tid] = i < n ? x[3 * (int64_t)i + c] * scale : 0.0;
    } else if (tid < IB + kB) {
        const int j = b * kB + tid - IB;
        for (int c = 0; c < 3; ++c) xb[c][tid - IB] = j < n ? x[3 * (int64_t)j + c] * scale : 0.0;
    }
    __syncthreads();
    T *out = tab + ((int64_t)blockIdx.y * na + a) * (IB * kB * kPairVals);
    for (int e = tid; e < IB * kB; e += 256) {
        const int jl = e / IB, il = e % IB;
        const int i = a * IB + il, j = b * kB + jl;
        table_entry(xb[0][jl] - xa[0][il], xb[1][jl] - xa[1][il], xb[2][jl] - xa[2][il],
                    (i < j) && (j < n), out + kPairVals * e);
    }
}

// psi of one triple as the tiles evaluate it (phi = q_jk w_ij psi), from
// a = |x_j - x_i|^2, the (i, k) terms (g, wg) and the (j, k) terms
// (b, bb = b * b, ob = 3/8 / b).  Written once so that the binary32
// near-field refinement reproduces the tile's psi bit for bit.
template <typename T>
__device__ __forceinline__ T tile_psi(T a, T g, T wg, T b, T bb, T ob) {
    const T d = a - g;
    const T tt = (a + g) - b;
    const T m = fma(-d, d, bb);
    const T P = tt * m;
    return wg * fma(ob, P, a * g);
}

// One work unit of the triple sum: the I block, J block and K tile named by
// the index policy `ix` (see BlockIndex); ublk is the unit's (i, j) table,
// [jl][il][a, w] for the IB x JB pairs, read with scalar loads (a pointer
// into the constant address space where the caller cannot otherwise show
// the table is unchanged during the kernel).  x holds the coordinates the
// ranks index; sums go to phi[rank] (times out_scale).  Every thread of the
// workgroup calls it.
//
// kOrdered: every sum of the unit is formed in an order fixed by the code
// alone (per-wave partials, lane reductions by a fixed butterfly, waves
// combined in wave order), and phi is instead the unit's own row of
// IB + JB + KT values: the I block's sums, then the J block's, then the K
// tile's, times out_scale (empty slots get 0).  Adding the rows of all
// units in a fixed order then gives a result independent of scheduling.
// pjl (kOrdered only) is LDS for NW * JC * 64 Phi_j partials, one slot per
// (wave, j, lane), in place of the atomic mode's shared adds.
template <typename T, int JB, typename Shape, typename Ix, typename TabPtr, bool kOrdered = false>
__device__ __forceinline__ void tile_unit(DirectLds<T, JB, Shape> &s, const double *__restrict__ x,
                                          const Ix &ix, TabPtr ublk, double scale,
                                          double out_scale, double *__restrict__ phi,
                                          double *__restrict__ pjl = nullptr) {
    static_assert(!kOrdered || DirectLds<T, JB, Shape>::kOrderedFits,
                  "per-wave sums of the fixed-order mode fit in the LDS they reuse");
    constexpr int IPW = Shape::IPW;
    constexpr int IB = DirectLds<T, JB, Shape>::IB;
    constexpr int TPB = DirectLds<T, JB, Shape>::TPB;
    constexpr int kKR = DirectLds<T, JB, Shape>::KR;
    constexpr int kKT = DirectLds<T, JB, Shape>::KT;
    constexpr int XS = DirectLds<T, JB, Shape>::XS;
    constexpr int kJC = Shape::JC;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    constexpr int XI = 0, XJ = IB, XK = IB + JB;
    const TabPtr up = ublk + wave * (IPW * kPairVals);

    __syncthreads();  // the previous unit is done with the LDS
    for (int p = tid; p < XS; p += TPB) {
        const int g = ix.rank(p);
        const bool ok = g >= 0;
        s.xs[0][p] = ok ? x[3 * (int64_t)g + 0] * scale : 0.0;
        s.xs[1][p] = ok ? x[3 * (int64_t)g + 1] * scale : 0.0;
        s.xs[2][p] = ok ? x[3 * (int64_t)g + 2] * scale : 0.0;
    }
    if constexpr (!kOrdered)
        for (int e = tid; e < kKT; e += TPB) s.kacc[e] = 0.0;
    __syncthreads();

    // (i, k) pair terms of this wave, in registers for the whole unit
    T ag[IPW][kKR], aw[IPW][kKR];
    T acc_i[IPW];
    double acc_i64[IPW];
#pragma unroll
    for (int ii = 0; ii < IPW; ++ii) {
        const int il = wave * IPW + ii;
        const int i = ix.ri(il);
#pragma unroll
        for (int kk = 0; kk < kKR; ++kk) {
            const int kl = lane + 64 * kk;
            const int k = ix.rk(kl);
            const double dx = s.xs[0][XK + kl] - s.xs[0][XI + il];
            const double dy = s.xs[1][XK + kl] - s.xs[1][XI + il];
            const double dz = s.xs[2][XK + kl] - s.xs[2][XI + il];
            if constexpr (Shape::kPair32) {
                float pq, pia;
                pair_terms32(dx, dy, dz, (i >= 0) && (k > i), ag[ii][kk], pq, aw[ii][kk], pia);
            } else {
                double pa, pq, pw, pia;
                pair_terms(dx, dy, dz, (i >= 0) && (k > i), pa, pq, pw, pia);
                ag[ii][kk] = (T)pa;
                aw[ii][kk] = (T)pw;
            }
        }
        acc_i[ii] = T(0);
        acc_i64[ii] = 0.0;
    }
    double acck[kKR];
#pragma unroll
    for (int kk = 0; kk < kKR; ++kk) acck[kk] = 0.0;
    // binary32 tiles: Phi_k partials of the current chunk, folded into acck
    // once per chunk (binary64 tiles add into acck directly)
    constexpr int KR32 = sizeof(T) == 4 ? kKR : 1;
    T acck32[KR32];
#pragma unroll
    for (int kk = 0; kk < KR32; ++kk) acck32[kk] = T(0);

    for (int jc = 0; jc < JB / kJC; ++jc) {
        __syncthreads();  // previous chunk's readers are done
        for (int e = tid; e < kJC * kKT; e += TPB) {
            const int jj = e / kKT, kl = e % kKT;
            const int jl = jc * kJC + jj;
            const int j = ix.rj(jl), k = ix.rk(kl);
            const double dx = s.xs[0][XK + kl] - s.xs[0][XJ + jl];
            const double dy = s.xs[1][XK + kl] - s.xs[1][XJ + jl];
            const double dz = s.xs[2][XK + kl] - s.xs[2][XJ + jl];
            if constexpr (Shape::kPair32) {
                float pa, pq, pw, pia;
                pair_terms32(dx, dy, dz, (j >= 0) && (k > j), pa, pq, pw, pia);
                s.cb[jj][kl] = pa;
                s.cq[jj][kl] = pq;
                s.co[jj][kl] = 0.375f * pia;
                if constexpr (Shape::kLdsBB) s.cbb[jj][kl] = pa * pa;
            } else {
                double pa, pq, pw, pia;
                pair_terms(dx, dy, dz, (j >= 0) && (k > j), pa, pq, pw, pia);
                const T b = (T)pa;
                s.cb[jj][kl] = b;
                s.cq[jj][kl] = (T)pq;
                s.co[jj][kl] = (T)(0.375 * pia);
                if constexpr (Shape::kLdsBB) s.cbb[jj][kl] = b * b;
            }
        }
        if constexpr (!kOrdered)
            for (int e = tid; e < kJC * 64; e += TPB) s.pj[e / 64][e % 64] = 0.0;
        __syncthreads();

        const TabPtr uc = up + (jc * kJC) * (IB * kPairVals);
        // Operands of one j step: the (i, j) terms of the wave's IPW points
        // (uniform, SGPRs) and the (j, k) terms of the lane's KR k.
        constexpr int KBB = Shape::kLdsBB ? kKR : 1;
        struct Ops {
            T u[IPW * kPairVals];
            T cb[kKR], cq[kKR], co[kKR], bb[KBB];
        };
        auto load = [&](int jj, Ops &o) {
            const TabPtr p = uc + jj * (IB * kPairVals);
#pragma unroll
            for (int e = 0; e < IPW * kPairVals; ++e) o.u[e] = p[e];
#pragma unroll
            for (int kk = 0; kk < kKR; ++kk) {
                o.cb[kk] = s.cb[jj][lane + 64 * kk];
                o.cq[kk] = s.cq[jj][lane + 64 * kk];
                o.co[kk] = s.co[jj][lane + 64 * kk];
                if constexpr (Shape::kLdsBB) o.bb[kk] = s.cbb[jj][lane + 64 * kk];
            }
        };
        // One j step: KR * IPW triples per lane.
        auto step = [&](int jj, const Ops &o) {
            T bb[kKR], sk[kKR];
#pragma unroll
            for (int kk = 0; kk < kKR; ++kk) {
                if constexpr (Shape::kLdsBB)
                    bb[kk] = o.bb[kk];
                else
                    bb[kk] = o.cb[kk] * o.cb[kk];
            }
#pragma unroll
            for (int ii = 0; ii < IPW; ++ii) {
                const T al = o.u[kPairVals * ii], wa = o.u[kPairVals * ii + 1];
                T ti = T(0);
#pragma unroll
                for (int kk = 0; kk < kKR; ++kk) {
                    const T psi =
                        tile_psi(al, ag[ii][kk], aw[ii][kk], o.cb[kk], bb[kk], o.co[kk]);
                    sk[kk] = ii ? fma(wa, psi, sk[kk]) : wa * psi;
                    ti = kk ? fma(o.cq[kk], psi, ti) : o.cq[kk] * psi;
                }
                acc_i[ii] = fma(wa, ti, acc_i[ii]);
            }
            T pj32 = T(0);
#pragma unroll
            for (int kk = 0; kk < kKR; ++kk) {
                pj32 = fma(o.cq[kk], sk[kk], pj32);
                if constexpr (sizeof(T) == 4)
                    acck32[kk % KR32] = fma(o.cq[kk], sk[kk], acck32[kk % KR32]);
                else
                    acck[kk] = fma((double)o.cq[kk], (double)sk[kk], acck[kk]);
            }
            if constexpr (kOrdered) {
                pjl[(wave * kJC + jj) * 64 + lane] = (double)pj32;
            } else {
                atomicAdd(&s.pj[jj][lane], (double)pj32);
            }
        };
        // Two operand sets: everything step jj + 1 reads is loaded while
        // step jj computes, so one wait per step covers loads issued a
        // whole step earlier (LDS and scalar loads share one counter).
        // The explicit wait + scheduling barriers keep the compiler from
        // hoisting the next set's loads above the wait for this set.
        Ops A, B;
        load(0, A);
#pragma unroll 1
        for (int jj = 0; jj < kJC; jj += 2) {
            lgkm_wait_all();
            load(jj + 1, B);
            sched_fence();
            step(jj, A);
            lgkm_wait_all();
            if (jj + 2 < kJC) load(jj + 2, A);
            sched_fence();
            step(jj + 1, B);
#if MB_FOLD_J < 16
            if constexpr (sizeof(T) == 4) {
                if (((jj + 2) % MB_FOLD_J) == 0 && jj + 2 < kJC) {
#pragma unroll
                    for (int ii = 0; ii < IPW; ++ii) {
                        acc_i64[ii] += (double)acc_i[ii];
                        acc_i[ii] = T(0);
                    }
                }
            }
#endif
        }
        // fold the short binary32 partial sums of Phi_i into binary64
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int ii = 0; ii < IPW; ++ii) {
                acc_i64[ii] += (double)acc_i[ii];
                acc_i[ii] = T(0);
            }
        }
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int kk = 0; kk < kKR; ++kk) {
                acck[kk] += (double)acck32[kk % KR32];
                acck32[kk % KR32] = T(0);
            }
        }
        __syncthreads();
        if constexpr (kOrdered) {
            // the waves' partials of each (j, lane), added in wave order
            for (int e = tid; e < kJC * 64; e += TPB) {
                double v = 0.0;
#pragma unroll
                for (int w = 0; w < Shape::NW; ++w) v += pjl[w * kJC * 64 + e];
                s.pj[e / 64][e % 64] = v;
            }
            __syncthreads();
        }
        // Phi_j of the chunk: 16 rows of 64 slots, 32 threads per row (a
        // fixed order: the two halves of a row, then a butterfly)
#pragma unroll
        for (int r0 = 0; r0 < kJC; r0 += TPB / 32) {
            const int row = r0 + (tid >> 5), c = tid & 31;
            // whole 32-lane groups drop out together, so the shuffles stay
            // inside groups that are all active
            if (row < kJC) {
                double v = s.pj[row][c] + s.pj[row][c + 32];
#pragma unroll
                for (int m = 16; m >= 1; m >>= 1) v += __shfl_xor(v, m);
                if (c == 0) s.pjacc[jc * kJC + row] = v;
            }
        }
    }

    if constexpr (kOrdered) {
        constexpr int NW = Shape::NW;
#pragma unroll
        for (int ii = 0; ii < IPW; ++ii) {
            const double v = wave_sum(sizeof(T) == 4 ? acc_i64[ii] : (double)acc_i[ii]);
            if (lane == 0) phi[wave * IPW + ii] = ix.ri(wave * IPW + ii) >= 0 ? v * out_scale : 0.0;
        }
        // the last chunk's barrier has passed: every wave is done with cb
#pragma unroll
        for (int kk = 0; kk < kKR; ++kk) s.kw[wave][lane + 64 * kk] = acck[kk];
        __syncthreads();
        for (int e = tid; e < kKT + JB; e += TPB) {
            double v = 0.0;
            if (e < kKT) {
#pragma unroll
                for (int w = 0; w < NW; ++w) v += s.kw[w][e];
                phi[IB + JB + e] = ix.rk(e) >= 0 ? v * out_scale : 0.0;
            } else {
                v = s.pjacc[e - kKT];
                phi[IB + e - kKT] = ix.rj(e - kKT) >= 0 ? v * out_scale : 0.0;
            }
        }
        return;
    }
#pragma unroll
    for (int ii = 0; ii < IPW; ++ii) {
        const double v = wave_sum(sizeof(T) == 4 ? acc_i64[ii] : (double)acc_i[ii]);
        const int i = ix.ri(wave * IPW + ii);
        if (lane == 0 && i >= 0) atomicAdd(&phi[i], v * out_scale);
    }
#pragma unroll
    for (int kk = 0; kk < kKR; ++kk) atomicAdd(&s.kacc[lane + 64 * kk], acck[kk]);
    __syncthreads();
    for (int e = tid; e < kKT + JB; e += TPB) {
        if (e < kKT) {
            const int k = ix.rk(e);
            if (k >= 0) atomicAdd(&phi[k], s.kacc[e] * out_scale);
        } else {
            const int j = ix.rj(e - kKT);
            if (j >= 0) atomicAdd(&phi[j], s.pjacc[e - kKT] * out_scale);
        }
    }
}

// One unit (I block a, J block b, K tile t) of the exhaustive sum over the
// input order; ublk is the (i, j) table block of (a, b).  kOrdered: phi is
// the unit's row and pjl the per-wave LDS slots (tile_unit).
template <typename T, typename TabPtr = const T *, bool kOrdered = false>
__device__ __forceinline__ void direct_unit(DirectLds<T> &s, const double *__restrict__ x, int n,
                                            int a, int b, int t, TabPtr ublk, double scale,
                                            double out_scale, double *__restrict__ phi,
                                            double *__restrict__ pjl = nullptr) {
    const BlockIndex<DirectLds<T>::IB, kB, DirectLds<T>::KT> ix(n, a, b, t);
    tile_unit<T, kB, DirectShape<T>, BlockIndex<DirectLds<T>::IB, kB, DirectLds<T>::KT>, TabPtr,
              kOrdered>(s, x, ix, ublk, scale, out_scale, phi, pjl);
}

}  // namespace
}  // namespace mb
