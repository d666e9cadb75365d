// The three-body far-field expansion (Section 3.2) of one pair of source
// sets at a list of target points: the routine the traversal applies to
// its well-separated pruned node triples (farfield.hpp), exposed on its own.
#include "farfield.hpp"
#include "mb_internal.hpp"

namespace mb {
namespace {

// Centroid and second moments sum (y - c)(y - c)^T of a point set, by one
// workgroup: out = [c0, c1, c2, s00, s01, s02, s11, s12, s22].
__global__ __launch_bounds__(256) void set_moments_kernel(const double *__restrict__ y, int64_t n,
                                                          double *__restrict__ out) {
    __shared__ double red[256];
    __shared__ double c[3];
    const int tid = threadIdx.x;
    auto block_sum = [&](double v) -> double {
        red[tid] = v;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (tid < h) red[tid] += red[tid + h];
            __syncthreads();
        }
        const double r = red[0];
        __syncthreads();
        return r;
    };
    for (int d = 0; d < 3; ++d) {
        double s = 0.0;
        for (int64_t i = tid; i < n; i += 256) s += y[3 * i + d];
        const double tot = block_sum(s);
        if (tid == 0) c[d] = tot / (double)n;
        __syncthreads();
    }
    const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
    for (int m = 0; m < 6; ++m) {
        double s = 0.0;
        for (int64_t i = tid; i < n; i += 256)
            s += (y[3 * i + pa[m]] - c[pa[m]]) * (y[3 * i + pb[m]] - c[pb[m]]);
        const double tot = block_sum(s);
        if (tid == 0) out[3 + m] = tot;
    }
    if (tid < 3) out[tid] = c[tid];
}

__global__ void farfield_points_kernel(const double *__restrict__ x, int64_t nx,
                                       const double *__restrict__ my,
                                       const double *__restrict__ mz, double ny, double nz,
                                       int order, double *__restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nx) return;
    const double xi[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
    out[i] = farfield_value(xi, my, mz, ny, nz, my + 3, mz + 3, order);
}

}  // namespace

mb_status farfield_eval(const double *x, int64_t nx, const double *y, int64_t ny, const double *z,
                        int64_t nz, int order, double *out, hipStream_t s) {
    Scratch sc;
    mb_status st = sc.alloc(sizeof(double) * 18, s);
    if (st != MB_OK) return st;
    double *m = sc.as<double>();
    set_moments_kernel<<<1, 256, 0, s>>>(y, ny, m);
    set_moments_kernel<<<1, 256, 0, s>>>(z, nz, m + 9);
    if (nx > 0)
        farfield_points_kernel<<<(unsigned)((nx + 255) / 256), 256, 0, s>>>(
            x, nx, m, m + 9, (double)ny, (double)nz, order, out);
    MB_HIP(hipGetLastError());
    return MB_OK;
}

}  // namespace mb
