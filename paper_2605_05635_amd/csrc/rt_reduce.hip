// rt_reduce.hip -- per-image reductions (Sec. 6.2): total flux
// F = int I dX dY and the intensity-weighted centroid (X_c, Y_c), by the
// midpoint rule over pixel centres.
//
// Two passes with a fixed shape, so the result is bitwise reproducible run to
// run: kReduceBlocks workgroups each sum one contiguous slice of the image
// (coalesced reads, a fixed-order tree in LDS) into a partial triple, then one
// workgroup adds the partials in index order and forms F, X_c, Y_c.
#include "rt_kernels.h"

namespace rt {
namespace {

constexpr int kReduceThreads = 256;

__device__ __forceinline__ void block_sum3(double& a, double& b, double& c) {
    __shared__ double s0[kReduceThreads], s1[kReduceThreads], s2[kReduceThreads];
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    s2[threadIdx.x] = c;
    __syncthreads();
    for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s2[threadIdx.x] += s2[threadIdx.x + w];
        }
        __syncthreads();
    }
    a = s0[0];
    b = s1[0];
    c = s2[0];
}

__global__ __launch_bounds__(kReduceThreads) void reduce_partial(ImageConst c,
                                                                 const double* __restrict__ I,
                                                                 double* __restrict__ part) {
    const int64_t per = (c.n_pix + kReduceBlocks - 1) / kReduceBlocks;
    const int64_t lo = per * blockIdx.x;
    const int64_t hi = lo + per < c.n_pix ? lo + per : c.n_pix;
    // the row by an exact binary64 quotient, floor((p + 1/2)/nx), not a 64-bit
    // integer division (emulated in software)
    const double inv_nx = 1.0 / static_cast<double>(c.nx);
    double f = 0.0, fx = 0.0, fy = 0.0;
    for (int64_t p = lo + threadIdx.x; p < hi; p += kReduceThreads) {
        const double v = I[p];
        const int64_t iy = static_cast<int64_t>((static_cast<double>(p) + 0.5) * inv_nx);
        const int64_t ix = p - iy * c.nx;
        f += v;
        fx += (c.x0 + (static_cast<double>(ix) + 0.5) * c.dx) * v;
        fy += (c.y0 + (static_cast<double>(iy) + 0.5) * c.dy) * v;
    }
    block_sum3(f, fx, fy);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = f;
        part[3 * blockIdx.x + 1] = fx;
        part[3 * blockIdx.x + 2] = fy;
    }
}

__global__ __launch_bounds__(kReduceThreads) void reduce_final(ImageConst c,
                                                               const double* __restrict__ part,
                                                               double* __restrict__ out) {
    double f = 0.0, fx = 0.0, fy = 0.0;
    for (int b = threadIdx.x; b < kReduceBlocks; b += kReduceThreads) {
        f += part[3 * b + 0];
        fx += part[3 * b + 1];
        fy += part[3 * b + 2];
    }
    block_sum3(f, fx, fy);
    if (threadIdx.x == 0) {
        out[0] = f * c.dx * c.dy;
        out[1] = fx / f;
        out[2] = fy / f;
    }
}

}  // namespace

hipError_t launch_reduce(const ImageConst& c, const double* intensity, double* partials,
                         double* out, hipStream_t stream) {
    hipLaunchKernelGGL(reduce_partial, dim3(kReduceBlocks), dim3(kReduceThreads), 0, stream, c,
                       intensity, partials);
    hipLaunchKernelGGL(reduce_final, dim3(1), dim3(kReduceThreads), 0, stream, c, partials, out);
    return hipGetLastError();
}

}  // namespace rt
