// rt_reduce.hip -- per-image reductions (Sec. 6.2): total flux
// F = int I dX dY and the intensity-weighted centroid (X_c, Y_c), by the
// midpoint rule over pixel centres.
//
// One workgroup of 1024 threads per image.  Each thread accumulates a fixed
// strided subset of pixels, then a fixed-shape tree in LDS combines the
// partial sums, so the result is bitwise reproducible run to run.
#include "rt_kernels.h"

namespace rt {
namespace {

constexpr int kReduceThreads = 1024;

__global__ __launch_bounds__(kReduceThreads) void reduce_kernel(ImageConst c,
                                                                const double* __restrict__ I,
                                                                double* __restrict__ out) {
    __shared__ double s0[kReduceThreads], s1[kReduceThreads], s2[kReduceThreads];
    double f = 0.0, fx = 0.0, fy = 0.0;
    for (int64_t p = threadIdx.x; p < c.n_pix; p += kReduceThreads) {
        const double v = I[p];
        const int64_t iy = p / c.nx;
        const int64_t ix = p - iy * c.nx;
        const double X = c.x0 + (static_cast<double>(ix) + 0.5) * c.dx;
        const double Y = c.y0 + (static_cast<double>(iy) + 0.5) * c.dy;
        f += v;
        fx += X * v;
        fy += Y * v;
    }
    s0[threadIdx.x] = f;
    s1[threadIdx.x] = fx;
    s2[threadIdx.x] = fy;
    __syncthreads();
    for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s2[threadIdx.x] += s2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s0[0] * c.dx * c.dy;
        out[1] = s1[0] / s0[0];
        out[2] = s2[0] / s0[0];
    }
}

}  // namespace

hipError_t launch_reduce(const ImageConst& c, const double* intensity, double* out,
                         hipStream_t stream) {
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kReduceThreads), 0, stream, c, intensity,
                       out);
    return hipGetLastError();
}

}  // namespace rt
