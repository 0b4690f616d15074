// rt_visibility.hip -- normalised visibility amplitudes of a traced image
// (Sec. 6.4, eqs. (108)-(109)):
//   V(u,v) = sum_{pixels} I(X,Y) exp(-2 pi i (u X + v Y)) dX dY,
//   amp(u,v) = |V(u,v)| / |V(0,0)|,
// the midpoint rule over the pixel centres, at K arbitrary (u, v) points.
//
// The phase factorises over the screen axes, exp(-2 pi i u X) exp(-2 pi i v Y),
// so with Ex[k][x] = exp(-2 pi i u_k X_x)
//   A[k][y] = sum_x Ex[k][x] I[y][x]          (a dense real-by-complex product)
//   V_k     = dX dY sum_y exp(-2 pi i v_k Y_y) A[k][y].
// The first contraction, 4 K nx ny flops, is one FP64 GEMM of the stacked
// [Re Ex; Im Ex] (2K x nx) with the image (rocBLAS, on the matrix cores); the
// second, 8 K ny flops plus K ny phases, is a small kernel that forms partial
// sums over blocks of rows in a fixed order, then one kernel adds them in
// index order and normalises by the flux.  Deterministic run to run.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cstdint>

#include "rt_kernels.h"
#include "rt_math.h"

namespace rt {
namespace {

constexpr double kTwoPi = 6.283185307179586;
constexpr int kVisThreads = 256;
constexpr int kRowsPerBlock = 32;

// Ex2[j][x], j < K: cos(2 pi u_j X_x); K <= j < 2K: -sin(2 pi u_{j-K} X_x).
__global__ void phase_table(const double* __restrict__ uv, int32_t K, int32_t nx, double x0,
                            double dx, double* __restrict__ ex2) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= static_cast<int64_t>(K) * nx) return;
    const int32_t k = static_cast<int32_t>(i / nx);
    const int32_t x = static_cast<int32_t>(i - static_cast<int64_t>(k) * nx);
    const double X = x0 + (static_cast<double>(x) + 0.5) * dx;
    double s, c;
    dm::sincos(kTwoPi * uv[2 * k] * X, &s, &c);
    ex2[static_cast<int64_t>(k) * nx + x] = c;
    ex2[static_cast<int64_t>(k + K) * nx + x] = -s;
}

// Partial V_k over rows [b kRowsPerBlock, (b+1) kRowsPerBlock): thread per k
// (coalesced reads of the GEMM result A, column-major 2K x ny).
__global__ void row_phase_partials(const double* __restrict__ A, const double* __restrict__ uv,
                                   int32_t K, int32_t ny, double y0, double dy,
                                   double* __restrict__ part) {
    const int32_t k = static_cast<int32_t>(blockIdx.x) * kVisThreads + threadIdx.x;
    if (k >= K) return;
    const int32_t b = blockIdx.y;
    const int32_t lo = b * kRowsPerBlock;
    const int32_t hi = lo + kRowsPerBlock < ny ? lo + kRowsPerBlock : ny;
    const double v = uv[2 * k + 1];
    double re = 0.0, im = 0.0;
    for (int32_t y = lo; y < hi; ++y) {
        const double Y = y0 + (static_cast<double>(y) + 0.5) * dy;
        double s, c;
        dm::sincos(kTwoPi * v * Y, &s, &c);          // exp(-i phi) = c - i s
        const double ar = A[static_cast<int64_t>(y) * 2 * K + k];
        const double ai = A[static_cast<int64_t>(y) * 2 * K + K + k];
        re += c * ar + s * ai;
        im += c * ai - s * ar;
    }
    part[(static_cast<int64_t>(b) * K + k) * 2] = re;
    part[(static_cast<int64_t>(b) * K + k) * 2 + 1] = im;
}

__global__ void finish_amplitudes(const double* __restrict__ part, int32_t K, int32_t nblocks,
                                  double dxdy, const double* __restrict__ flux,
                                  double* __restrict__ amp, double* __restrict__ vis) {
    const int32_t k = static_cast<int32_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= K) return;
    double re = 0.0, im = 0.0;
    for (int32_t b = 0; b < nblocks; ++b) {
        re += part[(static_cast<int64_t>(b) * K + k) * 2];
        im += part[(static_cast<int64_t>(b) * K + k) * 2 + 1];
    }
    re *= dxdy;
    im *= dxdy;
    if (vis) {
        vis[2 * k] = re;
        vis[2 * k + 1] = im;
    }
    if (amp) amp[k] = sqrt(re * re + im * im) / fabs(flux[0]);
}

}  // namespace

size_t visibility_scratch_bytes(int32_t K, int32_t nx, int32_t ny) {
    const size_t nblocks = (static_cast<size_t>(ny) + kRowsPerBlock - 1) / kRowsPerBlock;
    return sizeof(double) * (2ull * K * nx + 2ull * K * ny + 2ull * K * nblocks + 8);
}

hipError_t launch_visibility(void* blas, const ImageConst& c, const double* intensity,
                             const double* uv, int32_t K, double* flux, double* amp, double* vis,
                             double* scratch, double* reduce_partials, hipStream_t stream,
                             const char** what) {
    const int32_t nx = c.nx, ny = c.ny;
    const int64_t nblocks = (ny + kRowsPerBlock - 1) / kRowsPerBlock;
    double* ex2 = scratch;                                         // 2K x nx
    double* A = ex2 + 2ll * K * nx;                                // column-major 2K x ny
    double* part = A + 2ll * K * ny;                               // nblocks x K x 2
    hipError_t e = launch_reduce(c, intensity, reduce_partials, flux, stream);
    if (e != hipSuccess) { *what = "flux reduction"; return e; }
    const int64_t n = static_cast<int64_t>(K) * nx;
    hipLaunchKernelGGL(phase_table, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                       stream, uv, K, nx, c.x0, c.dx, ex2);
    if ((e = hipGetLastError()) != hipSuccess) { *what = "phase table"; return e; }
    // A (2K x ny, column-major) = Ex2 (2K x nx) . I^T, with Ex2 stored
    // row-major = column-major nx x 2K (transposed operand) and the image
    // I[y][x] = column-major nx x ny.
    rocblas_handle h = static_cast<rocblas_handle>(blas);
    const double one = 1.0, zero = 0.0;
    if (rocblas_set_stream(h, stream) != rocblas_status_success ||
        rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, 2 * K, ny, nx, &one,
                      ex2, nx, intensity, nx, &zero, A, 2 * K) != rocblas_status_success) {
        *what = "rocblas_dgemm";
        return hipErrorLaunchFailure;
    }
    hipLaunchKernelGGL(row_phase_partials,
                       dim3(static_cast<unsigned>((K + kVisThreads - 1) / kVisThreads),
                            static_cast<unsigned>(nblocks)),
                       dim3(kVisThreads), 0, stream, A, uv, K, ny, c.y0, c.dy, part);
    if ((e = hipGetLastError()) != hipSuccess) { *what = "row phases"; return e; }
    hipLaunchKernelGGL(finish_amplitudes, dim3(static_cast<unsigned>((K + 255) / 256)), dim3(256),
                       0, stream, part, K, static_cast<int32_t>(nblocks), c.dx * c.dy, flux, amp,
                       vis);
    if ((e = hipGetLastError()) != hipSuccess) { *what = "amplitudes"; return e; }
    return hipSuccess;
}

void* blas_create() {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) return nullptr;
    return h;
}

}  // namespace rt
