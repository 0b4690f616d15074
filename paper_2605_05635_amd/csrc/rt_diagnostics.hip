// rt_diagnostics.hip -- image-level morphology diagnostics of a raw intensity
// map (Sec. 6.2) and its origin-centred radial profile with the bright-peak
// scale (Sec. 6.3), by the midpoint rule over pixel centres.
//
// Fixed-shape passes, so every result is bitwise reproducible: flux and
// centroid (the reduce kernels), then one pass for the moments about the
// centroid that need only the centroid (sum rho I, the fluxes right and left
// of X_c, the emitting pixels' sum and count, the peak intensity), one pass
// for the width about the mean radius, one workgroup per radial bin for the
// profile (its threads take whole rows and visit only the columns that can
// reach its annulus, keeping the pixels whose bin is exactly its own), and one
// workgroup that picks the first bin of largest mean.
#include <mutex>

#include "rt_kernels.h"

namespace rt {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double s[kThreads];
    __syncthreads();
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    return s[0];
}

__device__ __forceinline__ double block_max(double v) {
    __shared__ double s[kThreads];
    __syncthreads();
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    return s[0];
}

// Pixel centre coordinates, one rounding per operation (no contraction), the
// way the screen is written down: X = x_min + (ix + 1/2) dx.
__device__ __forceinline__ double centre(double x0, double d, int64_t i) {
    const double t = (static_cast<double>(i) + 0.5) * d;
    return x0 + t;
}

constexpr int kA = 6;   // sum rho I, F_R, F_L, emitting sum, emitting count, max I

__global__ __launch_bounds__(kThreads) void diag_a_partial(ImageConst c, const double* __restrict__ I,
                                                           const double* __restrict__ fc,
                                                           double* __restrict__ part) {
    const double xc = fc[1], yc = fc[2];
    const int64_t per = (c.n_pix + kReduceBlocks - 1) / kReduceBlocks;
    const int64_t lo = per * blockIdx.x;
    const int64_t hi = lo + per < c.n_pix ? lo + per : c.n_pix;
    double srho = 0.0, fr = 0.0, fl = 0.0, se = 0.0, ne = 0.0, mx = -INFINITY;
    for (int64_t p = lo + threadIdx.x; p < hi; p += kThreads) {
        const double v = I[p];
        const int64_t iy = p / c.nx;
        const int64_t ix = p - iy * c.nx;
        const double X = centre(c.x0, c.dx, ix), Y = centre(c.y0, c.dy, iy);
        srho += sqrt((X - xc) * (X - xc) + (Y - yc) * (Y - yc)) * v;
        if (X > xc) fr += v;
        if (X < xc) fl += v;
        if (v > 0.0) {
            se += v;
            ne += 1.0;
        }
        mx = fmax(mx, v);
    }
    const double r[kA] = {block_sum(srho), block_sum(fr), block_sum(fl), block_sum(se),
                          block_sum(ne), block_max(mx)};
    if (threadIdx.x == 0)
        for (int j = 0; j < kA; ++j) part[kA * blockIdx.x + j] = r[j];
}

// out: F, X_c, Y_c, C, rho_bar, d_img, (w, w/d later), A_LR, I_max, <I>_img, P
__global__ __launch_bounds__(kThreads) void diag_a_final(ImageConst c, const double* __restrict__ part,
                                                         const double* __restrict__ fc,
                                                         double* __restrict__ out) {
    double v[kA] = {0.0, 0.0, 0.0, 0.0, 0.0, -INFINITY};
    for (int b = threadIdx.x; b < kReduceBlocks; b += kThreads) {
        for (int j = 0; j < 5; ++j) v[j] += part[kA * b + j];
        v[5] = fmax(v[5], part[kA * b + 5]);
    }
    const double srho = block_sum(v[0]), fr = block_sum(v[1]), fl = block_sum(v[2]),
                 se = block_sum(v[3]), ne = block_sum(v[4]), mx = block_max(v[5]);
    if (threadIdx.x == 0) {
        const double F = fc[0], xc = fc[1], yc = fc[2];
        const double rho_bar = srho * c.dx * c.dy / F;
        const double mean = ne > 0.0 ? se / ne : 0.0;
        out[0] = F;
        out[1] = xc;
        out[2] = yc;
        out[3] = sqrt(xc * xc + yc * yc);
        out[4] = rho_bar;
        out[5] = 2.0 * rho_bar;
        out[8] = (fr - fl) / (fr + fl);
        out[9] = mx;
        out[10] = mean;
        out[11] = mean > 0.0 ? mx / mean : 0.0;
    }
}

__global__ __launch_bounds__(kThreads) void diag_b_partial(ImageConst c, const double* __restrict__ I,
                                                           const double* __restrict__ out,
                                                           double* __restrict__ part) {
    const double xc = out[1], yc = out[2], rho_bar = out[4];
    const int64_t per = (c.n_pix + kReduceBlocks - 1) / kReduceBlocks;
    const int64_t lo = per * blockIdx.x;
    const int64_t hi = lo + per < c.n_pix ? lo + per : c.n_pix;
    double s = 0.0;
    for (int64_t p = lo + threadIdx.x; p < hi; p += kThreads) {
        const int64_t iy = p / c.nx;
        const int64_t ix = p - iy * c.nx;
        const double X = centre(c.x0, c.dx, ix), Y = centre(c.y0, c.dy, iy);
        const double d = sqrt((X - xc) * (X - xc) + (Y - yc) * (Y - yc)) - rho_bar;
        s += d * d * I[p];
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void diag_b_final(ImageConst c, const double* __restrict__ part,
                                                         double* __restrict__ out) {
    double s = 0.0;
    for (int b = threadIdx.x; b < kReduceBlocks; b += kThreads) s += part[b];
    s = block_sum(s);
    if (threadIdx.x == 0) {
        const double w = sqrt(s * c.dx * c.dy / out[0]);
        out[6] = w;
        out[7] = w / out[5];
    }
}

// Radial bin of a pixel centre: floor(rho_0 / bw), each operation rounded once.
__device__ __forceinline__ int64_t radial_bin(double X, double Y, double bw) {
    const double xx = X * X;
    const double yy = Y * Y;
    const double s = xx + yy;
    return static_cast<int64_t>(floor(sqrt(s) / bw));
}

// One workgroup per bin k: the mean intensity of the pixels with
// floor(rho_0 / bw) == k (NaN if none).  Each thread takes whole rows (rows
// t, t + 256, ...): it visits the column runs of its row that can reach the
// annulus [k bw, (k + 1) bw), widened by two pixels on each side, and keeps
// the pixels of exactly this bin; rows farther than the annulus are skipped.
// A thread's rows and pixels go in a fixed order, then a fixed-order tree
// over the threads.  (dx, dy > 0: the screen extent is validated.)
__global__ __launch_bounds__(kThreads) void profile_kernel(ImageConst c, const double* __restrict__ I,
                                                           double bw, double* __restrict__ profile) {
    const int64_t k = blockIdx.x;
    const double r_lo = static_cast<double>(k) * bw, r_hi = static_cast<double>(k + 1) * bw;
    const double inv_dx = 1.0 / c.dx;   // column bounds only: the margins absorb its rounding
    auto first_col = [&](double a) {
        const double f = floor((a - c.x0) * inv_dx - 0.5);
        return f < 0.0 ? int64_t(0) : static_cast<int64_t>(fmin(f, static_cast<double>(c.nx)));
    };
    auto last_col = [&](double b) {
        const double f = ceil((b - c.x0) * inv_dx - 0.5);
        return f > static_cast<double>(c.nx - 1) ? static_cast<int64_t>(c.nx - 1)
                                                 : static_cast<int64_t>(fmax(f, -1.0));
    };
    double s = 0.0, n = 0.0;
    for (int64_t iy = threadIdx.x; iy < c.ny; iy += kThreads) {
        const double Y = centre(c.y0, c.dy, iy);
        if (fabs(Y) > r_hi + c.dy) continue;
        const double xo = sqrt(fmax(0.0, r_hi * r_hi - Y * Y)) + 2.0 * c.dx;
        const double xi = fmax(0.0, sqrt(fmax(0.0, r_lo * r_lo - Y * Y)) - 2.0 * c.dx);
        const int64_t a0 = first_col(-xo), a1 = last_col(-xi);
        const int64_t b0 = first_col(xi), b1 = last_col(xo);
        const bool one = b0 <= a1 + 1;   // the runs touch: visit [a0, b1] once
        const double* row = I + iy * c.nx;
        for (int run = 0; run < (one ? 1 : 2); ++run) {
            const int64_t lo = run == 0 ? a0 : b0;
            const int64_t hi = one ? b1 : (run == 0 ? a1 : b1);
            // four pixels a round: their loads are issued together, the sums
            // still taken in column order
            for (int64_t ix = lo; ix <= hi; ix += 4) {
                double v[4];
                bool in[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t j = ix + u;
                    in[u] = j <= hi && radial_bin(centre(c.x0, c.dx, j), Y, bw) == k;
                    v[u] = in[u] ? row[j] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (in[u]) {
                        s += v[u];
                        n += 1.0;
                    }
                }
            }
        }
    }
    s = block_sum(s);
    n = block_sum(n);
    if (threadIdx.x == 0) profile[k] = n > 0.0 ? s / n : __builtin_nan("");
}

// The first bin of largest mean (empty bins skipped): out[12] = its centre,
// out[13] = twice that.
__global__ __launch_bounds__(kThreads) void peak_kernel(const double* __restrict__ profile,
                                                        int32_t n_bins, double bw,
                                                        double* __restrict__ out) {
    __shared__ double sv[kThreads];
    __shared__ int32_t si[kThreads];
    double best = -INFINITY;
    int32_t bi = n_bins;
    for (int32_t k = threadIdx.x; k < n_bins; k += kThreads) {
        const double v = profile[k];
        if (v > best) {   // NaN never wins; strict: the first of equal values in this thread
            best = v;
            bi = k;
        }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) {
            const double v2 = sv[threadIdx.x + w];
            const int32_t i2 = si[threadIdx.x + w];
            if (v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 < si[threadIdx.x])) {
                sv[threadIdx.x] = v2;
                si[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int32_t k = si[0] < n_bins ? si[0] : 0;
        const double rho = (static_cast<double>(k) + 0.5) * bw;
        out[12] = rho;
        out[13] = 2.0 * rho;
    }
}

// delta[i] = (q[i] - ref[i]) / ref[i].
__global__ void relative_kernel(const double* __restrict__ q, const double* __restrict__ ref,
                                int32_t n, double* __restrict__ delta) {
    const int32_t i = static_cast<int32_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) delta[i] = (q[i] - ref[i]) / ref[i];
}

}  // namespace

hipError_t launch_relative(const double* q, const double* ref, int32_t n, double* delta,
                           hipStream_t stream) {
    hipLaunchKernelGGL(relative_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                       stream, q, ref, n, delta);
    return hipGetLastError();
}

size_t diagnostics_scratch_doubles(int32_t n_bins) {
    return 3 + 3 * kReduceBlocks + kA * kReduceBlocks + kReduceBlocks + static_cast<size_t>(n_bins);
}

// Work memory of rt_image_diagnostics_noalloc: the partial sums and, when the
// caller passes no profile, up to kNoAllocMaxBins profile bins (~533 KB).
// Each device the library runs on holds its own copy until the process ends.
// In host code `scratch` names a host-side stand-in, never a device address:
// kernels get the address that hipGetSymbolAddress returns for the current
// device.
constexpr size_t kStaticWorkDoubles = 3 + (3 + kA + 1) * kReduceBlocks + kNoAllocMaxBins;
static __device__ __align__(256) double scratch[kStaticWorkDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_work_mu;
double* g_static_work[kMaxDevices] = {};   // device address of `scratch` per device
}  // namespace

hipError_t diagnostics_static_work(double** ptr, size_t* doubles) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_static_work_mu);
    if (!g_static_work[dev]) {
        double* p = nullptr;
        e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_static_work[dev] = p;
    }
    *ptr = g_static_work[dev];
    *doubles = kStaticWorkDoubles;
    return hipSuccess;
}

hipError_t launch_diagnostics(const ImageConst& c, const double* intensity, double bw,
                              int32_t n_bins, double* out, double* profile, double* work,
                              hipStream_t stream) {
    double* fc = work;                               // F, X_c, Y_c
    double* p3 = fc + 3;                             // flux / centroid partials
    double* pa = p3 + 3 * kReduceBlocks;
    double* pb = pa + kA * kReduceBlocks;
    double* prof = profile ? profile : pb + kReduceBlocks;
    hipError_t e = launch_reduce(c, intensity, p3, fc, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(diag_a_partial, dim3(kReduceBlocks), dim3(kThreads), 0, stream, c,
                       intensity, fc, pa);
    hipLaunchKernelGGL(diag_a_final, dim3(1), dim3(kThreads), 0, stream, c, pa, fc, out);
    hipLaunchKernelGGL(diag_b_partial, dim3(kReduceBlocks), dim3(kThreads), 0, stream, c,
                       intensity, out, pb);
    hipLaunchKernelGGL(diag_b_final, dim3(1), dim3(kThreads), 0, stream, c, pb, out);
    hipLaunchKernelGGL(profile_kernel, dim3(n_bins), dim3(kThreads), 0, stream, c, intensity, bw,
                       prof);
    hipLaunchKernelGGL(peak_kernel, dim3(1), dim3(kThreads), 0, stream, prof, n_bins, bw, out);
    return hipGetLastError();
}

}  // namespace rt
