// rt_diagnostics.hip -- image-level morphology diagnostics of a raw intensity
// map (Sec. 6.2) and its origin-centred radial profile with the bright-peak
// scale (Sec. 6.3), by the midpoint rule over pixel centres.
//
// Four launches of fixed shape, so every result is bitwise reproducible:
//   1. the flux and centroid partial sums (each of kReduceBlocks workgroups
//      one contiguous slice of the image) beside the radial profile, one
//      workgroup per bin (its threads take whole rows and visit only the
//      columns that can reach its annulus, keeping the pixels whose bin is
//      exactly its own): the profile needs none of the moments;
//   2. the moments about the centroid (sum rho I, the fluxes right and left of
//      X_c, the emitting pixels' sum and count, the peak intensity), each
//      workgroup first forming F, X_c, Y_c itself from the partial sums;
//   3. the width about the mean radius, each workgroup first forming the
//      moments' totals the same way;
//   4. one workgroup: the width and the first bin of largest mean.
// Every total is a fixed-order sum of fixed partial sums.  Workgroups of 1024
// threads: the passes are latency-bound (8 bytes a pixel), and a profile bin
// then takes one row per thread.
#include <mutex>

#include "rt_kernels.h"

namespace rt {
namespace {

constexpr int kThreads = 1024;

constexpr int kWaves = kThreads / 64;

// Block-wide sums (and, for `maxes`, maxima) of N values per thread, every
// thread receiving the totals: a butterfly over each wavefront's 64 lanes
// (shuffles, no barrier), then each thread adds the kWaves wavefront totals
// in wavefront order.  A fixed order throughout, so the totals are bitwise
// reproducible; two barriers for the whole set.
template <int N>
__device__ __forceinline__ void block_reduce(double (&v)[N], int maxes = 0) {
    __shared__ double s[N][kWaves];
    for (int j = 0; j < N; ++j)
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(v[j], off);
            v[j] = j >= N - maxes ? fmax(v[j], o) : v[j] + o;
        }
    const int w = static_cast<int>(threadIdx.x) / 64;
    __syncthreads();   // earlier readers of s are done
    if (__lane_id() == 0)
        for (int j = 0; j < N; ++j) s[j][w] = v[j];
    __syncthreads();
    for (int j = 0; j < N; ++j) {
        double t = s[j][0];
        for (int i = 1; i < kWaves; ++i) t = j >= N - maxes ? fmax(t, s[j][i]) : t + s[j][i];
        v[j] = t;
    }
}

// Row of pixel p of a screen nx pixels wide, inv_nx = 1/nx: floor((p + 1/2)
// inv_nx) is exact (its fraction stays 1/(2 nx) away from an integer, its
// rounding error is ~2e-16 p/nx), where a 64-bit integer division would be
// emulated in software.
__device__ __forceinline__ int64_t row_of(int64_t p, double inv_nx) {
    return static_cast<int64_t>((static_cast<double>(p) + 0.5) * inv_nx);
}

// Pixel centre coordinates, one rounding per operation (no contraction), the
// way the screen is written down: X = x_min + (ix + 1/2) dx.
__device__ __forceinline__ double centre(double x0, double d, int64_t i) {
    const double t = (static_cast<double>(i) + 0.5) * d;
    return x0 + t;
}

constexpr int kA = 6;   // sum rho I, F_R, F_L, emitting sum, emitting count, max I
constexpr int kSeg = 8;      // pixels of a profile segment, whose loads are issued together
constexpr int kPer = 4;      // pixels of a slice per thread and round, loaded together

// Flux and centroid partial sums of slice blk.
__device__ __forceinline__ void flux_partial(const ImageConst& c, const double* __restrict__ I,
                                             int blk, double* __restrict__ part) {
    const int64_t per = (c.n_pix + kReduceBlocks - 1) / kReduceBlocks;
    const double inv_nx = 1.0 / static_cast<double>(c.nx);
    const int64_t lo = per * blk;
    const int64_t hi = lo + per < c.n_pix ? lo + per : c.n_pix;
    double f = 0.0, fx = 0.0, fy = 0.0;
    for (int64_t p0 = lo + threadIdx.x; p0 < hi; p0 += kPer * kThreads) {
        double vv[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t p = p0 + u * kThreads;
            vv[u] = I[p < hi ? p : p0];   // p0 < hi
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t p = p0 + u * kThreads;
            if (p >= hi) break;
            const double v = vv[u];
            const int64_t iy = row_of(p, inv_nx);
            const int64_t ix = p - iy * c.nx;
            f += v;
            fx += (c.x0 + (static_cast<double>(ix) + 0.5) * c.dx) * v;
            fy += (c.y0 + (static_cast<double>(iy) + 0.5) * c.dy) * v;
        }
    }
    double t[3] = {f, fx, fy};
    block_reduce(t);
    if (threadIdx.x == 0) {
        part[3 * blk + 0] = t[0];
        part[3 * blk + 1] = t[1];
        part[3 * blk + 2] = t[2];
    }
}

// F, X_c, Y_c from the flux partial sums (thread t takes partial t).
__device__ __forceinline__ void flux_total(const ImageConst& c, const double* __restrict__ part,
                                           double fc[3]) {
    double f = 0.0, fx = 0.0, fy = 0.0;
    for (int b = threadIdx.x; b < kReduceBlocks; b += kThreads) {
        f += part[3 * b + 0];
        fx += part[3 * b + 1];
        fy += part[3 * b + 2];
    }
    double t[3] = {f, fx, fy};
    block_reduce(t);
    fc[0] = t[0] * c.dx * c.dy;
    fc[1] = t[1] / t[0];
    fc[2] = t[2] / t[0];
}

// Radial bin of a pixel centre: floor(rho_0 / bw), each operation rounded once.
__device__ __forceinline__ int64_t radial_bin(double X, double Y, double bw) {
    const double xx = X * X;
    const double yy = Y * Y;
    const double s = xx + yy;
    return static_cast<int64_t>(floor(sqrt(s) / bw));
}

// Bin k of the profile: the mean intensity of the pixels with
// floor(rho_0 / bw) == k (NaN if none).  A row of the screen meets the
// annulus [k bw, (k + 1) bw) in at most two column runs; widened by two pixels
// on each side they hold every pixel of the bin in that row.  Rows go in
// batches of kThreads: thread t finds the runs of row base + t (none for rows
// farther than the annulus) and cuts them into segments of kSeg pixels; a
// scan over the block numbers the segments, and thread t then takes segments
// t, t + kThreads, ... (a binary search over the scan finds a segment's row),
// so long runs (rows nearly tangent to the annulus) are shared out rather
// than left to one lane.  Each visited pixel is kept when its bin is exactly
// k.  Every thread's segments go in a fixed order, then a fixed-order
// reduction over the threads.  (dx, dy > 0: the screen extent is validated.)
__device__ __forceinline__ void profile_bin(const ImageConst& c, const double* __restrict__ I,
                                            double bw, int64_t k, double* __restrict__ profile) {
    __shared__ int32_t run[kThreads][4];   // a0, a1, b0, b1 (a1 < a0: no run)
    __shared__ int32_t first[kThreads];    // exclusive scan of the segment counts
    __shared__ int32_t total;
    const double r_lo = static_cast<double>(k) * bw, r_hi = static_cast<double>(k + 1) * bw;
    const double inv_dx = 1.0 / c.dx;   // column bounds only: the margins absorb its rounding
    auto first_col = [&](double a) {
        const double f = floor((a - c.x0) * inv_dx - 0.5);
        return f < 0.0 ? int32_t(0) : static_cast<int32_t>(fmin(f, static_cast<double>(c.nx)));
    };
    auto last_col = [&](double b) {
        const double f = ceil((b - c.x0) * inv_dx - 0.5);
        return f > static_cast<double>(c.nx - 1) ? static_cast<int32_t>(c.nx - 1)
                                                 : static_cast<int32_t>(fmax(f, -1.0));
    };
    const int t = static_cast<int>(threadIdx.x);
    double s = 0.0, n = 0.0;
    for (int64_t base = 0; base < c.ny; base += kThreads) {
        const int64_t iy = base + t;
        int32_t a0 = 0, a1 = -1, b0 = 0, b1 = -1;
        if (iy < c.ny) {
            const double Y = centre(c.y0, c.dy, iy);
            if (!(fabs(Y) > r_hi + c.dy)) {
                const double xo = sqrt(fmax(0.0, r_hi * r_hi - Y * Y)) + 2.0 * c.dx;
                const double xi = fmax(0.0, sqrt(fmax(0.0, r_lo * r_lo - Y * Y)) - 2.0 * c.dx);
                a0 = first_col(-xo);
                a1 = last_col(-xi);
                b0 = first_col(xi);
                b1 = last_col(xo);
                if (b0 <= a1 + 1) {   // the runs touch: one run [a0, b1]
                    a1 = b1;
                    b0 = 0;
                    b1 = -1;
                }
            }
        }
        run[t][0] = a0;
        run[t][1] = a1;
        run[t][2] = b0;
        run[t][3] = b1;
        const int32_t na = a1 >= a0 ? (a1 - a0 + kSeg) / kSeg : 0;
        const int32_t nb = b1 >= b0 ? (b1 - b0 + kSeg) / kSeg : 0;
        // inclusive scan of na + nb over the block (Hillis-Steele in LDS)
        first[t] = na + nb;
        __syncthreads();
        for (int off = 1; off < kThreads; off <<= 1) {
            const int32_t add = t >= off ? first[t - off] : 0;
            __syncthreads();
            first[t] += add;
            __syncthreads();
        }
        if (t == kThreads - 1) total = first[t];
        __syncthreads();
        const int32_t n_seg = total;
        for (int32_t g = t; g < n_seg; g += kThreads) {
            // the row whose segments include g: the first r with first[r] > g
            int32_t lo = 0, hi = kThreads - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (first[mid] > g) hi = mid; else lo = mid + 1;
            }
            const int32_t r = lo;
            const int32_t before = r > 0 ? first[r - 1] : 0;
            int32_t j = g - before;   // segment index within row r
            const int32_t ra0 = run[r][0], ra1 = run[r][1], rb0 = run[r][2], rb1 = run[r][3];
            const int32_t nra = ra1 >= ra0 ? (ra1 - ra0 + kSeg) / kSeg : 0;
            int32_t x0, x1;
            if (j < nra) {
                x0 = ra0 + j * kSeg;
                x1 = x0 + kSeg - 1 < ra1 ? x0 + kSeg - 1 : ra1;
            } else {
                j -= nra;
                x0 = rb0 + j * kSeg;
                x1 = x0 + kSeg - 1 < rb1 ? x0 + kSeg - 1 : rb1;
            }
            const int64_t row_y = base + r;
            const double Y = centre(c.y0, c.dy, row_y);
            const double* row = I + row_y * c.nx;
            double v[kSeg];
            bool in[kSeg];
#pragma unroll
            for (int u = 0; u < kSeg; ++u) {
                const int32_t x = x0 + u;
                in[u] = x <= x1 && radial_bin(centre(c.x0, c.dx, x), Y, bw) == k;
                const double val = row[in[u] ? x : x0];   // x0 is in the row
                v[u] = in[u] ? val : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kSeg; ++u) {
                if (in[u]) {
                    s += v[u];
                    n += 1.0;
                }
            }
        }
        __syncthreads();   // run and first are rewritten by the next batch
    }
    double tt[2] = {s, n};
    block_reduce(tt);
    if (threadIdx.x == 0) profile[k] = tt[1] > 0.0 ? tt[0] / tt[1] : __builtin_nan("");
}

// Launch 1: workgroups [0, kReduceBlocks) the flux partial sums, then one
// workgroup per profile bin.
__global__ __launch_bounds__(kThreads) void diag_first(ImageConst c, const double* __restrict__ I,
                                                       double bw, double* __restrict__ p3,
                                                       double* __restrict__ profile) {
    const int64_t b = blockIdx.x;
    if (b < kReduceBlocks)
        flux_partial(c, I, static_cast<int>(b), p3);
    else
        profile_bin(c, I, bw, b - kReduceBlocks, profile);
}

// Launch 2: F, X_c, Y_c (workgroup 0 stores them in fc), then the moments'
// partial sums of slice blk.
__global__ __launch_bounds__(kThreads) void diag_a_partial(ImageConst c, const double* __restrict__ I,
                                                           const double* __restrict__ p3,
                                                           double* __restrict__ fc_out,
                                                           double* __restrict__ part) {
    double fc[3];
    flux_total(c, p3, fc);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int j = 0; j < 3; ++j) fc_out[j] = fc[j];
    const double xc = fc[1], yc = fc[2];
    const int64_t per = (c.n_pix + kReduceBlocks - 1) / kReduceBlocks;
    const double inv_nx = 1.0 / static_cast<double>(c.nx);
    const int64_t lo = per * blockIdx.x;
    const int64_t hi = lo + per < c.n_pix ? lo + per : c.n_pix;
    double srho = 0.0, fr = 0.0, fl = 0.0, se = 0.0, ne = 0.0, mx = -INFINITY;
    for (int64_t p0 = lo + threadIdx.x; p0 < hi; p0 += kPer * kThreads) {
        double vv[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t p = p0 + u * kThreads;
            vv[u] = I[p < hi ? p : p0];   // p0 < hi
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t p = p0 + u * kThreads;
            if (p >= hi) break;
            const double v = vv[u];
            const int64_t iy = row_of(p, inv_nx);
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
    }
    double r[kA] = {srho, fr, fl, se, ne, mx};
    block_reduce(r, 1);
    if (threadIdx.x == 0)
        for (int j = 0; j < kA; ++j) part[kA * blockIdx.x + j] = r[j];
}

// Launch 3: the moments' totals (workgroup 0 writes out: F, X_c, Y_c, C,
// rho_bar, d_img, A_LR, I_max, <I>_img, P), then the width's partial sum of
// slice blk.
__global__ __launch_bounds__(kThreads) void diag_b_partial(ImageConst c, const double* __restrict__ I,
                                                           const double* __restrict__ fc,
                                                           const double* __restrict__ pa,
                                                           double* __restrict__ out,
                                                           double* __restrict__ part) {
    double v[kA] = {0.0, 0.0, 0.0, 0.0, 0.0, -INFINITY};
    for (int b = threadIdx.x; b < kReduceBlocks; b += kThreads) {
        for (int j = 0; j < 5; ++j) v[j] += pa[kA * b + j];
        v[5] = fmax(v[5], pa[kA * b + 5]);
    }
    block_reduce(v, 1);
    const double srho = v[0], fr = v[1], fl = v[2], se = v[3], ne = v[4], mx = v[5];
    const double F = fc[0], xc = fc[1], yc = fc[2];
    const double rho_bar = srho * c.dx * c.dy / F;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
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
    const int64_t per = (c.n_pix + kReduceBlocks - 1) / kReduceBlocks;
    const double inv_nx = 1.0 / static_cast<double>(c.nx);
    const int64_t lo = per * blockIdx.x;
    const int64_t hi = lo + per < c.n_pix ? lo + per : c.n_pix;
    double s = 0.0;
    for (int64_t p0 = lo + threadIdx.x; p0 < hi; p0 += kPer * kThreads) {
        double vv[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t p = p0 + u * kThreads;
            vv[u] = I[p < hi ? p : p0];   // p0 < hi
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t p = p0 + u * kThreads;
            if (p >= hi) break;
            const int64_t iy = row_of(p, inv_nx);
            const int64_t ix = p - iy * c.nx;
            const double X = centre(c.x0, c.dx, ix), Y = centre(c.y0, c.dy, iy);
            const double d = sqrt((X - xc) * (X - xc) + (Y - yc) * (Y - yc)) - rho_bar;
            s += d * d * vv[u];
        }
    }
    double t[1] = {s};
    block_reduce(t);
    if (threadIdx.x == 0) part[blockIdx.x] = t[0];
}

// Launch 4, one workgroup: the width (out[6], out[7]), then the first bin of
// largest mean (empty bins skipped): out[12] = its centre, out[13] = twice
// that.
__global__ __launch_bounds__(kThreads) void diag_last(ImageConst c, const double* __restrict__ pb,
                                                      const double* __restrict__ profile,
                                                      int32_t n_bins, double bw,
                                                      double* __restrict__ out) {
    double s = 0.0;
    for (int b = threadIdx.x; b < kReduceBlocks; b += kThreads) s += pb[b];
    double t[1] = {s};
    block_reduce(t);
    if (threadIdx.x == 0) {
        const double w = sqrt(t[0] * c.dx * c.dy / out[0]);
        out[6] = w;
        out[7] = w / out[5];
    }
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
    hipLaunchKernelGGL(diag_first, dim3(static_cast<unsigned>(kReduceBlocks + n_bins)),
                       dim3(kThreads), 0, stream, c, intensity, bw, p3, prof);
    hipLaunchKernelGGL(diag_a_partial, dim3(kReduceBlocks), dim3(kThreads), 0, stream, c,
                       intensity, p3, fc, pa);
    hipLaunchKernelGGL(diag_b_partial, dim3(kReduceBlocks), dim3(kThreads), 0, stream, c,
                       intensity, fc, pa, out, pb);
    hipLaunchKernelGGL(diag_last, dim3(1), dim3(kThreads), 0, stream, c, pb, prof, n_bins, bw,
                       out);
    return hipGetLastError();
}

}  // namespace rt
