// rt_visibility.hip -- normalised visibility amplitudes of traced images
// (Sec. 6.4): V(u,v) = sum over the pixel centres of I(X,Y) exp(-2 pi i (u X
// + v Y)) dX dY and amp(u,v) = |V(u,v)| / |V(0,0)|, the midpoint rule, at K
// arbitrary (u, v) points per image; many images in one launch.
//
// The phase factorises over the screen axes: with D_k(x) = sum_y I[y][x]
// exp(-2 pi i v_k Y_y), V_k = dX dY sum_x exp(-2 pi i u_k X_x) D_k(x).  The
// contraction over y (2 K nx ny multiply-adds) is the work; it is done on the
// binary64 vector ALU with the phases generated in registers, never stored:
//   * one wavefront per work item = (image, 64 consecutive points, a block of
//     kVisCols = 16 consecutive columns); lane j owns point k = 64 g + j;
//   * the 16 pixels of a row in the block are the same for every lane: they
//     are read with two 64-byte scalar loads (wave-uniform address, the
//     scalar cache) and enter the multiply-adds as scalar operands;
//   * each lane advances its row phase exp(-2 pi i v Y) from one row to the
//     next by one complex multiplication with exp(-2 pi i v dY) (four
//     operations shared by the 16 columns), re-seeded from an exact sine and
//     cosine every kReseed rows, so the recurrence error stays ~1e-14;
//   * the column phases exp(-2 pi i u X) of the block's columns likewise.
// Each work item writes one partial sum per point; a second kernel adds a
// point's partials over the column blocks in index order, scales by dX dY and
// divides by the flux |V(0,0)| from a fixed-order reduction of the image.
// Deterministic run to run; no matrix cores (VALU only).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "rt_kernels.h"
#include "rt_math.h"

namespace rt {
namespace {

constexpr double kTwoPi = 6.283185307179586;
constexpr int kVisThreads = 256;            // four work items (wavefronts) per block
constexpr int kReseed = 64;                 // columns between exact column phases

// Image values are read through the constant address space: wave-uniform
// loads from it are scalar loads (the image is not written while the kernel
// runs).  A work item's kVisCols consecutive pixels of a row are 16 doubles
// = two 64-byte scalar loads.
typedef const __attribute__((address_space(4))) double* ConstPix;
static_assert(kVisCols == 16, "the row loads below move 16 doubles");

struct Row16 {
    double v[16];
};

// Waits for every scalar load in flight (s_waitcnt lgkmcnt(0), the other
// counters left alone).
__device__ __forceinline__ void wait_scalar_loads() { __builtin_amdgcn_s_waitcnt(0xc07f); }

// One row's contribution: D(c) += (c_ + i s_) a[c].
__device__ __forceinline__ void add_row(const Row16& a, double c_, double s_,
                                        double* __restrict__ are, double* __restrict__ aim) {
#pragma unroll
    for (int j = 0; j < kVisCols; ++j) {
        are[j] = fma(c_, a.v[j], are[j]);
        aim[j] = fma(s_, a.v[j], aim[j]);
    }
}

// D(c) += exp(i t Y_y) I[y][c] over all rows y for the 16 full columns at p
// (row stride nx): each row's 16 pixels are two 64-byte scalar loads, issued
// one row ahead of their use (rows taken in pairs, so that the wait before a
// row's multiply-adds covers only loads issued a row earlier; the loads ahead
// are clamped to the last row).
__device__ __forceinline__ void accumulate_rows_full(ConstPix p, int32_t nx, int32_t ny, double y0,
                                                     double dy, double t, double* __restrict__ are,
                                                     double* __restrict__ aim) {
    double ws, wc;
    dm::sincos(t * dy, &ws, &wc);
    auto row = [&](int32_t y) {
        const int32_t yy = y < ny ? y : ny - 1;
        const ConstPix q = p + static_cast<int64_t>(yy) * nx;
        Row16 a;
#pragma unroll
        for (int j = 0; j < kVisCols; ++j) a.v[j] = q[j];
        return a;
    };
    double s = 0.0, c = 1.0;
    Row16 A = row(0), B;
    for (int32_t y = 0; y < ny; y += 2) {
        if ((y & (kReseed - 1)) == 0)   // exact phase every kReseed rows
            dm::sincos(t * (y0 + (static_cast<double>(y) + 0.5) * dy), &s, &c);
        wait_scalar_loads();
        B = row(y + 1);
        __builtin_amdgcn_sched_barrier(0);   // the loads stay ahead of the multiply-adds
        add_row(A, c, s, are, aim);
        double cn = c * wc - s * ws;
        s = s * wc + c * ws;
        c = cn;
        // the odd row past the end of an odd-height screen enters with weight 0
        const double wB = y + 1 < ny ? 1.0 : 0.0;
        wait_scalar_loads();
        A = row(y + 2);
        __builtin_amdgcn_sched_barrier(0);
        add_row(B, c * wB, s * wB, are, aim);
        cn = c * wc - s * ws;
        s = s * wc + c * ws;
        c = cn;
    }
}

// As accumulate_rows_full for the screen's last column block, narrower than
// 16 columns: only its first ncols pixels of a row are read.
__device__ __forceinline__ void accumulate_rows_tail(ConstPix p, int32_t nx, int32_t ny,
                                                     int32_t ncols, double y0, double dy, double t,
                                                     double* __restrict__ are,
                                                     double* __restrict__ aim) {
    double ws, wc;
    dm::sincos(t * dy, &ws, &wc);
    for (int32_t yb = 0; yb < ny; yb += kReseed) {
        const double Y = y0 + (static_cast<double>(yb) + 0.5) * dy;
        double s, c;
        dm::sincos(t * Y, &s, &c);
        const int32_t ye = yb + kReseed < ny ? yb + kReseed : ny;
        for (int32_t y = yb; y < ye; ++y) {
            Row16 a;
#pragma unroll
            for (int j = 0; j < kVisCols; ++j) a.v[j] = j < ncols ? p[j] : 0.0;
            add_row(a, c, s, are, aim);
            const double cn = c * wc - s * ws;
            s = s * wc + c * ws;
            c = cn;
            p += nx;
        }
    }
}

// Partial sums of V over one work item: the kVisCols columns [c0, c0 + 16)
// of the image, all rows, for the 64 points of the item's group (one per
// lane).  With D_k(c) = sum_y exp(-2 pi i v_k Y_y) I[y][c], each lane forms
// D_k over the rows (two multiply-adds per pixel with the row's phase), then
// the partial V_k = sum_c exp(-2 pi i u_k X_c) D_k(c).
__global__ __launch_bounds__(kVisThreads) void vis_partial_kernel(
    const VisImage* __restrict__ tab, int32_t n_img, int32_t n_items,
    double2* __restrict__ part) {
    // work item = wavefront; made explicitly wave-uniform for the scalar path
    const int32_t w = __builtin_amdgcn_readfirstlane(
        static_cast<int32_t>(blockIdx.x) * (kVisThreads / 64) + static_cast<int32_t>(threadIdx.x >> 6));
    if (w >= n_items) return;
    int32_t lo = 0, hi = n_img - 1;   // the image whose items hold w
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (tab[mid].item0 <= w) lo = mid; else hi = mid - 1;
    }
    const VisImage& m = tab[lo];
    const int32_t local = w - m.item0;
    const int32_t cb = local / m.nkg, kg = local - cb * m.nkg;
    const int32_t k = kg * 64 + static_cast<int32_t>(__lane_id());
    const bool valid = k < m.K;
    const double u = valid ? m.uv[2 * k] : 0.0;
    const double v = valid ? m.uv[2 * k + 1] : 0.0;
    const int32_t nx = m.nx;
    const int32_t c0 = cb * kVisCols;
    const int32_t ncols = nx - c0 < kVisCols ? nx - c0 : kVisCols;
    double are[kVisCols], aim[kVisCols];
#pragma unroll
    for (int c = 0; c < kVisCols; ++c) are[c] = aim[c] = 0.0;
    // rows: exp(i t Y) with t = -2 pi v
    const ConstPix p = (ConstPix)(m.I + c0);
    if (ncols == kVisCols)
        accumulate_rows_full(p, nx, m.ny, m.y0, m.dy, -kTwoPi * v, are, aim);
    else
        accumulate_rows_tail(p, nx, m.ny, ncols, m.y0, m.dy, -kTwoPi * v, are, aim);
    // columns: exp(i t' X) with t' = -2 pi u, stepped by exp(i t' dX)
    const double tx = -kTwoPi * u;
    double vs, vc, xs, xc;
    dm::sincos(tx * m.dx, &vs, &vc);
    dm::sincos(tx * (m.x0 + (static_cast<double>(c0) + 0.5) * m.dx), &xs, &xc);
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int j = 0; j < kVisCols; ++j) {
        if (j < ncols) {
            re += xc * are[j] - xs * aim[j];
            im += xc * aim[j] + xs * are[j];
        }
        const double cn = xc * vc - xs * vs;
        xs = xs * vc + xc * vs;
        xc = cn;
    }
    if (valid) part[m.part0 + static_cast<int64_t>(cb) * m.K + k] = make_double2(re, im);
}

// Flux partials: block b of image i sums the contiguous slice b of its pixels
// (a fixed order: thread-strided, then a tree) into fpart[i kFluxBlocks + b].
__global__ __launch_bounds__(kVisThreads) void vis_flux_kernel(const VisImage* __restrict__ tab,
                                                               double* __restrict__ fpart) {
    __shared__ double sh[kVisThreads];
    const VisImage& m = tab[blockIdx.y];
    const int64_t n = static_cast<int64_t>(m.nx) * m.ny;
    const int64_t per = (n + kVisFluxBlocks - 1) / kVisFluxBlocks;
    const int64_t lo = per * blockIdx.x;
    const int64_t hi = lo + per < n ? lo + per : n;
    double s = 0.0;
    for (int64_t p = lo + threadIdx.x; p < hi; p += kVisThreads) s += m.I[p];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kVisThreads / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) fpart[blockIdx.y * kVisFluxBlocks + blockIdx.x] = sh[0];
}

// V_k = dX dY sum over column blocks (index order), amp_k = |V_k| / |F|.
__global__ __launch_bounds__(kVisThreads) void vis_finish_kernel(const VisImage* __restrict__ tab,
                                                                 const double2* __restrict__ part,
                                                                 const double* __restrict__ fpart) {
    const VisImage& m = tab[blockIdx.y];
    const int32_t k = static_cast<int32_t>(blockIdx.x) * kVisThreads + threadIdx.x;
    if (k >= m.K) return;
    double f = 0.0;
    for (int b = 0; b < kVisFluxBlocks; ++b) f += fpart[blockIdx.y * kVisFluxBlocks + b];
    const double dxdy = m.dx * m.dy;
    f *= dxdy;
    double re = 0.0, im = 0.0;
    for (int32_t cb = 0; cb < m.ncb; ++cb) {
        const double2 p = part[m.part0 + static_cast<int64_t>(cb) * m.K + k];
        re += p.x;
        im += p.y;
    }
    re *= dxdy;
    im *= dxdy;
    if (m.vis) {
        m.vis[2 * k] = re;
        m.vis[2 * k + 1] = im;
    }
    if (m.amp) m.amp[k] = sqrt(re * re + im * im) / fabs(f);
}

// Points on rings: uv[j n_angles + a] = q_j (cos phi_a, sin phi_a),
// phi_a = 2 pi a / n_angles.
__global__ void ring_points_kernel(const double* __restrict__ q, int32_t n_q, int32_t n_angles,
                                   double* __restrict__ uv) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= static_cast<int64_t>(n_q) * n_angles) return;
    const int32_t j = static_cast<int32_t>(i / n_angles);
    const int32_t a = static_cast<int32_t>(i - static_cast<int64_t>(j) * n_angles);
    double s, c;
    dm::sincos(kTwoPi * static_cast<double>(a) / static_cast<double>(n_angles), &s, &c);
    uv[2 * i] = q[j] * c;
    uv[2 * i + 1] = q[j] * s;
}

// avg[j] = mean over the ring's n_angles amplitudes (index order); cut[j] =
// the amplitude at phi = 0, i.e. at (u, v) = (q_j, 0).
__global__ void ring_average_kernel(const double* __restrict__ amp, int32_t n_q, int32_t n_angles,
                                    double* __restrict__ avg, double* __restrict__ cut) {
    const int32_t j = static_cast<int32_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= n_q) return;
    const double* a = amp + static_cast<int64_t>(j) * n_angles;
    double s = 0.0;
    for (int32_t i = 0; i < n_angles; ++i) s += a[i];
    if (avg) avg[j] = s / static_cast<double>(n_angles);
    if (cut) cut[j] = a[0];
}

}  // namespace

void vis_layout(VisImage* tab, int32_t n_img, int32_t* n_items, int64_t* n_part) {
    int64_t items = 0, parts = 0;
    for (int32_t i = 0; i < n_img; ++i) {
        VisImage& m = tab[i];
        m.nkg = (m.K + 63) / 64;
        m.ncb = (m.nx + kVisCols - 1) / kVisCols;
        m.item0 = static_cast<int32_t>(items);
        m.part0 = parts;
        items += static_cast<int64_t>(m.nkg) * m.ncb;
        parts += static_cast<int64_t>(m.ncb) * m.K;
    }
    *n_items = static_cast<int32_t>(items);
    *n_part = parts;
}

hipError_t launch_visibility(const VisImage* d_tab, int32_t n_img, int32_t n_items, int32_t max_k,
                             double2* part, double* fpart, hipStream_t stream) {
    hipLaunchKernelGGL(vis_flux_kernel, dim3(kVisFluxBlocks, static_cast<unsigned>(n_img)),
                       dim3(kVisThreads), 0, stream, d_tab, fpart);
    const int32_t per_block = kVisThreads / 64;
    hipLaunchKernelGGL(vis_partial_kernel,
                       dim3(static_cast<unsigned>((n_items + per_block - 1) / per_block)),
                       dim3(kVisThreads), 0, stream, d_tab, n_img, n_items, part);
    hipLaunchKernelGGL(vis_finish_kernel,
                       dim3(static_cast<unsigned>((max_k + kVisThreads - 1) / kVisThreads),
                            static_cast<unsigned>(n_img)),
                       dim3(kVisThreads), 0, stream, d_tab, part, fpart);
    return hipGetLastError();
}

hipError_t launch_ring_points(const double* q, int32_t n_q, int32_t n_angles, double* uv,
                              hipStream_t stream) {
    const int64_t n = static_cast<int64_t>(n_q) * n_angles;
    hipLaunchKernelGGL(ring_points_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256),
                       0, stream, q, n_q, n_angles, uv);
    return hipGetLastError();
}

hipError_t launch_ring_average(const double* amp, int32_t n_q, int32_t n_angles, double* avg,
                               double* cut, hipStream_t stream) {
    hipLaunchKernelGGL(ring_average_kernel, dim3(static_cast<unsigned>((n_q + 255) / 256)),
                       dim3(256), 0, stream, amp, n_q, n_angles, avg, cut);
    return hipGetLastError();
}

}  // namespace rt
