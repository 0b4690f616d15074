// rt_adjoint.hip -- gfx950 kernels of the image gradient: reverse mode
// through the computed discrete map of every ray (the per-ray pieces are in
// rt_vjp.h).  Three persistent passes, each lane owning one ray at a time:
//
//  1. count:   trace every pixel whose loss cotangent is non-zero and count
//              the accepted steps up to and including the last one whose
//              crossing emits (nothing after it reaches the intensity);
//  2. tape:    re-trace the pixels with a non-zero count, in the order the
//              host gives (longest first), writing each accepted step's
//              start state, size and crossing index to the ray's tape;
//  3. reverse: walk each tape backwards with reverse_step, then chain the
//              adjoint of the initial state through the screen map and write
//              the pixel's gradient along the four image parameters.
//
// Pass 2 reproduces pass 1's rays bit for bit (same code, same inputs), so
// the tape has exactly the counted length.  The reverse pass recomputes the
// stage derivatives of a step from its tape record instead of storing them
// (48 bytes per step, not 336).  A last pair of kernels sums the per-pixel
// gradients in a fixed order.
#include "rt_vjp.h"

namespace rt {
namespace {

using namespace ray;
using vjp::kRecDoubles;

static_assert(vjp::kPrims == kVjpPrims, "parameter-adjoint count");
static_assert(kRecDoubles * 8 == kVjpRecBytes, "tape record size");

struct ListShape {
    int32_t chunk;
};

template <int METRIC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 8))) void vjp_count_kernel(
    ImageConst c, const double* __restrict__ dl_dI, int32_t* __restrict__ count,
    unsigned long long* queue, LaunchShape shape) {
    const Hot k = hot_of(c);
    const OutPtrs none{};
    Ray r;
    int32_t acc = 0, last = -1;
    bool live = false;
    bool active = false, exhausted = false;
    int64_t next = 0, end = 0;
    auto claim = [&]() { return claim_chunk(queue, shape.chunk, c.n_pix, next, end); };
    auto take = [&](int64_t ordinal) {
        const int64_t pix = tile_pixel(ordinal, c.nx, c.ny, shape.tile_w, shape.tile_h);
        start_ray<METRIC>(c, k, pix, r);
        acc = 0;
        last = -1;
        live = dl_dI[pix] != 0.0;
    };
    for (;;) {
        if (!exhausted) refill(active, exhausted, next, end, claim, take);
        if (__ballot(active) == 0ull) break;
        if (active) {
            bool done = !live;
            if (live) {
                const int32_t n0 = r.ncross;
                const int32_t st = attempt<METRIC>(k, none, c.n_pix, r);
                if (st != RAY_STEP_LIMIT && r.after_reject == 0) {
                    if (r.ncross != n0 && n0 < 3) {
                        const double Rc = n0 == 0 ? r.rc[0] : (n0 == 1 ? r.rc[1] : r.rc[2]);
                        if (vjp::emits<METRIC>(c, k, Rc, r.E, r.L)) last = acc;
                    }
                    ++acc;
                }
                done = st != 0 || r.ncross >= 3;
            }
            if (done) {
                count[r.pix] = last + 1;
                active = false;
            }
        }
    }
}

template <int METRIC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 8))) void vjp_tape_kernel(
    ImageConst c, const int32_t* __restrict__ list_pix, const int64_t* __restrict__ list_off,
    const int32_t* __restrict__ count, int64_t n_list, int64_t rec_base,
    double* __restrict__ tape, int32_t* __restrict__ taped, unsigned long long* queue,
    ListShape shape) {
    const Hot k = hot_of(c);
    const OutPtrs none{};
    Ray r;
    int64_t entry = 0, rec = 0;
    int32_t acc = 0, want = 0;
    bool active = false, exhausted = false;
    int64_t next = 0, end = 0;
    auto claim = [&]() { return claim_chunk(queue, shape.chunk, n_list, next, end); };
    auto take = [&](int64_t e) {
        entry = e;
        const int64_t pix = list_pix[e];
        start_ray<METRIC>(c, k, pix, r);
        rec = list_off[e] - rec_base;
        want = count[pix];
        acc = 0;
    };
    for (;;) {
        if (!exhausted) refill(active, exhausted, next, end, claim, take);
        if (__ballot(active) == 0ull) break;
        if (active) {
            const double x0 = r.y[1], x1 = r.y[2], x2 = r.y[4], x3 = r.y[5], h = r.h;
            const int32_t n0 = r.ncross;
            const int32_t st = attempt<METRIC>(k, none, c.n_pix, r);
            if (st != RAY_STEP_LIMIT && r.after_reject == 0) {
                double2* p = reinterpret_cast<double2*>(tape + (rec + acc) * kRecDoubles);
                const double cross = (r.ncross != n0 && n0 < 3) ? static_cast<double>(n0) : -1.0;
                p[0] = make_double2(x0, x1);
                p[1] = make_double2(x2, x3);
                p[2] = make_double2(h, cross);
                ++acc;
            }
            if (acc >= want || st != 0) {
                taped[entry] = acc;
                active = false;
            }
        }
    }
}

struct JacArg {
    double m[kVjpPrims][4];
};

template <int METRIC>
__global__ __launch_bounds__(kBlock) void vjp_reverse_kernel(
    ImageConst c, const double* __restrict__ dl_dI, const int32_t* __restrict__ list_pix,
    const int64_t* __restrict__ list_off, const int32_t* __restrict__ taped, int64_t n_list,
    int64_t rec_base, const double* __restrict__ tape, JacArg J, double* __restrict__ grad_pix,
    unsigned long long* queue, ListShape shape) {
    const Hot k = hot_of(c);
    int64_t pix = 0, rec = 0;
    int32_t step = 0;
    double E = 0.0, L = 0.0, Ib = 0.0;
    ScreenDir dir{0.0, 0.0, 0.0};
    double xb[4], Eb, Lb, pb[4], rinb;
    bool active = false, exhausted = false;
    int64_t next = 0, end = 0;
    auto claim = [&]() { return claim_chunk(queue, shape.chunk, n_list, next, end); };
    auto take = [&](int64_t e) {
        pix = list_pix[e];
        rec = list_off[e] - rec_base;
        step = taped[e] - 1;
        dir = screen_dir(c, pix);
        E = c.obs_N - c.obs_gTph_over_sq_gphph * dir.nph;
        L = c.obs_sq_gphph * dir.nph;
        Ib = dl_dI[pix];
        for (int i = 0; i < 4; ++i) {
            xb[i] = 0.0;
            pb[i] = 0.0;
        }
        Eb = Lb = rinb = 0.0;
    };
    for (;;) {
        if (!exhausted) refill(active, exhausted, next, end, claim, take);
        if (__ballot(active) == 0ull) break;
        if (active) {
            if (step >= 0) {
                const double2* p = reinterpret_cast<const double2*>(tape + (rec + step) * kRecDoubles);
                const double2 a = p[0], b = p[1], hc = p[2];
                const double x0[4] = {a.x, a.y, b.x, b.y};
                vjp::reverse_step<METRIC>(c, k, E, L, x0, hc.x, static_cast<int>(hc.y), Ib, xb, Eb,
                                          Lb, pb, rinb);
                --step;
            }
            if (step < 0) {
                // Initial state (0, R_o, theta_o, 0, sqrt(g_RR) n_R, sqrt(g_thth) n_theta),
                // E = N_o - (g_Tphi/sqrt(g_phiphi)) n_phi, l = sqrt(g_phiphi) n_phi.
                double prim[kVjpPrims];
                prim[vjp::P_CHI] = pb[0];
                prim[vjp::P_M0] = pb[1];
                prim[vjp::P_M1] = pb[2];
                prim[vjp::P_M2] = pb[3];
                prim[vjp::P_RIN] = rinb;
                prim[vjp::P_OBS_N] = Eb;
                prim[vjp::P_OBS_TPH] = -Eb * dir.nph;
                prim[vjp::P_OBS_PH] = Lb * dir.nph;
                prim[vjp::P_OBS_R] = xb[2] * dir.nR;
                prim[vjp::P_OBS_TH] = xb[3] * dir.nth;
                prim[vjp::P_INCL] = xb[1];
                for (int j = 0; j < 4; ++j) {
                    double g = 0.0;
                    for (int m = 0; m < kVjpPrims; ++m) g += prim[m] * J.m[m][j];
                    grad_pix[pix * 4 + j] = g;
                }
                active = false;
            }
        }
    }
}

__global__ void fill_zero(double* __restrict__ p, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// Gradient sum over pixels in a fixed order: block b adds the pixels
// [b n/B, (b+1) n/B) with a fixed tree in LDS; one block then adds the B
// partial sums in index order.
constexpr int kGradThreads = 256;

__global__ __launch_bounds__(kGradThreads) void grad_partial(const double* __restrict__ gp,
                                                             int64_t n_pix,
                                                             double* __restrict__ part) {
    __shared__ double sh[4][kGradThreads];
    const int64_t per = (n_pix + gridDim.x - 1) / gridDim.x;
    const int64_t lo = per * blockIdx.x;
    const int64_t hi = lo + per < n_pix ? lo + per : n_pix;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t p = lo + threadIdx.x; p < hi; p += kGradThreads)
        for (int j = 0; j < 4; ++j) acc[j] += gp[p * 4 + j];
    for (int j = 0; j < 4; ++j) sh[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int w = kGradThreads / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w)
            for (int j = 0; j < 4; ++j) sh[j][threadIdx.x] += sh[j][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void grad_final(const double* __restrict__ part, int32_t nblocks,
                           double* __restrict__ grad) {
    const int j = threadIdx.x;
    if (j >= 4) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[b * 4 + j];
    grad[j] = s;
}

template <class Kern>
int occupancy(Kern kern) {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, kBlock, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace

hipError_t launch_vjp_count(const ImageConst& c, const double* dl_dI, int32_t* count,
                            unsigned long long* queue, const LaunchShape& shape, int32_t grid,
                            hipStream_t stream) {
    if (c.metric == KERR)
        hipLaunchKernelGGL(vjp_count_kernel<KERR>, dim3(grid), dim3(kBlock), 0, stream, c, dl_dI,
                           count, queue, shape);
    else if (c.metric == EINASTO)
        hipLaunchKernelGGL(vjp_count_kernel<EINASTO>, dim3(grid), dim3(kBlock), 0, stream, c,
                           dl_dI, count, queue, shape);
    else
        hipLaunchKernelGGL(vjp_count_kernel<CNFW>, dim3(grid), dim3(kBlock), 0, stream, c, dl_dI,
                           count, queue, shape);
    return hipGetLastError();
}

hipError_t launch_vjp_tape(const ImageConst& c, const int32_t* list_pix, const int64_t* list_off,
                           const int32_t* count, int64_t n_list, int64_t rec_base, double* tape,
                           int32_t* taped, unsigned long long* queue, int32_t chunk,
                           int32_t grid, hipStream_t stream) {
    const ListShape sh{chunk};
    if (c.metric == KERR)
        hipLaunchKernelGGL(vjp_tape_kernel<KERR>, dim3(grid), dim3(kBlock), 0, stream, c,
                           list_pix, list_off, count, n_list, rec_base, tape, taped, queue, sh);
    else if (c.metric == EINASTO)
        hipLaunchKernelGGL(vjp_tape_kernel<EINASTO>, dim3(grid), dim3(kBlock), 0, stream, c,
                           list_pix, list_off, count, n_list, rec_base, tape, taped, queue, sh);
    else
        hipLaunchKernelGGL(vjp_tape_kernel<CNFW>, dim3(grid), dim3(kBlock), 0, stream, c,
                           list_pix, list_off, count, n_list, rec_base, tape, taped, queue, sh);
    return hipGetLastError();
}

hipError_t launch_vjp_reverse(const ImageConst& c, const double* dl_dI, const int32_t* list_pix,
                              const int64_t* list_off, const int32_t* taped, int64_t n_list,
                              int64_t rec_base, const double* tape,
                              const double (&jac)[kVjpPrims][4], double* grad_pix,
                              unsigned long long* queue, int32_t chunk, int32_t grid,
                              hipStream_t stream) {
    JacArg J;
    for (int m = 0; m < kVjpPrims; ++m)
        for (int j = 0; j < 4; ++j) J.m[m][j] = jac[m][j];
    const ListShape sh{chunk};
    if (c.metric == KERR)
        hipLaunchKernelGGL(vjp_reverse_kernel<KERR>, dim3(grid), dim3(kBlock), 0, stream, c,
                           dl_dI, list_pix, list_off, taped, n_list, rec_base, tape, J, grad_pix,
                           queue, sh);
    else if (c.metric == EINASTO)
        hipLaunchKernelGGL(vjp_reverse_kernel<EINASTO>, dim3(grid), dim3(kBlock), 0, stream, c,
                           dl_dI, list_pix, list_off, taped, n_list, rec_base, tape, J, grad_pix,
                           queue, sh);
    else
        hipLaunchKernelGGL(vjp_reverse_kernel<CNFW>, dim3(grid), dim3(kBlock), 0, stream, c,
                           dl_dI, list_pix, list_off, taped, n_list, rec_base, tape, J, grad_pix,
                           queue, sh);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double* p, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_zero, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                       stream, p, n);
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const double* grad_pix, int64_t n_pix, double* partials,
                              double* grad, hipStream_t stream) {
    hipLaunchKernelGGL(grad_partial, dim3(kGradBlocks), dim3(kGradThreads), 0, stream, grad_pix,
                       n_pix, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(grad_final, dim3(1), dim3(64), 0, stream, partials, kGradBlocks, grad);
    return hipGetLastError();
}

int vjp_blocks_per_cu(int metric, int pass) {
    if (pass == 0) {
        if (metric == KERR) return occupancy(vjp_count_kernel<KERR>);
        if (metric == EINASTO) return occupancy(vjp_count_kernel<EINASTO>);
        return occupancy(vjp_count_kernel<CNFW>);
    }
    if (pass == 1) {
        if (metric == KERR) return occupancy(vjp_tape_kernel<KERR>);
        if (metric == EINASTO) return occupancy(vjp_tape_kernel<EINASTO>);
        return occupancy(vjp_tape_kernel<CNFW>);
    }
    if (metric == KERR) return occupancy(vjp_reverse_kernel<KERR>);
    if (metric == EINASTO) return occupancy(vjp_reverse_kernel<EINASTO>);
    return occupancy(vjp_reverse_kernel<CNFW>);
}

}  // namespace rt
